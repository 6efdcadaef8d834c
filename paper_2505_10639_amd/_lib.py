"""ctypes binding of libmomfbd.so: the C-ABI functions under the same names.

Argument marshalling only.  Device arrays are torch tensors (their data
pointers are passed); host arrays for plan creation are numpy arrays.  The
stream defaults to torch's current stream on the tensors' device.  There is
no fallback: if the library is not built, every call raises.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MOMFBD_LIBRARY names another build of the same sources (the tests' host
# sanitizer build); by default the in-tree library.
LIB_PATH = os.environ.get("MOMFBD_LIBRARY") or os.path.join(_HERE, "libmomfbd.so")

MOMFBD_OK = 0
MOMFBD_EINVAL = -1
MOMFBD_EUNSUPPORTED = -2
MOMFBD_EWORKSPACE = -3
MOMFBD_EDEVICE = -4
MOMFBD_ESCRATCH = -5


class MomfbdError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {momfbd_status_string(status)} (status {status})")


class momfbd_lbfgs_params(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("max_evals", ctypes.c_int), ("c1", ctypes.c_double),
                ("c2", ctypes.c_double), ("ftol", ctypes.c_double)]


MOMFBD_FILTER_NONE, MOMFBD_FILTER_TOPHAT, MOMFBD_FILTER_SCHARMER = 0, 1, 2


class momfbd_filter(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("f_lo", ctypes.c_float), ("f_hi", ctypes.c_float),
                ("diff_limit", ctypes.c_float), ("noise_power", ctypes.c_float)]


class momfbd_tuning(ctypes.Structure):
    _fields_ = [("xcd_forward", ctypes.c_int), ("xcd_adjoint", ctypes.c_int),
                ("object_pairs_per_thread", ctypes.c_int), ("grad_waves", ctypes.c_int),
                ("grad_splits", ctypes.c_int), ("grad_row_tiles", ctypes.c_int),
                ("phase_col_tiles", ctypes.c_int), ("phase_waves", ctypes.c_int),
                ("object_fused", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class momfbd_desc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("P", ctypes.c_int), ("C", ctypes.c_int),
                ("K", ctypes.c_int), ("J", ctypes.c_int), ("M", ctypes.c_int),
                ("channel_object", ctypes.POINTER(ctypes.c_int))]


class momfbd_field(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("alpha", ctypes.c_void_p), ("D", ctypes.c_void_p),
                ("gamma", ctypes.c_void_p), ("gamma_scalar", ctypes.c_float),
                ("weights", ctypes.c_void_p), ("ws", ctypes.c_void_p),
                ("ws_bytes", ctypes.c_size_t), ("state", ctypes.c_void_p),
                ("state_bytes", ctypes.c_size_t), ("loss", ctypes.c_void_p),
                ("grad", ctypes.c_void_p), ("loss_accepted", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("alpha_accepted", ctypes.c_void_p)]


_lib = None
_vp = ctypes.c_void_p
_STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported configuration",
           -3: "workspace missing, misaligned or too small", -4: "HIP device error",
           -5: "problem needs more scratch than the allocation-free entry point's fixed buffer"}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MomfbdError(MOMFBD_EDEVICE, f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        i, f, d = ctypes.c_int, ctypes.c_float, ctypes.c_double
        L.momfbd_plan_create.argtypes = [ctypes.POINTER(momfbd_desc), _vp, _vp, _vp,
                                         ctypes.POINTER(_vp)]
        L.momfbd_plan_destroy.argtypes = [_vp]
        L.momfbd_workspace_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
        z = ctypes.c_size_t
        L.momfbd_prepare_data.argtypes = [_vp, _vp, i, i, i, _vp, _vp, _vp, z, _vp]
        L.momfbd_forward.argtypes = [_vp, _vp, _vp, _vp, _vp, z, _vp]
        L.momfbd_loss_grad.argtypes = [_vp, _vp, _vp, _vp, f, _vp, _vp, _vp, _vp, z, _vp]
        L.momfbd_loss_grad_noalloc.argtypes = [_vp, _vp, _vp, _vp, f, _vp, _vp, _vp, _vp]
        L.momfbd_object_estimate.argtypes = [_vp, _vp, _vp, _vp, f, _vp, _vp, _vp, z, _vp]
        L.momfbd_status_string.argtypes = [i]
        L.momfbd_status_string.restype = ctypes.c_char_p
        L.momfbd_plan_dims.argtypes = [_vp] + [ctypes.POINTER(i)] * 6
        L.momfbd_object_filtered.argtypes = [_vp, _vp, _vp, _vp, f, _vp,
                                             ctypes.POINTER(momfbd_filter), _vp, _vp, _vp, z,
                                             _vp]
        L.momfbd_mosaic.argtypes = [_vp, _vp, i, i, i, i, _vp, _vp]
        L.momfbd_synthesize.argtypes = [_vp] * 9 + [z, _vp]
        tp = ctypes.POINTER(momfbd_tuning)
        L.momfbd_plan_set_tuning.argtypes = [_vp, tp]
        L.momfbd_plan_get_tuning.argtypes = [_vp, tp]
        L.momfbd_plan_autotune.argtypes = [_vp, _vp, _vp, _vp, f, _vp, i, _vp, _vp, _vp, z, _vp,
                                           tp]
        L.momfbd_power_spectrum_workspace.argtypes = [i, i, ctypes.POINTER(ctypes.c_size_t)]
        L.momfbd_power_spectrum.argtypes = [i, _vp, _vp, _vp, _vp, _vp, i, _vp, z, _vp]
        L.momfbd_lbfgs_rounds.argtypes = [_vp, ctypes.POINTER(momfbd_lbfgs_params), _vp, z, _vp,
                                          _vp, _vp, f, _vp, i, _vp, _vp, _vp, _vp, z, _vp]
        L.momfbd_cnn_create.argtypes = [i, i, i, i, _vp, ctypes.POINTER(_vp)]
        L.momfbd_cnn_destroy.argtypes = [_vp]
        L.momfbd_cnn_sizes.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(ctypes.c_size_t)]
        L.momfbd_cnn_init.argtypes = [_vp] * 4 + [z, _vp]
        L.momfbd_cnn_load.argtypes = [_vp] * 3 + [z, _vp]
        L.momfbd_cnn_forward.argtypes = [_vp, _vp, _vp, i, i, _vp, _vp, z, _vp]
        L.momfbd_cnn_loss_grad.argtypes = [_vp, _vp, _vp, i, _vp, i, _vp, _vp, _vp, z, _vp]
        L.momfbd_cnn_input.argtypes = [_vp, _vp, i, i, _vp, _vp, z, _vp]
        L.momfbd_cnn_adam.argtypes = [_vp, _vp, _vp, _vp, _vp, i, f, f, f, f, _vp, z, _vp]
        L.momfbd_smoothness_gamma.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.momfbd_profile_start.argtypes = [_vp, i]
        L.momfbd_profile_repeat.argtypes = [_vp, ctypes.c_char_p, i]
        pp = ctypes.POINTER(momfbd_lbfgs_params)
        L.momfbd_lbfgs_state_size.argtypes = [_vp, pp, ctypes.POINTER(ctypes.c_size_t)]
        L.momfbd_lbfgs_init.argtypes = [_vp, pp, _vp, z, _vp, _vp, _vp, f, _vp, _vp, _vp, z, _vp]
        L.momfbd_lbfgs_step.argtypes = [_vp, pp, _vp, z, _vp, _vp, _vp, f, _vp, _vp, _vp, _vp, z,
                                        _vp]
        L.momfbd_profile_stop.argtypes = [_vp, i, ctypes.POINTER(ctypes.c_char_p),
                                          ctypes.POINTER(d), ctypes.POINTER(i)]
        u64 = ctypes.c_ulonglong
        L.momfbd_random_normal.argtypes = [u64, u64, u64, z, _vp, _vp, _vp]
        L.momfbd_group_create.argtypes = [ctypes.POINTER(momfbd_field), i, pp,
                                          ctypes.POINTER(_vp)]
        L.momfbd_group_destroy.argtypes = [_vp]
        L.momfbd_group_loss_grad.argtypes = [_vp, _vp]
        L.momfbd_group_lbfgs_rounds.argtypes = [_vp, i, _vp]
        L.momfbd_group_set_tuning.argtypes = [_vp, tp]
        L.momfbd_group_get_tuning.argtypes = [_vp, tp]
        L.momfbd_group_autotune.argtypes = [_vp, i, _vp, tp]
        for name in ("momfbd_plan_create", "momfbd_plan_destroy", "momfbd_workspace_size",
                     "momfbd_prepare_data", "momfbd_forward", "momfbd_loss_grad",
                     "momfbd_object_estimate", "momfbd_plan_dims", "momfbd_profile_start",
                     "momfbd_profile_repeat", "momfbd_profile_stop", "momfbd_lbfgs_state_size",
                     "momfbd_lbfgs_init", "momfbd_lbfgs_step", "momfbd_smoothness_gamma",
                     "momfbd_object_filtered", "momfbd_mosaic", "momfbd_synthesize", "momfbd_cnn_create",
                     "momfbd_cnn_destroy", "momfbd_cnn_sizes", "momfbd_cnn_init",
                     "momfbd_cnn_load", "momfbd_cnn_forward", "momfbd_cnn_loss_grad",
                     "momfbd_cnn_input",
                     "momfbd_cnn_adam", "momfbd_lbfgs_rounds", "momfbd_power_spectrum_workspace",
                     "momfbd_power_spectrum", "momfbd_plan_set_tuning", "momfbd_plan_get_tuning",
                     "momfbd_plan_autotune", "momfbd_loss_grad_noalloc",
                     "momfbd_group_create", "momfbd_group_destroy", "momfbd_group_loss_grad",
                     "momfbd_group_lbfgs_rounds", "momfbd_group_set_tuning",
                     "momfbd_group_get_tuning", "momfbd_group_autotune",
                     "momfbd_random_normal"):
            getattr(L, name).restype = i
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != MOMFBD_OK:
        raise MomfbdError(status, where)


def _ptr(t):
    """Device/host pointer of a tensor or ndarray; None -> NULL."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _nbytes(t):
    """Length in bytes of a workspace or state buffer (tensor or ndarray); 0 for None."""
    if t is None:
        return 0
    if isinstance(t, np.ndarray):
        return int(t.nbytes)
    return int(t.numel() * t.element_size())


def _stream(stream, *tensors):
    if stream is not None:
        return stream
    import torch
    for t in tensors:
        if t is not None and hasattr(t, "is_cuda") and t.is_cuda:
            return torch.cuda.current_stream(t.device).cuda_stream
    return None


def momfbd_status_string(status: int) -> str:
    if _lib is None and not os.path.exists(LIB_PATH):
        return _STATUS.get(status, "unknown status")
    return lib().momfbd_status_string(status).decode()


def momfbd_plan_create(N, P, C, K, J, M, channel_object, pupil, basis, diversity=None):
    """Create a plan from host arrays; returns the opaque plan handle (int)."""
    co = (ctypes.c_int * C)(*[int(v) for v in channel_object])
    desc = momfbd_desc(N, P, C, K, J, M, co)
    pupil = np.ascontiguousarray(pupil, dtype=np.float32)
    basis = np.ascontiguousarray(basis, dtype=np.float32)
    if pupil.size != C * N * N or basis.size != C * M * N * N:
        raise MomfbdError(MOMFBD_EINVAL, "momfbd_plan_create: array sizes")
    div = None if diversity is None else np.ascontiguousarray(diversity, dtype=np.float32)
    if div is not None and div.size != C * N * N:
        raise MomfbdError(MOMFBD_EINVAL, "momfbd_plan_create: diversity size")
    out = _vp()
    _check(lib().momfbd_plan_create(ctypes.byref(desc), _ptr(pupil), _ptr(basis), _ptr(div),
                                    ctypes.byref(out)), "momfbd_plan_create")
    return out.value


def momfbd_plan_destroy(plan):
    _check(lib().momfbd_plan_destroy(plan), "momfbd_plan_destroy")


def momfbd_workspace_size(plan) -> int:
    n = ctypes.c_size_t()
    _check(lib().momfbd_workspace_size(plan, ctypes.byref(n)), "momfbd_workspace_size")
    return n.value


def momfbd_plan_dims(plan):
    v = [ctypes.c_int() for _ in range(6)]
    _check(lib().momfbd_plan_dims(plan, *[ctypes.byref(x) for x in v]), "momfbd_plan_dims")
    return tuple(x.value for x in v)


def momfbd_smoothness_gamma(plan, gamma0, lam, gamma, stream=None):
    g0 = np.ascontiguousarray(gamma0, np.float32)
    lm = np.ascontiguousarray(lam, np.float32)
    _check(lib().momfbd_smoothness_gamma(plan, _ptr(g0), _ptr(lm), _ptr(gamma),
                                         _stream(stream, gamma)), "momfbd_smoothness_gamma")


def momfbd_prepare_data(plan, frames, H, W, stride, apod, D, ws, stream=None):
    _check(lib().momfbd_prepare_data(plan, _ptr(frames), H, W, stride, _ptr(apod), _ptr(D),
                                     _ptr(ws), _nbytes(ws), _stream(stream, frames)),
           "momfbd_prepare_data")


def momfbd_forward(plan, alpha, psf, otf, ws, stream=None):
    _check(lib().momfbd_forward(plan, _ptr(alpha), _ptr(psf), _ptr(otf), _ptr(ws), _nbytes(ws),
                                _stream(stream, alpha)), "momfbd_forward")


def momfbd_loss_grad(plan, alpha, D, gamma, gamma_scalar, weights, loss, grad, ws, stream=None):
    _check(lib().momfbd_loss_grad(plan, _ptr(alpha), _ptr(D), _ptr(gamma), float(gamma_scalar),
                                  _ptr(weights), _ptr(loss), _ptr(grad), _ptr(ws), _nbytes(ws),
                                  _stream(stream, alpha)), "momfbd_loss_grad")


def momfbd_loss_grad_noalloc(plan, alpha, D, gamma, gamma_scalar, weights, loss, grad,
                             stream=None):
    _check(lib().momfbd_loss_grad_noalloc(plan, _ptr(alpha), _ptr(D), _ptr(gamma),
                                          float(gamma_scalar), _ptr(weights), _ptr(loss),
                                          _ptr(grad), _stream(stream, alpha)),
           "momfbd_loss_grad_noalloc")


def momfbd_object_estimate(plan, alpha, D, gamma, gamma_scalar, weights, obj, ws, stream=None):
    _check(lib().momfbd_object_estimate(plan, _ptr(alpha), _ptr(D), _ptr(gamma),
                                        float(gamma_scalar), _ptr(weights), _ptr(obj), _ptr(ws),
                                        _nbytes(ws), _stream(stream, alpha)),
           "momfbd_object_estimate")


def filter_spec(kind, f_lo=0.0, f_hi=0.0, diff_limit=0.0, noise_power=0.0):
    """One object's filter: kind "none", "tophat" or "scharmer"."""
    k = {"none": MOMFBD_FILTER_NONE, "tophat": MOMFBD_FILTER_TOPHAT,
         "scharmer": MOMFBD_FILTER_SCHARMER}[kind]
    return momfbd_filter(k, f_lo, f_hi, diff_limit, noise_power)


def momfbd_object_filtered(plan, alpha, D, gamma, gamma_scalar, weights, filters, obj, H, ws,
                           stream=None):
    arr = (momfbd_filter * len(filters))(*filters)
    _check(lib().momfbd_object_filtered(plan, _ptr(alpha), _ptr(D), _ptr(gamma),
                                        float(gamma_scalar), _ptr(weights), arr, _ptr(obj),
                                        _ptr(H), _ptr(ws), _nbytes(ws), _stream(stream, alpha)),
           "momfbd_object_filtered")


def momfbd_mosaic(plan, obj, ny, nx, stride, border, out, stream=None):
    _check(lib().momfbd_mosaic(plan, _ptr(obj), int(ny), int(nx), int(stride), int(border),
                               _ptr(out), _stream(stream, obj)), "momfbd_mosaic")


def momfbd_lbfgs_rounds(plan, params, state, alpha, D, gamma, gamma_scalar, weights, rounds, loss,
                        status, alpha_accepted, ws, stream=None):
    _check(lib().momfbd_lbfgs_rounds(plan, ctypes.byref(params), _ptr(state), _nbytes(state),
                                     _ptr(alpha), _ptr(D), _ptr(gamma), float(gamma_scalar),
                                     _ptr(weights), int(rounds), _ptr(loss), _ptr(status),
                                     _ptr(alpha_accepted), _ptr(ws), _nbytes(ws),
                                     _stream(stream, alpha)),
           "momfbd_lbfgs_rounds")


def momfbd_power_spectrum(image, window=None, nbins=None, stream=None):
    """(power [L][L], sector mean [nbins] FP64, counts [nbins]) of a square
    device image (torch float32)."""
    import torch
    L = int(image.shape[0])
    if image.shape != (L, L) or image.dtype != torch.float32 or not image.is_contiguous():
        raise ValueError("image must be a contiguous float32 [L][L] tensor")
    nb = L // 2 + 1 if nbins is None else int(nbins)
    n = ctypes.c_size_t()
    _check(lib().momfbd_power_spectrum_workspace(L, nb, ctypes.byref(n)),
           "momfbd_power_spectrum_workspace")
    ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=image.device)
    power = torch.empty((L, L), dtype=torch.float32, device=image.device)
    sector = torch.empty(nb, dtype=torch.float64, device=image.device)
    counts = torch.empty(nb, dtype=torch.int32, device=image.device)
    _check(lib().momfbd_power_spectrum(L, _ptr(image), _ptr(window), _ptr(power), _ptr(sector),
                                       _ptr(counts), nb, _ptr(ws), _nbytes(ws),
                                       _stream(stream, image)),
           "momfbd_power_spectrum")
    return power, sector, counts


def momfbd_plan_set_tuning(plan, xcd_forward, xcd_adjoint, object_pairs_per_thread, grad_waves,
                           grad_splits=0, grad_row_tiles=0, phase_col_tiles=0, phase_waves=0,
                           object_fused=0):
    t = momfbd_tuning(xcd_forward, xcd_adjoint, object_pairs_per_thread, grad_waves, grad_splits,
                      grad_row_tiles, phase_col_tiles, phase_waves, object_fused)
    _check(lib().momfbd_plan_set_tuning(plan, ctypes.byref(t)), "momfbd_plan_set_tuning")


def momfbd_plan_get_tuning(plan):
    t = momfbd_tuning()
    _check(lib().momfbd_plan_get_tuning(plan, ctypes.byref(t)), "momfbd_plan_get_tuning")
    return t.as_dict()


def momfbd_plan_autotune(plan, alpha, D, gamma, gamma_scalar, weights, reps, loss, grad, ws,
                         stream=None):
    t = momfbd_tuning()
    _check(lib().momfbd_plan_autotune(plan, _ptr(alpha), _ptr(D), _ptr(gamma), float(gamma_scalar),
                                      _ptr(weights), int(reps), _ptr(loss), _ptr(grad), _ptr(ws),
                                      _nbytes(ws), _stream(stream, alpha), ctypes.byref(t)),
           "momfbd_plan_autotune")
    return t.as_dict()


def momfbd_synthesize(plan, alpha, O, noise, sigma, apod, frames, D, ws, stream=None):
    _check(lib().momfbd_synthesize(plan, _ptr(alpha), _ptr(O), _ptr(noise), _ptr(sigma),
                                   _ptr(apod), _ptr(frames), _ptr(D), _ptr(ws), _nbytes(ws),
                                   _stream(stream, alpha)), "momfbd_synthesize")


def momfbd_cnn_create(N, J, M, batch_max, mode_scale):
    sc = np.ascontiguousarray(mode_scale, np.float32)
    out = _vp()
    _check(lib().momfbd_cnn_create(int(N), int(J), int(M), int(batch_max), sc.ctypes.data,
                                   ctypes.byref(out)), "momfbd_cnn_create")
    return out.value


def momfbd_cnn_destroy(net):
    _check(lib().momfbd_cnn_destroy(net), "momfbd_cnn_destroy")


def momfbd_cnn_sizes(net):
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().momfbd_cnn_sizes(net, ctypes.byref(a), ctypes.byref(b)), "momfbd_cnn_sizes")
    return a.value, b.value


def momfbd_cnn_init(net, normals, params, ws, stream=None):
    _check(lib().momfbd_cnn_init(net, _ptr(normals), _ptr(params), _ptr(ws), _nbytes(ws),
                                 _stream(stream, params)), "momfbd_cnn_init")


def momfbd_cnn_load(net, params, ws, stream=None):
    _check(lib().momfbd_cnn_load(net, _ptr(params), _ptr(ws), _nbytes(ws),
                                 _stream(stream, params)),
           "momfbd_cnn_load")


def momfbd_cnn_forward(net, params, D, B, C, alpha, ws, stream=None):
    _check(lib().momfbd_cnn_forward(net, _ptr(params), _ptr(D), int(B), int(C), _ptr(alpha),
                                    _ptr(ws), _nbytes(ws), _stream(stream, params)),
           "momfbd_cnn_forward")


def momfbd_cnn_input(net, D, B, C, x, ws, stream=None):
    _check(lib().momfbd_cnn_input(net, _ptr(D), int(B), int(C), _ptr(x), _ptr(ws), _nbytes(ws),
                                  _stream(stream, x)),
           "momfbd_cnn_input")


def momfbd_cnn_loss_grad(net, params, D, C, target, B, loss, grad, ws, stream=None):
    _check(lib().momfbd_cnn_loss_grad(net, _ptr(params), _ptr(D), int(C), _ptr(target), int(B),
                                      _ptr(loss), _ptr(grad), _ptr(ws), _nbytes(ws),
                                      _stream(stream, params)),
           "momfbd_cnn_loss_grad")


def momfbd_cnn_adam(net, params, grad, m1, m2, step, lr, beta1, beta2, eps, ws, stream=None):
    _check(lib().momfbd_cnn_adam(net, _ptr(params), _ptr(grad), _ptr(m1), _ptr(m2), int(step),
                                 float(lr), float(beta1), float(beta2), float(eps), _ptr(ws),
                                 _nbytes(ws), _stream(stream, params)), "momfbd_cnn_adam")


def momfbd_profile_start(plan, max_launches: int):
    _check(lib().momfbd_profile_start(plan, int(max_launches)), "momfbd_profile_start")


def momfbd_profile_repeat(plan, kind: str, reps: int):
    _check(lib().momfbd_profile_repeat(plan, kind.encode(), int(reps)), "momfbd_profile_repeat")


def momfbd_profile_stop(plan) -> dict:
    """{kernel name: (total ms, launches)} since momfbd_profile_start."""
    cap = 16
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int * cap)()
    n = lib().momfbd_profile_stop(plan, cap, names, ms, cnt)
    if n < 0:
        raise MomfbdError(n, "momfbd_profile_stop")
    return {names[k].decode(): (ms[k], cnt[k]) for k in range(n)}


def lbfgs_params(m=10, max_evals=20, c1=1e-4, c2=0.9, ftol=0.0):
    return momfbd_lbfgs_params(int(m), int(max_evals), float(c1), float(c2), float(ftol))


def momfbd_lbfgs_state_size(plan, params) -> int:
    n = ctypes.c_size_t()
    _check(lib().momfbd_lbfgs_state_size(plan, ctypes.byref(params), ctypes.byref(n)),
           "momfbd_lbfgs_state_size")
    return n.value


def momfbd_lbfgs_init(plan, params, state, alpha, D, gamma, gamma_scalar, weights, loss, ws,
                      stream=None):
    _check(lib().momfbd_lbfgs_init(plan, ctypes.byref(params), _ptr(state), _nbytes(state),
                                   _ptr(alpha), _ptr(D), _ptr(gamma), float(gamma_scalar),
                                   _ptr(weights), _ptr(loss), _ptr(ws), _nbytes(ws),
                                   _stream(stream, alpha)), "momfbd_lbfgs_init")


def momfbd_lbfgs_step(plan, params, state, alpha, D, gamma, gamma_scalar, weights, loss, status,
                      ws, stream=None):
    _check(lib().momfbd_lbfgs_step(plan, ctypes.byref(params), _ptr(state), _nbytes(state),
                                   _ptr(alpha), _ptr(D), _ptr(gamma), float(gamma_scalar),
                                   _ptr(weights), _ptr(loss), _ptr(status), _ptr(ws), _nbytes(ws),
                                   _stream(stream, alpha)), "momfbd_lbfgs_step")


def field_spec(plan, alpha, D, gamma, gamma_scalar, weights, ws, state=None, loss=None,
               grad=None, loss_accepted=None, status=None, alpha_accepted=None):
    """One momfbd_field (device pointers of tensors; None -> NULL)."""
    return momfbd_field(plan, _ptr(alpha), _ptr(D), _ptr(gamma), float(gamma_scalar),
                        _ptr(weights), _ptr(ws), _nbytes(ws), _ptr(state), _nbytes(state),
                        _ptr(loss), _ptr(grad), _ptr(loss_accepted), _ptr(status),
                        _ptr(alpha_accepted))


def momfbd_group_create(fields, params=None):
    arr = (momfbd_field * len(fields))(*fields)
    out = _vp()
    _check(lib().momfbd_group_create(arr, len(fields),
                                     None if params is None else ctypes.byref(params),
                                     ctypes.byref(out)), "momfbd_group_create")
    return out.value


def momfbd_group_destroy(group):
    _check(lib().momfbd_group_destroy(group), "momfbd_group_destroy")


def momfbd_group_loss_grad(group, stream):
    _check(lib().momfbd_group_loss_grad(group, stream), "momfbd_group_loss_grad")


def momfbd_group_lbfgs_rounds(group, rounds, stream):
    _check(lib().momfbd_group_lbfgs_rounds(group, int(rounds), stream),
           "momfbd_group_lbfgs_rounds")


def momfbd_group_set_tuning(group, xcd_forward, xcd_adjoint, grad_splits=0, grad_row_tiles=4):
    t = momfbd_tuning(xcd_forward, xcd_adjoint, 1, 4, grad_splits, grad_row_tiles)
    _check(lib().momfbd_group_set_tuning(group, ctypes.byref(t)), "momfbd_group_set_tuning")


def momfbd_group_get_tuning(group):
    t = momfbd_tuning()
    _check(lib().momfbd_group_get_tuning(group, ctypes.byref(t)), "momfbd_group_get_tuning")
    return t.as_dict()


def momfbd_group_autotune(group, reps, stream):
    t = momfbd_tuning()
    _check(lib().momfbd_group_autotune(group, int(reps), stream, ctypes.byref(t)),
           "momfbd_group_autotune")
    return t.as_dict()


def momfbd_random_normal(seed, stream_id, counter0, out, bits=None, stream=None):
    """Fill the float32 device tensor `out` with standard normal draws (and
    `bits`, uint32 as int32 storage, with the generator words) from the
    library's counter-based generator."""
    _check(lib().momfbd_random_normal(int(seed), int(stream_id), int(counter0), out.numel(),
                                      _ptr(out), _ptr(bits), _stream(stream, out)),
           "momfbd_random_normal")
