"""CPU-side checks of the C-ABI library: it loads, exports every declared
symbol, and rejects bad arguments before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "momfbd.h")


@pytest.fixture(scope="module")
def L():
    from paper_2505_10639_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmomfbd.so is not built: run __graft_entry__.build()")
    return _lib.lib()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(momfbd_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("momfbd_plan_create", "momfbd_plan_destroy", "momfbd_workspace_size",
                     "momfbd_prepare_data", "momfbd_forward", "momfbd_loss_grad",
                     "momfbd_object_estimate", "momfbd_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings(L):
    from paper_2505_10639_amd import momfbd_status_string
    assert momfbd_status_string(0) == "ok"
    assert momfbd_status_string(-1) == "invalid argument"
    assert momfbd_status_string(-2) == "unsupported configuration"
    assert momfbd_status_string(-3).startswith("workspace")
    assert momfbd_status_string(-4).startswith("HIP")


def _arrays(N=64, C=1, M=6, frac=0.45):
    A = np.broadcast_to(synth.pupil_mask(N, frac), (C, N, N)).astype(np.float32)
    Z = np.broadcast_to(synth.zernike_basis(N, M, frac), (C, M, N, N)).astype(np.float32)
    return np.ascontiguousarray(A), np.ascontiguousarray(Z)


def _create(L, N=64, P=2, C=1, K=1, J=3, M=6, co=None, A=None, Z=None, desc_null=False):
    from paper_2505_10639_amd._lib import momfbd_desc
    co = co if co is not None else [0] * C
    arr = (ctypes.c_int * C)(*co)
    desc = momfbd_desc(N, P, C, K, J, M, arr)
    if A is None:
        A, Z = _arrays(N, C, M)
    out = ctypes.c_void_p()
    st = L.momfbd_plan_create(None if desc_null else ctypes.byref(desc),
                              A.ctypes.data if A is not None else None,
                              Z.ctypes.data if Z is not None else None, None, ctypes.byref(out))
    return st, out


def test_plan_create_rejects_bad_arguments_without_a_device(L):
    assert _create(L, desc_null=True)[0] == -1
    assert _create(L, P=0)[0] == -1
    assert _create(L, J=0)[0] == -1
    assert _create(L, C=2, K=1, co=[0, 1])[0] == -1           # object id out of range
    assert _create(L, C=2, K=2, co=[0, 0])[0] == -1           # object 1 owns no channel
    A, Z = _arrays(80, 1, 6)
    assert _create(L, N=80, A=A, Z=Z)[0] == -2                # patch size unsupported
    assert _create(L, M=300, A=_arrays(64, 1, 300)[0], Z=_arrays(64, 1, 300)[1])[0] == -2
    assert _create(L, J=100, M=100, A=_arrays(64, 1, 100)[0], Z=_arrays(64, 1, 100)[1])[0] == -2
    A, Z = _arrays(64, 33, 6)
    assert _create(L, C=33, K=1, A=A, Z=Z)[0] == -2           # more channels than the plan holds
    A, Z = _arrays(64, 1, 6, frac=0.6)                        # pupil wider than N/2
    assert _create(L, A=A, Z=Z)[0] == -2
    A0 = np.zeros((1, 64, 64), np.float32)
    assert _create(L, A=A0, Z=_arrays(64, 1, 6)[1])[0] == -1  # empty pupil
    An = _arrays(64, 1, 6)[0].copy()
    An[0, 30, 30] = np.nan
    assert _create(L, A=An, Z=_arrays(64, 1, 6)[1])[0] == -1  # NaN in the pupil


def test_calls_reject_null_plan_and_workspace(L):
    assert L.momfbd_loss_grad(None, None, None, None, 1e-3, None, None, None, None, 0,
                              None) == -1
    assert L.momfbd_forward(None, None, None, None, None, 0, None) == -1
    assert L.momfbd_object_estimate(None, None, None, None, 1e-3, None, None, None, 0,
                                    None) == -1
    assert L.momfbd_prepare_data(None, None, 64, 64, 32, None, None, None, 0, None) == -1
    assert L.momfbd_plan_destroy(None) == 0
    n = ctypes.c_size_t()
    assert L.momfbd_workspace_size(None, ctypes.byref(n)) == -1
    assert L.momfbd_smoothness_gamma(None, None, None, None, None) == -1
    assert L.momfbd_mosaic(None, None, 1, 1, 1, 0, None, None) == -1
    assert L.momfbd_object_filtered(None, None, None, None, 1e-3, None, None, None, None, None,
                                    0, None) == -1
    n = ctypes.c_size_t()
    assert L.momfbd_power_spectrum_workspace(100, 10, ctypes.byref(n)) == -1   # not a power of two
    assert L.momfbd_power_spectrum_workspace(64, 65, ctypes.byref(n)) == -1    # nbins > L
    assert L.momfbd_power_spectrum_workspace(64, 33, ctypes.byref(n)) == 0 and n.value > 64 * 64 * 8
    assert L.momfbd_plan_set_tuning(None, None) == -1
    assert L.momfbd_plan_get_tuning(None, None) == -1
    assert L.momfbd_plan_autotune(None, None, None, None, 1e-3, None, 1, None, None, None, 0,
                                  None, None) == -1
    assert L.momfbd_profile_repeat(None, b"adjoint", 4) == -1


def _aligned(nbytes, fill):
    """A 256-byte aligned host buffer (a stand-in pointer: the calls below
    fail their argument checks before anything reads or writes it)."""
    raw = np.full(nbytes + 256, fill, np.uint8)
    off = (-raw.ctypes.data) % 256
    return raw, raw[off:off + nbytes]


def test_short_workspace_is_refused_before_any_work(L):
    """A workspace one byte short of the size query (or misaligned, or
    missing) returns EWORKSPACE, and the outputs are not written.  The power
    spectrum needs no plan, so the check runs here without a device."""
    Lsz, nb = 64, 33
    n = ctypes.c_size_t()
    assert L.momfbd_power_spectrum_workspace(Lsz, nb, ctypes.byref(n)) == 0
    _, img = _aligned(Lsz * Lsz * 4, 0)
    _, power = _aligned(Lsz * Lsz * 4, 0xA5)
    _, sector = _aligned(nb * 8, 0x5A)
    _, counts = _aligned(nb * 4, 0x3C)
    raw_ws, ws = _aligned(n.value, 0x77)
    ptr = lambda a: a.ctypes.data
    st = L.momfbd_power_spectrum(Lsz, ptr(img), None, ptr(power), ptr(sector), ptr(counts), nb,
                                 ptr(ws), n.value - 1, None)
    assert st == -3
    st = L.momfbd_power_spectrum(Lsz, ptr(img), None, ptr(power), ptr(sector), ptr(counts), nb,
                                 None, n.value, None)
    assert st == -3
    st = L.momfbd_power_spectrum(Lsz, ptr(img), None, ptr(power), ptr(sector), ptr(counts), nb,
                                 ptr(ws) + 8, n.value, None)
    assert st == -3
    assert np.all(power == 0xA5) and np.all(sector == 0x5A) and np.all(counts == 0x3C)
    assert np.all(raw_ws == 0x77)


def _declared_params():
    """{function: number of parameters} of every declaration in the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"\b(?:int|const char\*)\s+(momfbd_\w+)\s*\(([^)]*)\)\s*;", text):
        args = [a for a in m.group(2).split(",") if a.strip() and a.strip() != "void"]
        out[m.group(1)] = len(args)
    return out


def test_binding_signatures_match_the_header(L):
    """Every function the binding declares takes as many arguments as the
    header gives it (a missing size_t would shift every later argument)."""
    decl = _declared_params()
    checked = 0
    for name, nparams in decl.items():
        fn = getattr(L, name)
        if fn.argtypes is None:
            continue
        assert len(fn.argtypes) == nparams, (name, len(fn.argtypes), nparams)
        checked += 1
    assert checked >= 30


def test_binding_structs_match_the_header():
    """The ctypes structures of the binding list the header's fields in the
    same order (the library reads them by position)."""
    from paper_2505_10639_amd import _lib
    text = open(HEADER).read()
    for cname in ("momfbd_tuning", "momfbd_desc", "momfbd_field"):
        body = re.search(r"typedef struct\s*\{((?:(?!typedef struct).)*?)\}\s*" + cname + r"\s*;",
                         text, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = re.findall(r"(\w+)\s*;", body)
        assert [f for f, _ in getattr(_lib, cname)._fields_] == fields, cname
