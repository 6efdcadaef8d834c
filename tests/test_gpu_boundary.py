"""The boundary's workspace contract on the GPU: every per-call function of
a plan refuses a workspace one byte shorter than momfbd_workspace_size (and
the solver calls a state one byte shorter than momfbd_lbfgs_state_size)
with MOMFBD_EWORKSPACE before anything is enqueued, so real device outputs
keep their contents; with the full length the same calls succeed."""

import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2505_10639_amd import _lib
    _lib.lib()
    return torch.device("cuda:0")


def _filled(shape, dtype, dev, value):
    t = torch.empty(shape, dtype=dtype, device=dev)
    t.view(torch.uint8).fill_(value)
    return t


def test_short_workspace_and_state_leave_outputs_untouched(dev):
    from paper_2505_10639_amd import Plan, _lib
    L = _lib.lib()
    pr = synth.make_problem(61, N=64, P=2, J=3, M=12, channels=((0, 0.0), (0, 1.0)))
    plan = Plan(pr.N, pr.P, pr.J, pr.channel_object, pr.pupil, pr.basis, pr.diversity, dev)
    h, P, C, J, M, N = plan.handle, pr.P, pr.C, pr.J, pr.M, pr.N
    need = _lib.momfbd_workspace_size(h)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    wp, short = ws.data_ptr(), need - 1
    alpha = torch.from_numpy(pr.alpha_true).to(dev)
    D = torch.randn((P, C, J, N, N // 2 + 1), dtype=torch.complex64, device=dev)
    loss = _filled((P,), torch.float64, dev, 0xA5)
    grad = _filled((P, J, M), torch.float32, dev, 0xA5)
    obj = _filled((P, 1, N, N), torch.float32, dev, 0xA5)
    psf = _filled((P, C, J, N, N), torch.float32, dev, 0xA5)
    otf = _filled((P, C, J, N, N // 2 + 1), torch.complex64, dev, 0xA5)
    Dout = _filled((P, C, J, N, N // 2 + 1), torch.complex64, dev, 0xA5)
    frames = torch.ones((C, J, N + 32, N), dtype=torch.float32, device=dev)
    apod = torch.ones((N, N), dtype=torch.float32, device=dev)
    outs = [loss, grad, obj, psf, otf, Dout]
    snap = [o.clone() for o in outs]
    a, d = alpha.data_ptr(), D.data_ptr()
    filt = (_lib.momfbd_filter * 1)(_lib.filter_spec("none"))
    for n_ws, expect in ((short, -3), (need, 0)):
        print(f"[boundary] workspace {n_ws} of {need} bytes", flush=True)
        st = [L.momfbd_loss_grad(h, a, d, None, 1e-3, None, loss.data_ptr(), grad.data_ptr(),
                                 wp, n_ws, None),
              L.momfbd_forward(h, a, psf.data_ptr(), otf.data_ptr(), wp, n_ws, None),
              L.momfbd_object_estimate(h, a, d, None, 1e-3, None, obj.data_ptr(), wp, n_ws,
                                       None),
              L.momfbd_object_filtered(h, a, d, None, 1e-3, None, filt, obj.data_ptr(), None,
                                       wp, n_ws, None),
              L.momfbd_prepare_data(h, frames.data_ptr(), N + 32, N, 32, apod.data_ptr(),
                                    Dout.data_ptr(), wp, n_ws, None)]
        torch.cuda.synchronize()
        assert st == [expect] * 5, st
        if expect:
            for o, s in zip(outs, snap):
                assert torch.equal(o.view(torch.uint8), s.view(torch.uint8))
    # the solver state: one byte short is refused, the full length accepted
    params = _lib.lbfgs_params()
    nstate = _lib.momfbd_lbfgs_state_size(h, params)
    state = torch.empty(nstate, dtype=torch.uint8, device=dev)
    loss2 = _filled((P,), torch.float64, dev, 0x5A)
    before = loss2.clone()
    pp = ctypes.byref(params)
    assert L.momfbd_lbfgs_init(h, pp, state.data_ptr(), nstate - 1, a, d, None, 1e-3, None,
                               loss2.data_ptr(), wp, need, None) == -3
    assert L.momfbd_lbfgs_init(h, pp, state.data_ptr(), nstate, a, d, None, 1e-3, None,
                               loss2.data_ptr(), wp, need - 1, None) == -3
    torch.cuda.synchronize()
    assert torch.equal(loss2, before)
    assert L.momfbd_lbfgs_init(h, pp, state.data_ptr(), nstate, a, d, None, 1e-3, None,
                               loss2.data_ptr(), wp, need, None) == 0
    a2 = alpha.clone()
    assert L.momfbd_lbfgs_rounds(h, pp, state.data_ptr(), nstate - 1, a2.data_ptr(), d, None,
                                 1e-3, None, 2, None, None, None, wp, need, None) == -3
    assert L.momfbd_lbfgs_step(h, pp, state.data_ptr(), nstate - 1, a2.data_ptr(), d, None,
                               1e-3, None, None, None, wp, need, None) == -3
    torch.cuda.synchronize()
    assert torch.equal(a2, alpha)
    assert L.momfbd_lbfgs_rounds(h, pp, state.data_ptr(), nstate, a2.data_ptr(), d, None,
                                 1e-3, None, 2, None, None, None, wp, need, None) == 0
    torch.cuda.synchronize()
    plan.close()


def test_short_network_workspace(dev):
    from paper_2505_10639_amd import _lib
    L = _lib.lib()
    net = _lib.momfbd_cnn_create(64, 4, 10, 2, np.ones(10, np.float32))
    n_params, need = _lib.momfbd_cnn_sizes(net)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    params = _filled((n_params,), torch.float32, dev, 0x11)
    normals = torch.randn(n_params, device=dev)
    before = params.clone()
    assert L.momfbd_cnn_init(net, normals.data_ptr(), params.data_ptr(), ws.data_ptr(),
                             need - 1, None) == -3
    torch.cuda.synchronize()
    assert torch.equal(params.view(torch.uint8), before.view(torch.uint8))
    assert L.momfbd_cnn_init(net, normals.data_ptr(), params.data_ptr(), ws.data_ptr(), need,
                             None) == 0
    torch.cuda.synchronize()
    _lib.momfbd_cnn_destroy(net)
