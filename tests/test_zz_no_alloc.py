"""The allocation-free loss/gradient entry point: momfbd_loss_grad_noalloc
(fixed scratch inside the library) against momfbd_loss_grad (caller's
workspace) through the C-ABI, on two calls in a row, the second with a
smaller problem, and both against the FP64 oracle."""

import numpy as np
import pytest

import oracle
import synth
from helpers import LOSS_RTOL, assert_grad_close, simulate_D

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2505_10639_amd import _lib
    _lib.lib()
    return torch.device("cuda:0")


def _case(pr, dev, seed):
    from paper_2505_10639_amd import Plan, _lib
    plan = Plan(pr.N, pr.P, pr.J, pr.channel_object, pr.pupil, pr.basis, pr.diversity, dev)
    D_np = simulate_D(pr)
    D = torch.from_numpy(D_np).to(dev)
    rng = np.random.default_rng(seed)
    a_np = (pr.alpha_true + 0.3 * rng.standard_normal(pr.alpha_true.shape)).astype(np.float32)
    a = torch.from_numpy(a_np).to(dev)
    loss0 = torch.empty(pr.P, dtype=torch.float64, device=dev)
    grad0 = torch.empty((pr.P, pr.J, pr.M), dtype=torch.float32, device=dev)
    _lib.momfbd_loss_grad(plan.handle, a, D, None, pr.gamma, None, loss0, grad0, plan.ws)
    loss1 = torch.full((pr.P,), float("nan"), dtype=torch.float64, device=dev)
    grad1 = torch.full((pr.P, pr.J, pr.M), float("nan"), dtype=torch.float32, device=dev)
    _lib.momfbd_loss_grad_noalloc(plan.handle, a, D, None, pr.gamma, None, loss1, grad1)
    torch.cuda.synchronize()
    assert torch.equal(loss1, loss0) and torch.equal(grad1, grad0)
    ref = oracle.evaluate(a_np, D_np, pr.basis, pr.diversity, pr.pupil, pr.channel_object,
                          pr.gamma)
    l1 = loss1.cpu().numpy()
    assert np.all(np.abs(l1 - ref["loss"]) < LOSS_RTOL * np.abs(ref["loss"]))
    assert_grad_close(grad1.cpu().numpy(), ref["grad"], "noalloc")
    plan.close()


def test_noalloc_matches_the_workspace_entry_point(dev):
    big = synth.make_problem(71, N=64, P=5, J=6, M=30, channels=((0, 0.0), (1, 1.0)),
                             d_over_r0=np.linspace(6.0, 16.0, 5))
    small = synth.make_problem(72, N=64, P=2, J=3, M=12, channels=((0, 0.0),),
                               d_over_r0=np.array([8.0, 12.0]))
    print("[noalloc] first call P=5 J=6 M=30 C=2", flush=True)
    _case(big, dev, 1)
    print("[noalloc] second call P=2 J=3 M=12 C=1", flush=True)
    _case(small, dev, 2)


def test_noalloc_at_128_and_rejects_oversized_plans(dev):
    from paper_2505_10639_amd import Plan, _lib
    pr = synth.make_problem(73, N=128, P=2, J=3, M=20, channels=((0, 0.0), (0, 1.0)),
                            d_over_r0=np.array([8.0, 12.0]))
    print("[noalloc] N=128 P=2 J=3 M=20 C=2", flush=True)
    _case(pr, dev, 3)
    # a plan whose workspace exceeds the fixed scratch is refused, outputs untouched
    plan = Plan(64, 961, 12, [0, 1], np.stack([synth.pupil_mask(64)] * 2).astype(np.float32),
                np.repeat(synth.zernike_basis(64, 66)[None], 2, 0).astype(np.float32), None, dev)
    assert _lib.momfbd_workspace_size(plan.handle) > (64 << 20)
    a = torch.zeros((961, 12, 66), dtype=torch.float32, device=dev)
    D = torch.zeros((961, 2, 12, 64, 33), dtype=torch.complex64, device=dev)
    loss = torch.full((961,), 7.0, dtype=torch.float64, device=dev)
    with pytest.raises(_lib.MomfbdError) as e:
        _lib.momfbd_loss_grad_noalloc(plan.handle, a, D, None, 1e-3, None, loss, None)
    assert e.value.status == _lib.MOMFBD_ESCRATCH
    torch.cuda.synchronize()
    assert bool((loss == 7.0).all())
    plan.close()
