"""GPU parity: libmomfbd (hand-written gfx950 kernels through the C-ABI)
against the FP64 oracle, element by element on the same seeded inputs."""

import numpy as np
import pytest

import oracle
import synth
from helpers import (LOSS_RTOL, OBJ_RMS, alpha_points, assert_grad_close, fast_simulate_D,
                     simulate_D)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2505_10639_amd import _lib
    _lib.lib()      # raises if the library is not built
    return torch.device("cuda:0")


def make_plan(pr, dev):
    from paper_2505_10639_amd import Plan
    return Plan(pr.N, pr.P, pr.J, pr.channel_object, pr.pupil, pr.basis, pr.diversity, dev)


def to_dev(x, dev, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    return t.to(dev) if dtype is None else t.to(dev, dtype)


def run_gpu(plan, alpha, D, gamma, weights, dev):
    loss, grad = plan.loss_grad(to_dev(alpha, dev), D, gamma,
                                None if weights is None else to_dev(weights, dev))
    torch.cuda.synchronize()
    return loss.cpu().numpy(), grad.cpu().numpy()


def set_object_fused(plan, on):
    """Switch the one-launch forward/object pass on or off, keeping the other
    launch schedules; returns whether it is in use."""
    t = plan.tuning()
    plan.set_tuning(t["xcd_forward"], t["xcd_adjoint"], t["object_pairs_per_thread"],
                    t["grad_waves"], t["grad_splits"], t["grad_row_tiles"], t["phase_col_tiles"],
                    t["phase_waves"], int(on))
    return bool(plan.tuning()["object_fused"])


def check_patchwise(pr, D_np, alphas, dev, gamma=None, weights=None, patches=None):
    """Loss and gradient against the oracle on every (or the sampled)
    patch; where the plan allows the forward and object pass in one launch,
    that schedule must give the same loss and gradient bit for bit."""
    plan = make_plan(pr, dev)
    D = to_dev(D_np, dev)
    g = pr.gamma if gamma is None else gamma
    for name, a in alphas.items():
        print(f"[parity] N={pr.N} P={pr.P} C={pr.C} K={pr.K} J={pr.J} M={pr.M} alpha={name}",
              flush=True)
        loss, grad = run_gpu(plan, a, D, g if np.isscalar(g) else to_dev(g, dev), weights, dev)
        if set_object_fused(plan, True):
            l1, g1 = run_gpu(plan, a, D, g if np.isscalar(g) else to_dev(g, dev), weights, dev)
            assert np.array_equal(l1, loss) and np.array_equal(g1, grad), name
            set_object_fused(plan, False)
        idx = range(pr.P) if patches is None else patches
        g_ref = g if np.isscalar(g) else oracle.expand_half(g, pr.N).real
        ref = oracle.evaluate(a, D_np, pr.basis, pr.diversity, pr.pupil, pr.channel_object,
                              g_ref, weights, patches=list(idx))
        lrel = np.abs(loss[list(idx)] - ref["loss"]) / np.abs(ref["loss"])
        assert np.all(lrel < LOSS_RTOL), (name, lrel.max())
        assert_grad_close(grad[list(idx)], ref["grad"], name)
    plan.close()


def test_config0_loss_and_gradient(dev):
    pr = synth.config0()
    check_patchwise(pr, simulate_D(pr), alpha_points(pr), dev)


def test_ragged_multi_patch_phase_diversity(dev):
    # 3 patches, one object seen in focus and with +1 wave defocus, 5 frames
    pr = synth.make_problem(41, N=64, P=3, J=5, M=20, channels=((0, 0.0), (0, 1.0)),
                            d_over_r0=np.array([6.0, 12.0, 18.0]))
    check_patchwise(pr, simulate_D(pr), alpha_points(pr, 1), dev)


def test_two_objects_weights_and_gamma_array(dev):
    pr = synth.make_problem(42, N=64, P=2, J=3, M=30, channels=((0, 0.0), (1, 1.0), (1, 0.0)),
                            d_over_r0=10.0)
    w = np.array([[1.0, 0.5, 2.0], [0.7, 1.3, 1.0], [1.1, 0.9, 0.4]], np.float32)
    ky = np.fft.fftfreq(64)[:, None]
    kx = np.arange(33)[None, :] / 64.0
    gam = np.stack([1e-3 + 0.02 * (np.sin(np.pi * ky) ** 2 + np.sin(np.pi * kx) ** 2),
                    np.full((64, 33), 5e-3)]).astype(np.float32)
    check_patchwise(pr, simulate_D(pr), alpha_points(pr, 2), dev, gamma=gam, weights=w)


def test_single_frame_phase_diversity(dev):
    # One frame seen in focus and with +1 wave defocus (single-frame phase
    # diversity, as for the IMaX data of the results section).  Tip and tilt
    # then shift both images alike, to which the loss is exactly invariant, so
    # their gradient vanishes.
    pr = synth.make_problem(43, N=64, P=1, J=1, M=10, channels=((0, 0.0), (0, 1.0)),
                            d_over_r0=8.0)
    D = simulate_D(pr)
    check_patchwise(pr, D, alpha_points(pr, 3), dev)
    plan = make_plan(pr, dev)
    _, grad = run_gpu(plan, alpha_points(pr, 3)["perturbed"], to_dev(D, dev), pr.gamma, None,
                      dev)
    assert np.all(np.abs(grad[0, 0, :2]) <= 1e-4 * np.linalg.norm(grad[0, 0, 2:]))
    plan.close()


def test_forward_psf_and_otf(dev):
    pr = synth.make_problem(44, N=64, P=2, J=3, M=44, channels=((0, 0.0), (0, 1.0)),
                            d_over_r0=15.0)
    plan = make_plan(pr, dev)
    psf, otf = plan.forward(to_dev(pr.alpha_true, dev))
    psf, otf = psf.cpu().numpy(), otf.cpu().numpy()
    for p in range(2):
        for c in range(2):
            for j in range(3):
                phi = oracle.wavefront(pr.alpha_true[p, j], pr.basis[c], pr.diversity[c])
                s = oracle.psf(pr.pupil[c], phi)
                assert np.abs(psf[p, c, j] - s).max() <= 2e-6 * s.max()
                assert abs(psf[p, c, j].astype(np.float64).sum() - 1.0) < 1e-5
                S = oracle.otf(s)[:, :33]
                assert np.abs(otf[p, c, j] - S).max() <= 2e-6
    # flat wavefront: peak N_A/N^2 at pixel (0,0)
    psf0, _ = plan.forward(torch.zeros((2, 3, 44), device=dev), want_otf=False)
    assert abs(float(psf0[0, 0, 0, 0, 0]) - 657 / 4096) < 1e-6
    plan.close()


def test_object_estimate(dev):
    pr = synth.config0()
    D = simulate_D(pr)
    plan = make_plan(pr, dev)
    for name, a in alpha_points(pr, 4).items():
        obj = plan.object_estimate(to_dev(a, dev), to_dev(D, dev), pr.gamma).cpu().numpy()
        ref = oracle.evaluate(a, D, pr.basis, pr.diversity, pr.pupil, pr.channel_object,
                              pr.gamma, want_grad=False)
        o_ref = oracle.object_image(ref["O"][0, 0])
        rms = np.sqrt(np.mean((obj[0, 0] - o_ref) ** 2))
        assert rms < OBJ_RMS, (name, rms)
    plan.close()


def test_irregular_pupils_spectral_support(dev):
    """The kernels skip the spectra outside each object's spectral support
    (the difference set of its channels' pupils, bounded per column).  Two
    channels of one object with irregular pupils: two separate
    sub-apertures (a three-lobed difference set) and an off-centre annulus.
    Loss, gradient and restored object still match the oracle."""
    pr = synth.make_problem(79, N=64, P=2, J=4, M=20, channels=((0, 0.0), (0, 0.0)),
                            d_over_r0=np.array([8.0, 12.0]), border=6)
    y, x = np.mgrid[0:64, 0:64].astype(np.float64)
    two = (((y - 31) ** 2 + (x - 23) ** 2 <= 25) | ((y - 33) ** 2 + (x - 41) ** 2 <= 25))
    r2 = (y - 35) ** 2 + (x - 28) ** 2
    ring = (r2 <= 144) & (r2 >= 25)
    pr.pupil = np.stack([two, ring]).astype(np.float32)
    D_np = simulate_D(pr)
    check_patchwise(pr, D_np, alpha_points(pr, 13), dev)
    plan = make_plan(pr, dev)
    a = alpha_points(pr, 13)["perturbed"]
    obj = plan.object_estimate(to_dev(a, dev), to_dev(D_np, dev), pr.gamma).cpu().numpy()
    ref = oracle.evaluate(a, D_np, pr.basis, pr.diversity, pr.pupil, pr.channel_object,
                          pr.gamma, want_grad=False)
    for p in range(pr.P):
        rms = np.sqrt(np.mean((obj[p, 0] - oracle.object_image(ref["O"][p, 0])) ** 2))
        assert rms < OBJ_RMS, rms
    plan.close()


def test_prepare_data_ragged_grid(dev):
    rng = np.random.default_rng(45)
    C, J, H, W, stride = 2, 3, 150, 171, 40
    frames = (1.0 + 0.1 * rng.standard_normal((C, J, H, W))).astype(np.float32)
    win = synth.hann_window(64, 6).astype(np.float32)
    ny, nx = (H - 64) // stride + 1, (W - 64) // stride + 1
    pr = synth.make_problem(45, N=64, P=ny * nx, J=J, M=4, channels=((0, 0.0), (0, 1.0)))
    plan = make_plan(pr, dev)
    D = plan.prepare_data(to_dev(frames, dev), stride, to_dev(win, dev)).cpu().numpy()
    ref = oracle.prepare_data(frames, win, 64, stride)
    assert D.shape == ref.shape
    assert np.abs(D - ref).max() <= 1e-6 * np.abs(ref).max()
    plan.close()


def test_nan_propagates_to_its_patch_only(dev):
    pr = synth.make_problem(46, N=64, P=3, J=2, M=10)
    D = to_dev(simulate_D(pr), dev)
    plan = make_plan(pr, dev)
    a = pr.alpha_true.copy()
    l0, _ = run_gpu(plan, a, D, pr.gamma, None, dev)
    a[1, 0, 3] = np.nan
    l1, g1 = run_gpu(plan, a, D, pr.gamma, None, dev)
    assert np.isnan(l1[1]) and np.all(np.isnan(g1[1]))
    assert l1[0] == l0[0] and l1[2] == l0[2]
    plan.close()


def test_autograd_function(dev):
    from paper_2505_10639_amd import momfbd_loss
    pr = synth.config0()
    D = to_dev(simulate_D(pr), dev)
    plan = make_plan(pr, dev)
    a = to_dev(pr.alpha_true, dev).requires_grad_(True)
    L = momfbd_loss(a, plan, D, pr.gamma)
    (3.0 * L).backward()
    loss, grad = plan.loss_grad(a.detach(), D, pr.gamma)
    assert float(L.detach()) == float(loss.sum())
    assert torch.equal(a.grad, 3.0 * grad)
    plan.close()


def test_config1_full_size_sampled_patches(dev):
    """Full-field workload (961 patches, 12 frames, 2 objects, 66 modes) in the
    launch configuration of the benchmark; outputs compared on sampled patches.

    The data of every patch is synthesised with numpy.fft (inputs only); for
    the sampled patches it is replaced by the oracle's own simulation, which
    must agree with the fast one."""
    sample = [0, 30, 480, 517, 930, 960]
    pr_all = synth.config1_problem()
    D = fast_simulate_D(pr_all)
    D_s = simulate_D(synth.config1_problem(sample))
    assert np.abs(D[sample] - D_s).max() <= 1e-5 * np.abs(D_s).max()
    D[sample] = D_s
    rng = np.random.default_rng(47)
    alphas = {"perturbed": (pr_all.alpha_true
                            + 0.3 * rng.standard_normal(pr_all.alpha_true.shape)).astype(np.float32)}
    check_patchwise(pr_all, D, alphas, dev, patches=sample)


def test_config4_full_size_sampled_patches(dev):
    """Large multi-object workload at full size: 961 patches of 128x128, four
    objects at four wavelengths, 24 frames, 150 modes and the smoothness
    prior.  The launch schedule is the autotuned one the benchmark times;
    outputs are compared on sampled patches.

    Patches are independent, so only the sampled patches need the oracle's
    simulated data; the others hold seeded random spectra that fill the
    launch and are not compared."""
    from paper_2505_10639_amd import Plan
    sample = [0, 31, 517, 960]
    g = synth.config4_geometry()
    N, P, C, J = g["N"], g["P"], g["C"], g["J"]
    pr = synth.config4_problem(sample)
    D_s = simulate_D(pr)
    gen = torch.Generator(device=dev)
    gen.manual_seed(synth.SEED_ROOT + 41)
    D = float(np.sqrt(np.mean(np.abs(D_s) ** 2))) * torch.randn(
        (P, C, J, N, N // 2 + 1), dtype=torch.complex64, generator=gen, device=dev)
    D[sample] = to_dev(D_s, dev)
    rng = np.random.default_rng(48)
    a_all = synth.config4_alpha()
    a_all += (0.3 * rng.standard_normal(a_all.shape)).astype(np.float32)
    alpha = to_dev(a_all, dev)
    plan = Plan(N, P, J, pr.channel_object, pr.pupil, pr.basis, None, dev)
    g0, lam = [g["gamma"]] * g["K"], [g["smooth"]] * g["K"]
    g_dev = plan.smoothness_gamma(g0, lam)
    print(f"[config4] P={P} C={C} J={J} M={g['M']}: autotune", flush=True)
    plan.autotune(alpha, D, g_dev, None, reps=1)
    print(f"[config4] schedule {plan.tuning()}", flush=True)
    loss, grad = plan.loss_grad(alpha, D, g_dev)
    torch.cuda.synchronize()
    loss, grad = loss.cpu().numpy(), grad.cpu().numpy()
    assert np.all(np.isfinite(loss)) and np.all(np.isfinite(grad))
    ref = oracle.evaluate(a_all[sample], D_s, pr.basis, pr.diversity, pr.pupil,
                          pr.channel_object, oracle.smoothness_gamma(N, g0, lam))
    lrel = np.abs(loss[sample] - ref["loss"]) / np.abs(ref["loss"])
    assert np.all(lrel < LOSS_RTOL), lrel.max()
    assert_grad_close(grad[sample], ref["grad"], "config4")
    plan.close()


def test_lbfgs_first_step_matches_oracle_and_converges(dev):
    """Per-patch L-BFGS: the first iteration takes the same step as the
    reference solver; the loss never increases; after 150 iterations every
    patch is below the loss at the true coefficients."""
    from oracle.lbfgs import two_loop, wolfe_search
    from paper_2505_10639_amd import Solver
    pr = synth.make_problem(48, N=64, P=3, J=8, M=44, d_over_r0=np.array([6.0, 10.0, 14.0]))
    D_np = simulate_D(pr)
    D = to_dev(D_np, dev)
    plan = make_plan(pr, dev)
    alpha = torch.zeros((pr.P, pr.J, pr.M), device=dev)
    sol = Solver(plan, alpha, D, pr.gamma)
    l0 = sol.loss.cpu().numpy().copy()
    loss, status = sol.step()
    l1 = loss.cpu().numpy().copy()
    a1 = alpha.cpu().numpy().copy()
    for p in range(pr.P):
        shape = (pr.J, pr.M)

        def fg(x):
            r = oracle.evaluate_patch(x.reshape(shape), D_np[p], pr.basis, pr.diversity,
                                      pr.pupil, pr.channel_object, pr.gamma)
            return r["loss"], r["grad"].ravel()

        x = np.zeros(pr.J * pr.M)
        f, g = fg(x)
        assert abs(l0[p] - f) < LOSS_RTOL * f
        d = two_loop(g, [], [])
        t0 = min(1.0, 1.0 / np.max(np.abs(g)))
        t, fn, gn, _, ok = wolfe_search(fg, x, f, g, d, t0)
        assert ok
        assert abs(l1[p] - fn) < 1e-4 * fn, (p, l1[p], fn)
        np.testing.assert_allclose(a1[p].ravel(), t * d, rtol=1e-3, atol=1e-6 * np.abs(t * d).max())
    hist = [l1]
    for _ in range(149):
        loss, status = sol.step()
        hist.append(loss.cpu().numpy().copy())
    hist = np.array(hist)
    assert np.all(np.diff(hist, axis=0) <= 1e-9 * np.abs(hist[:-1]))
    l_true, _ = run_gpu(plan, pr.alpha_true, D, pr.gamma, None, dev)
    assert np.all(hist[-1] < l_true), (hist[-1], l_true)
    # the returned loss is the loss at the returned coefficients
    l_chk, _ = run_gpu(plan, alpha.cpu().numpy(), D, pr.gamma, None, dev)
    np.testing.assert_allclose(l_chk, hist[-1], rtol=1e-12)
    plan.close()


@pytest.mark.parametrize("N", [64, 128])
def test_smoothness_prior_gamma(dev, N):
    """The library's smoothness-prior gamma table matches the oracle's, and
    the loss and gradient under it match the oracle."""
    pr = synth.make_problem(50 + N, N=N, P=2, J=4, M=24, channels=((0, 0.0), (1, 1.0)),
                            d_over_r0=np.array([8.0, 14.0]))
    D_np = fast_simulate_D(pr)
    plan = make_plan(pr, dev)
    g0, lam = [1e-3, 4e-3], [0.05, 0.4]
    g_dev = plan.smoothness_gamma(g0, lam)
    torch.cuda.synchronize()
    g_ref = oracle.smoothness_gamma(N, g0, lam)
    np.testing.assert_allclose(g_dev.cpu().numpy(), g_ref[:, :, : N // 2 + 1], rtol=2e-7, atol=0)
    D = to_dev(D_np, dev)
    for name, a in alpha_points(pr, 3).items():
        print(f"[smoothness] N={N} alpha={name}", flush=True)
        loss, grad = plan.loss_grad(to_dev(a, dev), D, g_dev)
        ref = oracle.evaluate(a, D_np, pr.basis, pr.diversity, pr.pupil, pr.channel_object, g_ref)
        lrel = np.abs(loss.cpu().numpy() - ref["loss"]) / np.abs(ref["loss"])
        assert np.all(lrel < LOSS_RTOL), (name, lrel.max())
        assert_grad_close(grad.cpu().numpy(), ref["grad"], name)
    plan.close()


def test_lbfgs_later_steps_match_oracle(dev):
    """Iterations 2-4 (the two-loop recursion with one to three stored
    pairs): from each of the solver's accepted points, the reference solver
    given the same history (pairs formed from the solver's points and the
    oracle's gradients) takes the same step."""
    from oracle.lbfgs import two_loop, wolfe_search
    from paper_2505_10639_amd import Solver
    pr = synth.make_problem(49, N=64, P=2, J=4, M=20, d_over_r0=np.array([8.0, 12.0]))
    D_np = simulate_D(pr)
    D = to_dev(D_np, dev)
    plan = make_plan(pr, dev)
    alpha = torch.zeros((pr.P, pr.J, pr.M), device=dev)
    sol = Solver(plan, alpha, D, pr.gamma)
    xs = [alpha.cpu().numpy().reshape(pr.P, -1).astype(np.float64)]
    for _ in range(4):
        sol.step()
        xs.append(alpha.cpu().numpy().reshape(pr.P, -1).astype(np.float64))
    for p in range(pr.P):
        def fg(x):
            r = oracle.evaluate_patch(x.reshape(pr.J, pr.M), D_np[p], pr.basis, pr.diversity,
                                      pr.pupil, pr.channel_object, pr.gamma)
            return r["loss"], r["grad"].ravel()
        gs = [fg(x[p])[1] for x in xs]
        for k in range(1, 4):
            S = [xs[i + 1][p] - xs[i][p] for i in range(k)]
            Y = [gs[i + 1] - gs[i] for i in range(k)]
            f, g = fg(xs[k][p])
            d = two_loop(g, S, Y)
            t, fn, _, _, ok = wolfe_search(fg, xs[k][p], f, g, d, 1.0)
            assert ok
            step_ref, step_gpu = t * d, xs[k + 1][p] - xs[k][p]
            print(f"[lbfgs] patch {p} iteration {k + 1}: t {t:.4f} "
                  f"step rel diff {np.linalg.norm(step_gpu - step_ref) / np.linalg.norm(step_ref):.2e}",
                  flush=True)
            assert np.linalg.norm(step_gpu - step_ref) < 1e-4 * np.linalg.norm(step_ref)
    plan.close()


def test_lbfgs_long_coefficient_vectors_match_oracle(dev):
    """J M = 2304 coefficients per patch (past the register-resident
    two-loop, which holds up to 2048): iterations 2 and 3 match the
    reference solver from the solver's own points."""
    from oracle.lbfgs import two_loop, wolfe_search
    from paper_2505_10639_amd import Solver
    pr = synth.make_problem(51, N=64, P=1, J=24, M=96, d_over_r0=10.0)
    D_np = simulate_D(pr)
    D = to_dev(D_np, dev)
    plan = make_plan(pr, dev)
    alpha = torch.zeros((pr.P, pr.J, pr.M), device=dev)
    sol = Solver(plan, alpha, D, pr.gamma)
    xs = [alpha.cpu().numpy().reshape(-1).astype(np.float64)]
    for _ in range(3):
        sol.step()
        xs.append(alpha.cpu().numpy().reshape(-1).astype(np.float64))

    def fg(x):
        r = oracle.evaluate_patch(x.reshape(pr.J, pr.M), D_np[0], pr.basis, pr.diversity,
                                  pr.pupil, pr.channel_object, pr.gamma)
        return r["loss"], r["grad"].ravel()
    gs = [fg(x)[1] for x in xs]
    for k in (1, 2):
        S = [xs[i + 1] - xs[i] for i in range(k)]
        Y = [gs[i + 1] - gs[i] for i in range(k)]
        f, g = fg(xs[k])
        d = two_loop(g, S, Y)
        t, _, _, _, ok = wolfe_search(fg, xs[k], f, g, d, 1.0)
        assert ok
        step_ref, step_gpu = t * d, xs[k + 1] - xs[k]
        assert np.linalg.norm(step_gpu - step_ref) < 1e-4 * np.linalg.norm(step_ref)
    plan.close()


def test_lbfgs_rounds_follow_the_step_trajectories(dev):
    """Round mode (no host read-back) runs every patch through the same
    iterations as step mode: run both until every patch has stopped and
    compare the accepted coefficients and losses bit for bit."""
    from paper_2505_10639_amd import Solver
    pr = synth.make_problem(58, N=64, P=4, J=5, M=24, d_over_r0=np.array([6.0, 9.0, 12.0, 15.0]))
    D = to_dev(fast_simulate_D(pr), dev)
    plan = make_plan(pr, dev)
    x1 = torch.zeros((pr.P, pr.J, pr.M), device=dev)
    s1 = Solver(plan, x1, D, pr.gamma, ftol=1e-4)
    for _ in range(600):
        _, st = s1.step()
        if bool((st != 0).all()):
            break
    assert bool((s1.status != 0).all())
    x2 = torch.zeros_like(x1)
    out = torch.empty_like(x1)
    s2 = Solver(plan, x2, D, pr.gamma, ftol=1e-4)
    for _ in range(100):
        s2.rounds(25, out)
        if bool((s2.status != 0).all()):
            break
    torch.cuda.synchronize()
    assert bool((s2.status != 0).all())
    assert torch.equal(s1.status, s2.status)
    assert torch.equal(s1.loss, s2.loss)
    assert torch.equal(x1, out)
    # the forward and object pass in one launch, with the solver's per-patch
    # masks (patches stop at different rounds): the same trajectories
    assert set_object_fused(plan, True)
    x3 = torch.zeros_like(x1)
    out3 = torch.empty_like(x1)
    s3 = Solver(plan, x3, D, pr.gamma, ftol=1e-4)
    for _ in range(100):
        s3.rounds(25, out3)
        if bool((s3.status != 0).all()):
            break
    torch.cuda.synchronize()
    assert torch.equal(s1.status, s3.status)
    assert torch.equal(s1.loss, s3.loss)
    assert torch.equal(x1, out3)
    plan.close()


def test_solve_rounds_until_reports_the_accepted_point(dev):
    """The chunked round driver: the summed accepted loss never rises from
    chunk to chunk, it stops at the target, and the coefficients it returns
    have exactly the loss it reports."""
    from paper_2505_10639_amd.warmstart import solve_rounds_until
    pr = synth.make_problem(59, N=64, P=4, J=5, M=24, d_over_r0=np.array([6.0, 9.0, 12.0, 15.0]))
    D = to_dev(fast_simulate_D(pr), dev)
    plan = make_plan(pr, dev)
    zero = torch.zeros((pr.P, pr.J, pr.M), device=dev)
    h, _, acc, r = solve_rounds_until(plan, zero, D, pr.gamma, None, max_rounds=800, chunk=8,
                                      stall=5, rtol=1e-9)
    assert all(b <= a for a, b in zip(h, h[1:])) and h[-1] < 0.9 * h[0]
    assert r % 8 == 0 and r <= 800
    L = float(plan.loss_grad(acc, D, pr.gamma)[0].sum())
    assert L == pytest.approx(h[-1], rel=1e-12)
    target = h[0] - 0.9 * (h[0] - h[-1])
    h2, _, acc2, r2 = solve_rounds_until(plan, zero, D, pr.gamma, target, chunk=8)
    assert h2[-1] <= target and (len(h2) < 3 or h2[-2] > target) and r2 <= r
    plan.close()


def test_lbfgs_rounds_replay_from_a_hip_graph(dev):
    """Rounds captured once in a HIP graph and replayed four times, with
    other eager work in between, match eager rounds bit for bit."""
    from paper_2505_10639_amd import Solver
    pr = synth.make_problem(59, N=64, P=5, J=6, M=30, channels=((0, 0.0), (1, 1.0)))
    D = to_dev(fast_simulate_D(pr), dev)
    plan = make_plan(pr, dev)
    xa = torch.zeros((pr.P, pr.J, pr.M), device=dev)
    oa = torch.empty_like(xa)
    sa = Solver(plan, xa, D, pr.gamma)
    ref = []
    for _ in range(4):
        sa.rounds(5, oa)
        torch.cuda.synchronize()
        ref.append((oa.clone(), sa.loss.clone(), sa.status.clone()))
    xb = torch.zeros_like(xa)
    ob = torch.empty_like(xa)
    sb = Solver(plan, xb, D, pr.gamma)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sb.rounds(5, ob)
    other = to_dev(alpha_points(pr, 4)["perturbed"], dev)
    for k in range(4):
        g.replay()
        torch.cuda.synchronize()
        print(f"[graph] replay {k} loss {float(sb.loss.sum()):.6f}", flush=True)
        assert torch.equal(ob, ref[k][0]) and torch.equal(sb.loss, ref[k][1])
        assert torch.equal(sb.status, ref[k][2])
        plan.loss_grad(other, D, pr.gamma)        # eager work on the same plan in between
        torch.cuda.synchronize()
    plan.close()


def test_karhunen_loeve_basis(dev):
    """The same data with the KL modes as the basis (the paper's default):
    loss and gradient at the KL coefficients of the same wavefronts."""
    pr = synth.make_problem(57, N=64, P=2, J=6, M=30, channels=((0, 0.0), (0, 1.0)),
                            d_over_r0=np.array([8.0, 14.0]))
    D_np = simulate_D(pr)
    U, _ = synth.kl_transform(pr.M)
    KL, _ = synth.kl_basis(64, pr.M, 0.45)
    pr.basis = np.stack([KL] * pr.C).astype(np.float32)
    pr.alpha_true = (pr.alpha_true.astype(np.float64) @ U).astype(np.float32)
    check_patchwise(pr, D_np, alpha_points(pr, 5), dev)


@pytest.mark.parametrize("N", [64, 96, 128])
def test_launch_schedules_and_autotune(dev, N):
    """Every launch schedule gives the default results: bit for bit where
    only the order of the work changes (unit order), to the rounding of a
    regrouped sum where the grouping of partial sums changes (object pairs
    per thread: FP64 loss; gradient pixel-sum splits: FP32 gradient).  The
    gradient's waves and row tiles per wave change which wave sums a row,
    not the order of its sum, so they give the same gradient bit for bit at
    equal splits.  The split counts include ones that leave workgroups with
    different chunk counts (N = 96: 72 chunks of 32 pixels over 8 splits).
    The phase contraction's block shape changes which wave forms a value of
    phi, not its sum: bit for bit as well.  The autotuned plan still
    matches the oracle."""
    pr = synth.make_problem(70 + N, N=N, P=3, J=3, M=28, channels=((0, 0.0), (1, 1.0)),
                            d_over_r0=np.array([7.0, 11.0, 15.0]), border=N // 10)
    D_np = simulate_D(pr)
    D = to_dev(D_np, dev)
    a = to_dev(alpha_points(pr, 10)["perturbed"], dev)
    plan = make_plan(pr, dev)
    # 9 rows (p, j): one row block, so the automatic split count is the
    # largest that leaves every split at least 8 chunks of 32 pixels (one
    # shared basis: 32 chunks at N = 64, 72 at N = 96, 128 at N = 128)
    auto = {64: 4, 96: 8, 128: 8}[N]
    assert plan.tuning() == {"xcd_forward": 0, "xcd_adjoint": 1, "object_pairs_per_thread": 1,
                             "grad_waves": 4, "grad_splits": auto, "grad_row_tiles": 4,
                             "phase_col_tiles": 8, "phase_waves": 8, "object_fused": 0}
    # the forward and object pass in one launch applies at N = 64 (3 units per
    # (patch, object) here)
    fused = 1 if N == 64 else 0
    l0, g0 = (t.clone() for t in plan.loss_grad(a, D, pr.gamma))
    for knobs in [(1, 1, 1, 4), (0, 0, 1, 4), (0, 1, 2, 4), (0, 1, 4, 4), (0, 1, 1, 8),
                  (1, 0, 4, 8), (0, 1, 1, 4, 8), (0, 1, 1, 4, 1), (0, 1, 1, 4, 2),
                  (0, 1, 1, 8, 8), (0, 1, 1, 8, 1), (0, 1, 1, 4, 8, 3), (0, 1, 1, 4, 2, 3),
                  (0, 1, 1, 4, auto, 2), (0, 1, 1, 4, 1, 2), (0, 1, 1, 8, auto),
                  (0, 1, 1, 4, auto, 0, 4, 8), (0, 1, 1, 4, auto, 0, 8, 16),
                  (0, 1, 1, 4, auto, 0, 8, 8), (0, 1, 1, 4, auto, 0, 0, 0, 1),
                  (1, 0, 1, 4, auto, 0, 0, 0, 1), (0, 1, 2, 4, auto, 0, 4, 8, 1)]:
        print(f"[tuning] N={N} {knobs}", flush=True)
        plan.set_tuning(*knobs)
        l1, g1 = plan.loss_grad(a, D, pr.gamma)
        torch.cuda.synchronize()
        # the one-launch pass is the two-launch pass with one pair per thread
        assert plan.tuning()["object_fused"] == (fused if len(knobs) == 9 else 0)
        if knobs[2] == 1 or plan.tuning()["object_fused"]:
            assert torch.equal(l1, l0)
        else:
            assert float(((l1 - l0).abs() / l0.abs()).max()) < 1e-12
        if plan.tuning()["grad_splits"] == auto:
            assert torch.equal(g1, g0)
        else:
            assert float((g1 - g0).norm() / g0.norm()) < 1e-6
    plan.set_tuning(0, 1, 1, 4)
    chosen = plan.autotune(a, D, pr.gamma, reps=2)
    print(f"[tuning] N={N} autotuned {chosen}", flush=True)
    assert chosen == plan.tuning()
    loss, grad = run_gpu(plan, alpha_points(pr, 10)["perturbed"], D, pr.gamma, None, dev)
    ref = oracle.evaluate(alpha_points(pr, 10)["perturbed"], D_np, pr.basis, pr.diversity,
                          pr.pupil, pr.channel_object, pr.gamma)
    assert np.all(np.abs(loss - ref["loss"]) / np.abs(ref["loss"]) < LOSS_RTOL)
    assert_grad_close(grad, ref["grad"], "autotuned")
    with pytest.raises(Exception):
        plan.set_tuning(0, 1, 3, 4)
    with pytest.raises(Exception):
        plan.set_tuning(0, 1, 1, 4, 3)
    with pytest.raises(Exception):
        plan.set_tuning(0, 1, 1, 8, 0, 3)
    with pytest.raises(Exception):
        plan.set_tuning(0, 1, 1, 4, 0, 1)
    with pytest.raises(Exception):
        plan.set_tuning(0, 1, 1, 4, 0, 0, 4, 4)
    with pytest.raises(Exception):
        plan.set_tuning(0, 1, 1, 4, 0, 0, 8, 0)
    with pytest.raises(Exception):
        plan.set_tuning(0, 1, 1, 4, 0, 0, 0, 0, 2)
    plan.close()


def test_one_launch_pass_applies_up_to_twelve_units_per_object(dev):
    """The forward/object pass in one launch takes a (patch, object) per
    workgroup of at most 12 waves: a plan with 13 frames of one object keeps
    the two launches when asked for it (get_tuning reports 0) and gives the
    same results; with 12 frames it runs in one launch, bit for bit."""
    for J, fused in ((13, False), (12, True)):
        pr = synth.make_problem(230 + J, N=64, P=2, J=J, M=12, d_over_r0=8.0)
        D = to_dev(simulate_D(pr), dev)
        a = to_dev(alpha_points(pr, 1)["perturbed"], dev)
        plan = make_plan(pr, dev)
        l0, g0 = (t.clone() for t in plan.loss_grad(a, D, pr.gamma))
        assert set_object_fused(plan, True) == fused
        l1, g1 = plan.loss_grad(a, D, pr.gamma)
        torch.cuda.synchronize()
        assert torch.equal(l1, l0) and torch.equal(g1, g0)
        plan.close()


def test_kernel_timing_leaves_results_unchanged(dev):
    """The library's kernel timing (an event pair per launch, or one kind
    repeated back to back inside its pair) changes no result bit."""
    from paper_2505_10639_amd import (momfbd_profile_repeat, momfbd_profile_start,
                                      momfbd_profile_stop)

    pr = synth.make_problem(77, N=64, P=3, J=3, M=21, channels=((0, 0.0), (1, 1.0)),
                            d_over_r0=np.array([6.0, 10.0, 14.0]), border=6)
    D = to_dev(simulate_D(pr), dev)
    a = to_dev(alpha_points(pr, 11)["perturbed"], dev)
    plan = make_plan(pr, dev)
    l0, g0 = (t.clone() for t in plan.loss_grad(a, D, pr.gamma))
    # the forward and object pass in one launch (3 units per (patch, object)),
    # then in two
    for fused, kinds in ((1, ("phase", "forward_object", "adjoint", "grad")),
                         (0, ("phase", "forward", "object", "adjoint", "grad"))):
        plan.set_tuning(0, 1, 1, 4, object_fused=fused)
        momfbd_profile_start(plan.handle, 64)
        l1, g1 = plan.loss_grad(a, D, pr.gamma)
        kern = momfbd_profile_stop(plan.handle)
        assert torch.equal(l1, l0) and torch.equal(g1, g0)
        assert {k: v[1] for k, v in kern.items()} == {k: 1 for k in kinds}
        for kind in kinds:
            print(f"[timing] repeat {kind}", flush=True)
            momfbd_profile_start(plan.handle, 8)
            momfbd_profile_repeat(plan.handle, kind, 3)
            for _ in range(2):
                l1, g1 = plan.loss_grad(a, D, pr.gamma)
            kern = momfbd_profile_stop(plan.handle)
            assert torch.equal(l1, l0) and torch.equal(g1, g0)
            assert list(kern) == [kind] and kern[kind][1] == 6 and kern[kind][0] > 0
    momfbd_profile_start(plan.handle, 8)
    with pytest.raises(Exception):
        momfbd_profile_repeat(plan.handle, "filter", 2)
    with pytest.raises(Exception):
        momfbd_profile_repeat(plan.handle, "no_such_kernel", 2)
    momfbd_profile_stop(plan.handle)
    with pytest.raises(Exception):   # no timing started
        momfbd_profile_repeat(plan.handle, "adjoint", 2)
    plan.close()


# ------------------------------------------------------------ 128 x 128 patches

def test_n128_loss_and_gradient(dev):
    # config-4 patch size: 128x128 patches, 12-pixel apodization border
    pr = synth.make_problem(50, N=128, P=2, J=3, M=44, channels=((0, 0.0), (0, 1.0)),
                            d_over_r0=np.array([10.0, 15.0]), border=12)
    check_patchwise(pr, simulate_D(pr), alpha_points(pr, 5), dev)


def test_n128_multi_wavelength_objects(dev):
    # four objects at lambda_0/lambda = 1, 1/0.95, 1/1.05, 1/1.1 sharing the
    # wavefront coefficients (phases and pupil sizes scaled per channel)
    lam = [1.0, 1 / 0.95, 1 / 1.05, 1 / 1.1]
    pr = synth.make_problem(51, N=128, P=1, J=2, M=30,
                            channels=((0, 0.0), (1, 0.0), (2, 0.0), (3, 0.0)),
                            lam_ratios=lam, d_over_r0=15.0, border=12)
    check_patchwise(pr, simulate_D(pr), alpha_points(pr, 6), dev)


def test_n128_forward_object_prepare(dev):
    pr = synth.make_problem(52, N=128, P=2, J=2, M=20, d_over_r0=15.0, border=12)
    plan = make_plan(pr, dev)
    psf, otf = plan.forward(to_dev(pr.alpha_true, dev))
    psf, otf = psf.cpu().numpy(), otf.cpu().numpy()
    for p in range(2):
        for j in range(2):
            phi = oracle.wavefront(pr.alpha_true[p, j], pr.basis[0], pr.diversity[0])
            s = oracle.psf(pr.pupil[0], phi)
            assert np.abs(psf[p, 0, j] - s).max() <= 2e-6 * s.max()
            assert np.abs(otf[p, 0, j] - oracle.otf(s)[:, :65]).max() <= 2e-6
    psf0, _ = plan.forward(torch.zeros((2, 2, 20), device=dev), want_otf=False)
    assert abs(float(psf0[0, 0, 0, 0, 0]) - 2601 / 16384) < 1e-6
    D = simulate_D(pr)
    obj = plan.object_estimate(to_dev(pr.alpha_true, dev), to_dev(D, dev), pr.gamma).cpu().numpy()
    ref = oracle.evaluate(pr.alpha_true, D, pr.basis, pr.diversity, pr.pupil, pr.channel_object,
                          pr.gamma, want_grad=False)
    for p in range(2):
        rms = np.sqrt(np.mean((obj[p, 0] - oracle.object_image(ref["O"][p, 0])) ** 2))
        assert rms < OBJ_RMS, rms
    plan.close()
    rng = np.random.default_rng(53)
    frames = (1.0 + 0.1 * rng.standard_normal((1, 2, 300, 260))).astype(np.float32)
    win = synth.hann_window(128, 12).astype(np.float32)
    ny, nx = (300 - 128) // 64 + 1, (260 - 128) // 64 + 1
    pr2 = synth.make_problem(54, N=128, P=ny * nx, J=2, M=4)
    plan2 = make_plan(pr2, dev)
    Dg = plan2.prepare_data(to_dev(frames, dev), 64, to_dev(win, dev)).cpu().numpy()
    ref = oracle.prepare_data(frames, win, 128, 64)
    assert np.abs(Dg - ref).max() <= 1e-6 * np.abs(ref).max()
    plan2.close()


def test_shared_basis_matches_separate_bases(dev):
    """Channels with the same basis take one contraction for all channels
    (phase formed once, gradient over the channel sum); a plan whose third
    channel's basis differs in the last bits takes the per-channel
    contractions.  Both give the same loss, gradient and OTFs to within
    that perturbation."""
    from paper_2505_10639_amd import Plan

    pr = synth.make_problem(58, N=64, P=3, J=4, M=30, channels=((0, 0.0), (0, 1.0), (1, 0.0)),
                            d_over_r0=np.array([6.0, 10.0, 14.0]))
    D = to_dev(simulate_D(pr), dev)
    a = to_dev(alpha_points(pr, 12)["perturbed"], dev)
    basis2 = pr.basis.copy()
    basis2[2] *= 1.0 + 2.0 ** -20
    shared = make_plan(pr, dev)
    separate = Plan(pr.N, pr.P, pr.J, pr.channel_object, pr.pupil, basis2, pr.diversity, dev)
    l1, g1 = (t.clone() for t in shared.loss_grad(a, D, pr.gamma))
    l2, g2 = separate.loss_grad(a, D, pr.gamma)
    _, S1 = shared.forward(a, want_psf=False)
    _, S2 = separate.forward(a, want_psf=False)
    torch.cuda.synchronize()
    assert float(((l1 - l2).abs() / l2.abs()).max()) < 1e-5
    assert float((g1 - g2).norm() / g2.norm()) < 1e-4
    # channels 0 and 1 share the unperturbed basis in both plans
    s1, s2 = S1.reshape(pr.P, 3, -1), S2.reshape(pr.P, 3, -1)
    assert float((s1[:, :2] - s2[:, :2]).abs().max()) < 1e-6
    assert float((s1[:, 2] - s2[:, 2]).abs().max()) < 1e-4
    shared.close()
    separate.close()


@pytest.mark.parametrize("M", [1, 16, 17, 256])
def test_mode_count_extremes(dev, M):
    """One mode, a whole number of 16-mode tiles, one past it, and the
    largest basis the plan accepts (256 modes: 16 tiles in the gradient
    contraction, a 66 KB coefficient tile in the phase contraction)."""
    pr = synth.make_problem(200 + M, N=64, P=2, J=2, M=M, channels=((0, 0.0), (0, 1.0)),
                            d_over_r0=8.0)
    check_patchwise(pr, simulate_D(pr), alpha_points(pr, M), dev)


def test_many_channels_and_objects(dev):
    """Eight channels: four objects, each seen in focus and with diversity
    (the shared-basis contraction sums eight channels)."""
    ch = tuple((k, d) for k in range(4) for d in (0.0, 1.0))
    pr = synth.make_problem(210, N=64, P=2, J=2, M=20, channels=ch, d_over_r0=9.0)
    check_patchwise(pr, simulate_D(pr), alpha_points(pr, 3), dev)


def test_largest_channel_and_object_count(dev):
    """32 channels, each its own object (the most a plan holds)."""
    ch = tuple((k, 0.0 if k % 2 == 0 else 1.0) for k in range(32))
    pr = synth.make_problem(211, N=64, P=1, J=1, M=8, channels=ch, d_over_r0=9.0)
    check_patchwise(pr, simulate_D(pr), alpha_points(pr, 4), dev)


def test_multi_wavelength_n64(dev):
    pr = synth.make_problem(55, N=64, P=2, J=3, M=36, channels=((0, 0.0), (1, 0.0), (1, 1.0)),
                            lam_ratios=[1.0, 1 / 1.1, 1 / 1.1], d_over_r0=10.0)
    check_patchwise(pr, simulate_D(pr), alpha_points(pr, 7), dev)


# ------------------------------------------------------------ 96 x 96 patches

def test_n96_loss_and_gradient(dev):
    # 96x96 patches (radix-3 transforms), phase diversity, two objects
    pr = synth.make_problem(60, N=96, P=3, J=3, M=40, channels=((0, 0.0), (0, 1.0), (1, 0.0)),
                            d_over_r0=np.array([8.0, 12.0, 16.0]), border=9)
    check_patchwise(pr, simulate_D(pr), alpha_points(pr, 8), dev)


def test_n96_multi_wavelength_and_smoothness(dev):
    lam = [1.0, 1 / 0.95, 1 / 1.1]
    pr = synth.make_problem(61, N=96, P=2, J=2, M=24, channels=((0, 0.0), (1, 0.0), (2, 0.0)),
                            lam_ratios=lam, d_over_r0=12.0, border=9)
    g = oracle.smoothness_gamma(96, [1e-3] * 3, [0.05] * 3)[:, :, :49].astype(np.float32)
    check_patchwise(pr, simulate_D(pr), alpha_points(pr, 9), dev, gamma=g)


def test_n96_forward_object_prepare(dev):
    pr = synth.make_problem(62, N=96, P=2, J=2, M=20, d_over_r0=12.0, border=9)
    plan = make_plan(pr, dev)
    psf, otf = plan.forward(to_dev(pr.alpha_true, dev))
    psf, otf = psf.cpu().numpy(), otf.cpu().numpy()
    for p in range(2):
        for j in range(2):
            phi = oracle.wavefront(pr.alpha_true[p, j], pr.basis[0], pr.diversity[0])
            s = oracle.psf(pr.pupil[0], phi)
            assert np.abs(psf[p, 0, j] - s).max() <= 2e-6 * s.max()
            assert np.abs(otf[p, 0, j] - oracle.otf(s)[:, :49]).max() <= 2e-6
    psf0, _ = plan.forward(torch.zeros((2, 2, 20), device=dev), want_otf=False)
    NA = float(pr.pupil[0].sum())
    assert abs(float(psf0[0, 0, 0, 0, 0]) - NA / 9216) < 1e-6
    D = simulate_D(pr)
    obj = plan.object_estimate(to_dev(pr.alpha_true, dev), to_dev(D, dev), pr.gamma).cpu().numpy()
    ref = oracle.evaluate(pr.alpha_true, D, pr.basis, pr.diversity, pr.pupil, pr.channel_object,
                          pr.gamma, want_grad=False)
    for p in range(2):
        rms = np.sqrt(np.mean((obj[p, 0] - oracle.object_image(ref["O"][p, 0])) ** 2))
        assert rms < OBJ_RMS, rms
    plan.close()
    rng = np.random.default_rng(63)
    frames = (1.0 + 0.1 * rng.standard_normal((1, 2, 250, 200))).astype(np.float32)
    win = synth.hann_window(96, 9).astype(np.float32)
    ny, nx = (250 - 96) // 48 + 1, (200 - 96) // 48 + 1
    pr2 = synth.make_problem(64, N=96, P=ny * nx, J=2, M=4)
    plan2 = make_plan(pr2, dev)
    Dg = plan2.prepare_data(to_dev(frames, dev), 48, to_dev(win, dev)).cpu().numpy()
    ref = oracle.prepare_data(frames, win, 96, 48)
    assert np.abs(Dg - ref).max() <= 1e-6 * np.abs(ref).max()
    plan2.close()
