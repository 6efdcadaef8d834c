"""Uneven batches: fields of different patch sizes, frame, mode and object
counts advanced together from one HIP graph give, bit for bit, what each
field gives with eager solver rounds, and a sampled patch of every field
matches the oracle at the coefficients the rounds accepted."""

import numpy as np
import pytest

import oracle
import synth
from helpers import LOSS_RTOL, assert_grad_close, fast_simulate_D

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [  # N, P, J, M, channels (object, defocus waves)
    (64, 3, 4, 20, ((0, 0.0),)),
    (128, 2, 6, 24, ((0, 0.0), (1, 0.0))),
    (64, 4, 8, 30, ((0, 0.0), (0, 1.0))),
    (128, 1, 3, 16, ((0, 0.0),)),
    (96, 2, 4, 28, ((0, 0.0), (0, 1.0))),
    (64, 2, 5, 44, ((0, 0.0), (1, 1.0), (2, 0.0))),
]


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2505_10639_amd import _lib
    _lib.lib()
    return torch.device("cuda:0")


def make_problems():
    out = []
    for i, (N, P, J, M, ch) in enumerate(SHAPES):
        pr = synth.make_problem(90 + i, N=N, P=P, J=J, M=M, channels=ch,
                                d_over_r0=np.linspace(6.0, 14.0, P))
        out.append((pr, fast_simulate_D(pr)))
    return out


def make_fields(dev, problems):
    from paper_2505_10639_amd.batch import Field
    out = []
    for pr, D_np in problems:
        D = torch.from_numpy(D_np).to(dev)
        out.append(Field(pr.N, pr.P, pr.J, pr.channel_object, pr.pupil, pr.basis,
                         pr.diversity, D, pr.gamma, device=dev))
    return out


def test_uneven_fields_in_one_graph(dev):
    from paper_2505_10639_amd.batch import FieldBatch
    problems = make_problems()
    eager = FieldBatch(make_fields(dev, problems), rounds_per_launch=3)
    ref = []
    for _ in range(3):
        eager.eager()
        torch.cuda.synchronize()
        ref.append([(f.accepted.clone(), f.solver.loss.clone()) for f in eager.fields])
    graph = FieldBatch(make_fields(dev, problems), rounds_per_launch=3)
    graph.capture()
    for k in range(3):
        graph.launch()
        torch.cuda.synchronize()
        for f, (a, l) in zip(graph.fields, ref[k]):
            assert torch.equal(f.accepted, a) and torch.equal(f.solver.loss, l)
    # the loss went down in every field
    for f, (_, l0) in zip(graph.fields, ref[0]):
        assert bool((f.solver.loss <= l0).all())
    # one sampled patch per field against the oracle, at its accepted point:
    # the loss the solver reports and the gradient there
    for i, (f, (pr, D_np)) in enumerate(zip(graph.fields, problems)):
        p = (3 * i + 1) % pr.P
        a = f.accepted.cpu().numpy()
        print(f"[batch] field {i} N={pr.N} J={pr.J} M={pr.M} C={pr.C} patch {p}", flush=True)
        loss, grad = f.plan.loss_grad(f.accepted, f.D, pr.gamma)
        torch.cuda.synchronize()
        ref = oracle.evaluate(a, D_np, pr.basis, pr.diversity, pr.pupil, pr.channel_object,
                              pr.gamma, patches=[p])
        rep = float(f.solver.loss[p])
        assert abs(rep - ref["loss"][0]) < LOSS_RTOL * abs(ref["loss"][0]), (i, rep)
        assert abs(float(loss[p]) - ref["loss"][0]) < LOSS_RTOL * abs(ref["loss"][0])
        assert_grad_close(grad.cpu().numpy()[[p]], ref["grad"], f"field {i}")
    eager.close()
    graph.close()


def _set_alpha(fields, problems, seed):
    rng = np.random.default_rng(seed)
    for f, (pr, _) in zip(fields, problems):
        a = (pr.alpha_true + 0.3 * rng.standard_normal(pr.alpha_true.shape)).astype(np.float32)
        f.alpha.copy_(torch.from_numpy(a))


def test_group_evaluation_equals_each_plan(dev):
    """One launch per stage over every field of a patch size gives each
    field's loss and gradient bit for bit as its own plan does (same
    gradient splits), and they match the oracle on a sampled patch."""
    from paper_2505_10639_amd.batch import FieldGroup
    problems = make_problems()
    fields = make_fields(dev, problems)
    _set_alpha(fields, problems, 5)
    groups = {}
    for f in fields:
        groups.setdefault(f.plan.N, []).append(f)
    for N, fs in sorted(groups.items()):
        g = FieldGroup(fs)
        from paper_2505_10639_amd import _lib
        _lib.momfbd_group_set_tuning(g.handle, 0, 1, grad_splits=1, grad_row_tiles=4)
        print(f"[group] N={N}: {len(fs)} fields", flush=True)
        g.loss_grad()
        torch.cuda.synchronize()
        for f in fs:
            f.plan.set_tuning(0, 1, 1, 4, 1)
            loss, grad = f.plan.loss_grad(f.alpha, f.D, f.gamma)
            torch.cuda.synchronize()
            assert torch.equal(f.loss_eval, loss), (N, (f.loss_eval - loss).abs().max())
            assert torch.equal(f.grad_eval, grad), (N, (f.grad_eval - grad).abs().max())
        # another schedule of the group: same losses, gradients to rounding
        _lib.momfbd_group_set_tuning(g.handle, 1, 0, grad_splits=4, grad_row_tiles=3)
        ref = [(f.loss_eval.clone(), f.grad_eval.clone()) for f in fs]
        g.loss_grad()
        torch.cuda.synchronize()
        for f, (l0, g0) in zip(fs, ref):
            assert torch.equal(f.loss_eval, l0)
            assert float((f.grad_eval - g0).abs().max()) <= 1e-5 * float(g0.abs().max())
        g.close()
    for i, (f, (pr, D_np)) in enumerate(zip(fields, problems)):
        p = (2 * i + 1) % pr.P
        ref = oracle.evaluate(f.alpha.cpu().numpy(), D_np, pr.basis, pr.diversity, pr.pupil,
                              pr.channel_object, pr.gamma, patches=[p])
        assert abs(float(f.loss_eval[p]) - ref["loss"][0]) < LOSS_RTOL * abs(ref["loss"][0])
        assert_grad_close(f.grad_eval.cpu().numpy()[[p]], ref["grad"], f"group field {i}")
    for f in fields:
        f.close()


def test_group_wide_mode_counts(dev):
    """Fields of up to 200 modes (13 tiles of 16): the group's default row
    tiles per wave drop to 3, so that the accumulators fit the registers,
    and its loss and gradient are still each field's own plan's bit for bit
    (same gradient splits), and the oracle's on a sampled patch."""
    from paper_2505_10639_amd import _lib
    from paper_2505_10639_amd.batch import FieldGroup
    problems = []
    for i, M in enumerate((200, 180)):
        pr = synth.make_problem(130 + i, N=64, P=2, J=2, M=M, channels=((0, 0.0),),
                                d_over_r0=np.array([6.0, 9.0]))
        problems.append((pr, fast_simulate_D(pr)))
    fields = make_fields(dev, problems)
    _set_alpha(fields, problems, 7)
    g = FieldGroup(fields)
    assert _lib.momfbd_group_get_tuning(g.handle)["grad_row_tiles"] == 3
    _lib.momfbd_group_set_tuning(g.handle, 0, 1, grad_splits=1, grad_row_tiles=0)
    assert _lib.momfbd_group_get_tuning(g.handle)["grad_row_tiles"] == 3
    g.loss_grad()
    torch.cuda.synchronize()
    for i, (f, (pr, D_np)) in enumerate(zip(fields, problems)):
        f.plan.set_tuning(0, 1, 1, 4, 1)
        loss, grad = f.plan.loss_grad(f.alpha, f.D, f.gamma)
        torch.cuda.synchronize()
        assert torch.equal(f.loss_eval, loss) and torch.equal(f.grad_eval, grad), i
        ref = oracle.evaluate(f.alpha.cpu().numpy(), D_np, pr.basis, pr.diversity, pr.pupil,
                              pr.channel_object, pr.gamma, patches=[i])
        assert abs(float(f.loss_eval[i]) - ref["loss"][0]) < LOSS_RTOL * abs(ref["loss"][0])
        assert_grad_close(f.grad_eval.cpu().numpy()[[i]], ref["grad"], f"wide field {i}")
    g.close()
    for f in fields:
        f.close()


def test_group_rounds_equal_field_rounds_and_replay_from_a_graph(dev):
    """Solver rounds of a group (one launch per stage per patch size) follow
    each field's own solver rounds bit for bit, eagerly and replayed from a
    HIP graph; sampled patches match the oracle at the accepted point."""
    from paper_2505_10639_amd import _lib
    from paper_2505_10639_amd.batch import FieldBatch
    problems = make_problems()
    per_field = FieldBatch(make_fields(dev, problems), rounds_per_launch=3, mode="branches")
    for f in per_field.fields:
        f.plan.set_tuning(0, 1, 1, 4, 1)
    ref = []
    for _ in range(3):
        per_field.eager()
        torch.cuda.synchronize()
        ref.append([(f.accepted.clone(), f.solver.loss.clone(), f.solver.status.clone())
                    for f in per_field.fields])
    for mode_graph in (False, True):
        grouped = FieldBatch(make_fields(dev, problems), rounds_per_launch=3, mode="group")
        for g in grouped.groups:
            _lib.momfbd_group_set_tuning(g.handle, 0, 1, grad_splits=1, grad_row_tiles=4)
        if mode_graph:
            grouped.capture()
        for k in range(3):
            print(f"[group rounds] graph={mode_graph} launch {k}", flush=True)
            grouped.launch() if mode_graph else grouped.eager()
            torch.cuda.synchronize()
            for i, (f, (a, l, s)) in enumerate(zip(grouped.fields, ref[k])):
                assert torch.equal(f.accepted, a), (mode_graph, k, i)
                assert torch.equal(f.solver.loss, l), (mode_graph, k, i)
                assert torch.equal(f.solver.status, s), (mode_graph, k, i)
        if mode_graph:
            for i, (f, (pr, D_np)) in enumerate(zip(grouped.fields, problems)):
                p = i % pr.P
                r = oracle.evaluate(f.accepted.cpu().numpy(), D_np, pr.basis, pr.diversity,
                                    pr.pupil, pr.channel_object, pr.gamma, patches=[p])
                assert abs(float(f.solver.loss[p]) - r["loss"][0]) < LOSS_RTOL * abs(r["loss"][0])
        grouped.close()
    per_field.close()
