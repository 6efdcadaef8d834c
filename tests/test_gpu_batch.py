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
