"""Uneven batches: many independent fields with different patch sizes, frame
counts, mode counts and object counts solved together.

Every field keeps its own plan (tables sized for its shape) and per-patch
L-BFGS state; the solver rounds of all fields (momfbd_lbfgs_rounds, which
needs no host read-back) are captured once into one HIP graph, so a single
graph launch advances every patch of every field by the same number of
line-search trials.  The fields are captured as parallel branches (forked
over a few streams of default priority and joined at the end), so the
kernels of small fields can run beside each other.  The patches of all
fields are independent (Sect. "Optimization and paralellization"), so each
field's result is the one it would reach alone.
"""

from __future__ import annotations

import torch

from .plan import Plan, Solver


class Field:
    """One field: its plan, data, coefficients and solver."""

    def __init__(self, N, P, J, channel_object, pupil, basis, diversity, D, gamma=1e-3,
                 weights=None, alpha0=None, device="cuda:0", m=10, max_evals=20, ftol=0.0):
        self.plan = Plan(N, P, J, channel_object, pupil, basis, diversity, device)
        self.D = D
        self.gamma = gamma
        self.alpha = (torch.zeros((P, J, self.plan.M), dtype=torch.float32, device=device)
                      if alpha0 is None else alpha0.clone().contiguous())
        self.accepted = torch.empty_like(self.alpha)
        self.solver = Solver(self.plan, self.alpha, D, gamma, weights, m=m,
                             max_evals=max_evals, ftol=ftol)

    def close(self):
        self.plan.close()


class FieldBatch:
    """Solver rounds of several fields replayed from one HIP graph."""

    def __init__(self, fields, rounds_per_launch=1, branches=4):
        self.fields = list(fields)
        self.rounds = int(rounds_per_launch)
        self.branches = max(1, int(branches))
        self.graph = None
        self.streams = None

    def eager(self):
        for f in self.fields:
            f.solver.rounds(self.rounds, f.accepted)

    def _issue_branches(self):
        main = torch.cuda.current_stream()
        for s in self.streams:
            s.wait_stream(main)
        for i, f in enumerate(self.fields):
            with torch.cuda.stream(self.streams[i % len(self.streams)]):
                f.solver.rounds(self.rounds, f.accepted)
        for s in self.streams:
            main.wait_stream(s)

    def capture(self):
        torch.cuda.synchronize()
        if self.streams is None:
            self.streams = [torch.cuda.Stream() for _ in range(self.branches)]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._issue_branches()
        self.graph = g
        return g

    def launch(self, n=1):
        if self.graph is None:
            self.capture()
        for _ in range(n):
            self.graph.replay()

    def losses(self):
        return [f.solver.loss for f in self.fields]

    def close(self):
        self.graph = None
        for f in self.fields:
            f.close()
