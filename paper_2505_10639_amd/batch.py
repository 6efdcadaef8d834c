"""Uneven batches: many independent fields with different patch sizes, frame
counts, mode counts and object counts solved together.

Every field keeps its own plan (tables sized for its shape), workspace and
per-patch L-BFGS state.  Two ways to advance them all:

* ``mode="group"`` (default): the fields of each patch size form one
  library group (momfbd_group_*), whose solver rounds issue one kernel launch
  per stage for every patch of every field of that size; the size classes
  run as parallel branches of one HIP graph.
* ``mode="branches"``: each field issues its own solver rounds
  (momfbd_lbfgs_rounds), the fields spread over a few streams as parallel
  branches of one HIP graph.

The patches of all fields are independent (Sect. "Optimization and
paralellization"), so each field's result is the one it reaches alone, bit
for bit, either way.
"""

from __future__ import annotations

import torch

from . import _lib
from .plan import Plan, Solver


class Field:
    """One field: its plan, data, coefficients and solver."""

    def __init__(self, N, P, J, channel_object, pupil, basis, diversity, D, gamma=1e-3,
                 weights=None, alpha0=None, device="cuda:0", m=10, max_evals=20, ftol=0.0):
        self.plan = Plan(N, P, J, channel_object, pupil, basis, diversity, device)
        self.D = D
        self.gamma = gamma
        self.weights = weights
        self.alpha = (torch.zeros((P, J, self.plan.M), dtype=torch.float32, device=device)
                      if alpha0 is None else alpha0.clone().contiguous())
        self.accepted = torch.empty_like(self.alpha)
        self.solver = Solver(self.plan, self.alpha, D, gamma, weights, m=m,
                             max_evals=max_evals, ftol=ftol)
        # outputs of a group evaluation
        self.loss_eval = torch.empty(P, dtype=torch.float64, device=device)
        self.grad_eval = torch.empty_like(self.alpha)

    def spec(self):
        """This field's momfbd_field for a group."""
        g_arr, g_sc = self.plan._gamma(self.gamma)
        return _lib.field_spec(self.plan.handle, self.alpha, self.D, g_arr, g_sc, self.weights,
                               self.plan.ws, self.solver.state, self.loss_eval, self.grad_eval,
                               self.solver.loss, self.solver.status, self.accepted)

    def close(self):
        self.plan.close()


class FieldGroup:
    """Fields of one patch size advanced with one launch per stage."""

    def __init__(self, fields):
        self.fields = list(fields)
        if len({f.plan.N for f in self.fields}) != 1:
            raise ValueError("a group holds fields of one patch size")
        self.N = self.fields[0].plan.N
        self.device = self.fields[0].plan.device
        params = self.fields[0].solver.params
        with torch.cuda.device(self.device):
            self.handle = _lib.momfbd_group_create([f.spec() for f in self.fields], params)

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def rounds(self, n):
        _lib.momfbd_group_lbfgs_rounds(self.handle, n, self._stream())

    def loss_grad(self):
        """Loss and gradient of every field at its alpha, into each field's
        loss_eval and grad_eval."""
        _lib.momfbd_group_loss_grad(self.handle, self._stream())

    def autotune(self, reps=3):
        with torch.cuda.device(self.device):
            return _lib.momfbd_group_autotune(self.handle, reps, self._stream())

    def tuning(self):
        return _lib.momfbd_group_get_tuning(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            _lib.momfbd_group_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FieldBatch:
    """Solver rounds of many fields, eagerly or replayed from one HIP graph."""

    def __init__(self, fields, rounds_per_launch=1, branches=4, mode="group",
                 parallel_sizes=True):
        if mode not in ("group", "branches"):
            raise ValueError("mode is 'group' or 'branches'")
        self.fields = list(fields)
        self.rounds = int(rounds_per_launch)
        self.mode = mode
        self.graph = None
        self.streams = None
        if mode == "group":
            by_n = {}
            for f in self.fields:
                by_n.setdefault(f.plan.N, []).append(f)
            # largest patch size first: its kernels need the most LDS per
            # workgroup and are the last to find room beside the others
            self.groups = [FieldGroup(by_n[n]) for n in sorted(by_n, reverse=True)]
            self.branches = len(self.groups) if parallel_sizes else 1
        else:
            self.groups = []
            self.branches = max(1, int(branches))

    def _units(self):
        return self.groups if self.mode == "group" else self.fields

    def _issue(self, unit):
        if self.mode == "group":
            unit.rounds(self.rounds)
        else:
            unit.solver.rounds(self.rounds, unit.accepted)

    def eager(self):
        for u in self._units():
            self._issue(u)

    def autotune(self, reps=3):
        """Autotune every group's launch schedules (group mode)."""
        return [g.autotune(reps) for g in self.groups]

    def _issue_branches(self):
        main = torch.cuda.current_stream()
        for s in self.streams:
            s.wait_stream(main)
        for i, u in enumerate(self._units()):
            with torch.cuda.stream(self.streams[i % len(self.streams)]):
                self._issue(u)
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
        for g in self.groups:
            g.close()
        for f in self.fields:
            f.close()
