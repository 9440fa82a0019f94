"""The primal/adjoint pair as a ``torch.autograd.Function``.

forward(w)   -> J: records N primal steps of the library (full states every C
                steps and the moments the adjoint reads for C steps, C sized to
                the workspace budget) and evaluates the objective on the device
                (no host sync).
backward(gJ) -> gJ * dJ/dw: the hand-written adjoint kernel, run N reverse
                steps with segment recomputes from the checkpoints
                (theorem of Section 2.2, unsteady form), then the gradient.
                By default both stream in place and segments are recomputed
                inside their checkpoints.

The context (``Lbm``) holds one recorded trajectory at a time.  Each forward
overwrites it, so the backward of an earlier forward whose trajectory has been
overwritten raises instead of returning another design's gradient.
"""
from __future__ import annotations

import torch

from .lbm import Lbm, lbm_objective_async, lbm_required_bytes, make_config


class LbmObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w: torch.Tensor, solver: "LbmSolver", record: bool):
        L = solver.lbm
        L.set_design(w.detach().reshape(-1))
        L.reset()
        L.primal_steps(solver.nsteps, record=record)
        J = torch.empty(1, dtype=torch.float64, device=L.device)
        lbm_objective_async(L.ctx, J)
        solver._generation += 1
        solver._pending = record
        ctx.generation = solver._generation
        ctx.solver = solver
        ctx.w_shape = w.shape
        ctx.w_dtype = w.dtype
        return J.reshape(())

    @staticmethod
    def backward(ctx, gJ):
        solver = ctx.solver
        L = solver.lbm
        if ctx.generation != solver._generation or not solver._pending:
            raise RuntimeError("LbmObjective.backward: the recorded trajectory of this forward was overwritten "
                               "by a later evaluation on the same solver")
        try:
            L.adjoint_steps(solver.nsteps)
            g = L.gradient()
        finally:
            solver._pending = False
        grad_w = (gJ.to(g.dtype) * g).reshape(ctx.w_shape).to(ctx.w_dtype)
        return grad_w, None, None


def smallest_inplace_interval(params: dict, nsteps: int, precision: str) -> int:
    """Checkpoint interval C whose in-place workspace (ceil(N/C) checkpoint states
    and C moment sets besides the two working states) is smallest."""
    best = None
    for c in range(1, nsteps + 1):
        b = lbm_required_bytes(make_config(params, nsteps, precision, checkpoint_interval=c, inplace=True))
        if best is None or b < best[0]:
            best = (b, c)
    return best[1]


class LbmSolver:
    """Owns one GPU context sized for ``nsteps`` and exposes J(w) as a
    differentiable function: ``J = solver(w); J.backward()``."""

    def __init__(self, params: dict, nsteps: int, precision: str = "fp32", checkpoint_interval: int = 0,
                 hbm_budget_bytes: int = 0, device=None, differentiable: bool = True, inplace: bool = True):
        """differentiable=False sizes the workspace for unrecorded forwards only
        (five states instead of the checkpoint plan); such a solver offers value().
        inplace (default): one primal and one adjoint buffer streamed in place, the
        faster kernels; with neither checkpoint_interval nor hbm_budget_bytes given
        the checkpoint interval is the one with the smallest workspace (about
        sqrt(N Qt / moments per node) steps), as the ping-pong default is."""
        self.nsteps = int(nsteps)
        self.differentiable = differentiable
        n = self.nsteps if differentiable else 0
        if inplace and n > 0 and not checkpoint_interval and not hbm_budget_bytes:
            checkpoint_interval = smallest_inplace_interval(params, n, precision)
        self.lbm = Lbm(params, nsteps=n, precision=precision, checkpoint_interval=checkpoint_interval,
                       hbm_budget_bytes=hbm_budget_bytes, device=device, inplace=inplace)
        self._pending = False  # a recorded trajectory is waiting for its backward
        self._generation = 0   # forwards run so far (a backward must belong to the latest)

    @property
    def dtype(self):
        return self.lbm.dtype

    def __call__(self, w: torch.Tensor) -> torch.Tensor:
        if not self.differentiable:
            raise RuntimeError("LbmSolver built with differentiable=False offers value() only")
        # record the trajectory only when a backward can follow
        record = torch.is_grad_enabled() and w.requires_grad
        return LbmObjective.apply(w, self, record)

    def value(self, w: torch.Tensor) -> float:
        """J(w) only (unrecorded forward, synchronises)."""
        L = self.lbm
        self._generation += 1  # overwrites any recorded trajectory
        self._pending = False
        L.set_design(torch.as_tensor(w).reshape(-1))
        L.reset()
        L.primal_steps(self.nsteps, record=False)
        return L.objective()[0]

    def close(self):
        self.lbm.close()
