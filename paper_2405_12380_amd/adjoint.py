"""Differentiable Helmholtz solve for k^2 inversion (§2 eq. 1 differentiated).

``HelmholtzSolve`` maps (k^2, f) to u = A(k^2)^{-1} f with the meta-solver
and differentiates by the adjoint state: for a loss L(u) with PyTorch's
gradient g = dL/du (real and imaginary parts), A^H lam = g gives

    dL/dk^2_p = Re(conj(lam_p) (1 + i alpha_p) u_p)   (0 on the scatterer),
    dL/df     = lam.

``ReceiverMisfit`` is L = 1/2 ||P u - d||^2 on one grid plane, with P^T (P u - d)
as its gradient.  Every step runs in libhelm's kernels (the forward and
adjoint meta-solves, the misfit and the pointwise gradient); torch holds the
device memory.
"""
from __future__ import annotations

import torch

from . import helm


class Solver:
    """An op, an optional network and the meta-solver options of ``helm.meta_solve``.

    ``strict`` makes a non-converged solve raise instead of returning its last
    iterate."""

    def __init__(self, op: helm.Op, net: helm.DeepONet | None = None, strict: bool = True, **opts):
        self.op = op
        self.net = net
        self.opts = dict(kind="gmres", restart=50, tol=1e-8, max_iters=20000, n_r=3, omega=0.5)
        if net is not None:
            self.opts["p_used"] = net.p
        self.opts.update(opts)
        self.strict = strict
        self.stats = []
        self._ksq = None
        self._ksq_version = None

    def use_ksq(self, ksq: torch.Tensor):
        """Load k^2 into the op unless this very tensor (same version) is loaded."""
        if self._ksq is not ksq or self._ksq_version != ksq._version:
            self.op.set_ksq(ksq.detach())
            self._ksq, self._ksq_version = ksq, ksq._version

    def solve(self, rhs, adjoint=False):
        x = self.op.field()
        s, st = helm.meta_solve(self.op, self.net, rhs.contiguous(), x, adjoint=adjoint, **self.opts)
        st["adjoint"] = adjoint
        self.stats.append(st)
        if self.strict and s != helm.OK:
            raise RuntimeError(f"{'adjoint ' if adjoint else ''}meta-solve did not converge: {st}")
        return x


class HelmholtzSolve(torch.autograd.Function):
    """u = A(k^2)^{-1} f; backward by one adjoint meta-solve."""

    @staticmethod
    def forward(ctx, ksq: torch.Tensor, f: torch.Tensor, solver: Solver):
        solver.use_ksq(ksq)
        u = solver.solve(f)
        ctx.solver = solver
        ctx.save_for_backward(ksq, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        ksq, u = ctx.saved_tensors
        solver = ctx.solver
        solver.use_ksq(ksq)
        lam = solver.solve(grad_u.to(u.dtype), adjoint=True)
        g_ksq = solver.op.ksq_gradient(u, lam).to(ksq.dtype) if ctx.needs_input_grad[0] else None
        g_f = lam if ctx.needs_input_grad[1] else None
        return g_ksq, g_f, None


class ReceiverMisfit(torch.autograd.Function):
    """L = 1/2 ||P u - d||^2 on the plane {i_axis = index} (float64 scalar)."""

    @staticmethod
    def forward(ctx, u: torch.Tensor, d: torch.Tensor, op: helm.Op, axis: int, index: int):
        loss, g = op.misfit(axis, index, u.contiguous(), d.contiguous())
        ctx.save_for_backward(g)
        return torch.tensor(loss, dtype=torch.float64, device=u.device)

    @staticmethod
    def backward(ctx, grad_loss):
        (g,) = ctx.saved_tensors
        return g * grad_loss.to(g.real.dtype), None, None, None, None


def solve(ksq, f, solver: Solver):
    return HelmholtzSolve.apply(ksq, f, solver)


def misfit(u, d, op: helm.Op, axis: int, index: int):
    return ReceiverMisfit.apply(u, d, op, axis, index)
