"""Meta-solvers (oracle): eq. 3 of §3.1.1 and the Krylov variant of §3.1.2.

Relaxation meta-solver (eq. 3): a cycle is M1 = ``n_r`` relaxation sweeps
(damped Jacobi or red-black Gauss-Seidel) followed by M2 = one DeepONet
correction computed from the residual after the sweeps.  Reading: the
network is applied after sweeps n_r, 2 n_r, ...; the relative residual is
checked after every correction (or every n_r sweeps without a network);
the count is in sweeps.

Krylov preconditioner (§3.1.2 with App. C): M(r) is eq. 3 started from
z = 0 on A z = r, i.e. ``n_r`` smoother sweeps, then the residual
r1 = r - A z and z <- z + M2 r1 with the linear trunk-basis M2.  Because the
sweep count is fixed and M2 is linear, M is a fixed linear operator and is
used as a right preconditioner.
"""
from __future__ import annotations

import numpy as np

from . import operator as op
from . import krylov
from . import deeponet as don
from .coarse import CoarseSpace

JACOBI, RBGS = "jacobi", "rbgs"


def sweep(kind, u, f, s, mask, omega):
    if kind == JACOBI:
        return op.jacobi_sweep(u, f, s, mask, omega)
    if kind == RBGS:
        return op.rbgs_sweep(u, f, s, mask, omega)
    raise ValueError(kind)


def relaxation_meta(f, u0, s, mask, kind, omega, max_sweeps, nn_every, tol, correction=None,
                    history=None, fallback_restart=0, gs_passes=2):
    """eq. 3 with M1 = nn_every sweeps and M2 = ``correction(r)`` (or none).

    Krylov fallback (reading: the paper observes plain relaxation diverging on
    the cube scatterer, §4.1, and keeps Krylov solvers as the reference
    method): with ``fallback_restart = m >= 1``, a cycle that ends with a
    relative residual larger than the one before it (that of u0 for the first
    cycle) or not finite is undone, and standalone GMRES(m) runs from the
    iterate before it, to ``tol`` within ``max_sweeps`` Arnoldi steps
    (``gs_passes`` classical Gram-Schmidt passes per step).

    Returns (u, info); info["fallback_iters"] counts the fallback's steps."""
    u = np.array(u0, dtype=np.complex128)
    fn = np.linalg.norm(f)
    fs = fn if fn > 0 else 1.0  # residual scale (absolute residual when f = 0)
    count = 0
    ncorr = 0
    status = krylov.NOT_CONVERGED
    prev = np.linalg.norm(op.residual(u, f, s, mask)) / fs
    keep = u
    diverged = False
    while count < max_sweeps:
        cyc = min(nn_every, max_sweeps - count) if nn_every > 0 else max_sweeps - count
        for _ in range(cyc):
            u = sweep(kind, u, f, s, mask, omega)
            count += 1
        r = op.residual(u, f, s, mask)
        if correction is not None and nn_every > 0 and cyc == nn_every:
            u = u + correction(r)
            ncorr += 1
            r = op.residual(u, f, s, mask)
        rel = np.linalg.norm(r) / fs
        if history is not None:
            history.append(rel)
        if fallback_restart > 0 and not rel <= prev:
            diverged = True
            break
        if not np.isfinite(rel):
            status = krylov.NONFINITE
            break
        if rel <= tol:
            status = krylov.CONVERGED
            break
        keep, prev = u, rel
    fb_iters = 0
    if diverged:
        shape = np.shape(f)
        u, info = krylov.gmres(lambda v: op.apply(v.reshape(shape), s, mask).ravel(), np.ravel(f),
                               np.ravel(keep), fallback_restart, tol, max_sweeps, gs_passes=gs_passes)
        u = u.reshape(shape)
        status, fb_iters = info["status"], info["iters"]
    rel = np.linalg.norm(op.residual(u, f, s, mask)) / fs
    return u, dict(status=status, iters=count, rel_res=rel, corrections=ncorr, fallback_iters=fb_iters)


def deeponet_correction(s_field, mask, T, net):
    """M2 of eq. 3: the DeepONet acting on the residual."""
    def corr(r):
        return don.infer(r, mask, T, net["branch"], net["head"], net["p"], net["branch_grid"],
                         k=net.get("k"), k_input=net.get("k_input", False), act=net.get("act", "tanh"))
    return corr


def krylov_preconditioner(s, mask, smoother, n_r, omega, coarse: CoarseSpace | None):
    """M(r): n_r sweeps from zero, then the coarse correction of the residual."""
    shape = np.shape(s)

    def M(v):
        r = v.reshape(shape)
        z = np.zeros(shape, dtype=np.complex128)
        for _ in range(n_r):
            z = sweep(smoother, z, r, s, mask, omega)
        if coarse is not None:
            r1 = r - op.apply(z, s, mask)
            z = z + coarse.m2(r1)
        return z.ravel()
    return M


def krylov_meta(kind, f, u0, s, mask, restart, tol, max_iters, precond=None, history=None, gs_passes=2):
    """GMRES(m) or BiCGStab on A u = f, right-preconditioned by ``precond``
    (``gs_passes``: GMRES's classical Gram-Schmidt passes, 1 or 2)."""
    shape = np.shape(f)

    def A(v):
        return op.apply(v.reshape(shape), s, mask).ravel()
    ff = np.asarray(f, dtype=np.complex128).ravel()
    u0f = np.asarray(u0, dtype=np.complex128).ravel()
    if kind == "gmres":
        u, info = krylov.gmres(A, ff, u0f, restart, tol, max_iters, M=precond, history=history,
                               gs_passes=gs_passes)
    elif kind == "bicgstab":
        u, info = krylov.bicgstab(A, ff, u0f, tol, max_iters, M=precond, history=history)
    else:
        raise ValueError(kind)
    return u.reshape(shape), info
