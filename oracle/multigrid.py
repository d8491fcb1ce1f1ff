"""Geometric multigrid preconditioner with a DeepONet-Jacobi smoother
(oracle), §4.3 (the multigrid comparison figure: DeepONet-MG-Krylov).

Readings (the paper gives the variant in one paragraph and a figure):

* grids: level 0 is the problem's grid with n_a interior nodes per axis;
  level l + 1 keeps every second node, n' = (n + 1) / 2 - 1, so coarse node j
  sits on fine node 2 j + 1 and h' = 2 h (each n_a + 1 must be divisible by
  2^L for L coarsenings);
* coarse operators are rediscretisations: the coefficient s = k^2 (1 + i alpha)
  and the scatterer mask are injected (coarse node j takes the values of fine
  node 2 j + 1) and the operator of §2 eq. 1 is built on the coarse grid;
* restriction: full weighting, weight prod_a (1/2)^{|d_a|} / 2^dim over the
  3^dim fine neighbours of 2 j + 1, zero on coarse scatterer nodes;
* prolongation: multilinear interpolation from the coarse nodes with zero
  ghosts, zero on fine scatterer nodes; in the interior P = 2^dim R^T;
* smoothing: nu damped Jacobi sweeps (MG), or with a network a - 1 - b:
  a Jacobi sweeps, one trunk-basis correction u += Q A_c^{-1} Q^T (f - A u)
  of that level, b Jacobi sweeps, a + 1 + b = nu (the paper's 2-1-2 for nu = 5);
  the same before and after the coarse-grid correction;
* the coarsest level is solved exactly (LU);
* the preconditioner is one V-cycle started from zero.

TEST INFRASTRUCTURE ONLY, like the rest of this package.
"""
from __future__ import annotations

import numpy as np

from . import operator as op
from .coarse import CoarseSpace


def coarse_n(n):
    return tuple((v + 1) // 2 - 1 for v in n)


def points(n):
    """(N, dim) node coordinates (i + 1) / (n_a + 1), x fastest."""
    axes = [np.arange(1, m + 1) / (m + 1) for m in n]
    grids = np.meshgrid(*reversed(axes), indexing="ij")
    return np.stack([g.ravel() for g in reversed(grids)], axis=1)


def inject(a):
    """Values at coarse nodes: fine index 2 j + 1 on every axis."""
    a = np.asarray(a)
    return a[tuple(slice(1, None, 2) for _ in range(a.ndim))][tuple(slice(0, (m + 1) // 2 - 1) for m in a.shape)]


def restrict(r, mask_c):
    """Full weighting onto the coarse grid, zero on coarse scatterer nodes."""
    r = np.asarray(r)
    dim = r.ndim
    nc = tuple((m + 1) // 2 - 1 for m in r.shape)            # numpy shapes (z, y, x)
    out = np.zeros(nc, dtype=r.dtype)
    for d in np.ndindex(*([3] * dim)):
        off = [x - 1 for x in d]
        w = np.prod([0.5 ** abs(o) for o in off]) / 2 ** dim
        sl = tuple(slice(1 + o, 1 + o + 2 * m - 1, 2) for o, m in zip(off, nc))
        out += w * r[sl]
    out[np.asarray(mask_c).astype(bool)] = 0
    return out


def prolong(e, shape_f, mask_f):
    """Multilinear interpolation to the fine grid (zero coarse ghosts), zero
    on fine scatterer nodes."""
    e = np.asarray(e)
    out = e
    for ax in range(e.ndim):
        m = out.shape[ax]
        nf = shape_f[ax]
        pad = [(0, 0)] * out.ndim
        pad[ax] = (1, 1)
        ep = np.pad(out, pad)                                 # ghosts at -1 and m
        shp = list(out.shape)
        shp[ax] = nf
        res = np.zeros(shp, dtype=out.dtype)
        i = np.arange(nf)
        odd = i % 2 == 1
        # fine i odd -> coarse (i - 1) / 2 ; fine i even -> average of coarse i/2 - 1 and i/2
        idx_odd = (i[odd] - 1) // 2 + 1
        idx_lo = i[~odd] // 2 - 1 + 1
        take = lambda k: np.take(ep, k, axis=ax)
        sl_odd = [slice(None)] * out.ndim
        sl_odd[ax] = np.nonzero(odd)[0]
        sl_even = [slice(None)] * out.ndim
        sl_even[ax] = np.nonzero(~odd)[0]
        res[tuple(sl_odd)] = take(idx_odd)
        res[tuple(sl_even)] = 0.5 * (take(idx_lo) + take(idx_lo + 1))
        out = res
    out = np.array(out)
    out[np.asarray(mask_f).astype(bool)] = 0
    return out


class Hierarchy:
    """Levels of the preconditioner for s (coefficient field) and mask."""

    def __init__(self, s, mask, levels, omega=0.5, nu=5, trunk=None, p_used=32):
        self.omega, self.nu = omega, nu
        self.s = [np.asarray(s, dtype=np.complex128)]
        self.mask = [np.asarray(mask).astype(np.uint8)]
        for _ in range(levels):
            self.s.append(inject(self.s[-1]))
            self.mask.append(inject(self.mask[-1]))
        self.L = levels
        self.coarse = [None] * (levels + 1)
        if trunk is not None:
            from .deeponet import trunk_matrix
            for l in range(levels):
                n = tuple(reversed(self.s[l].shape))
                T = trunk_matrix(points(n), trunk)
                self.coarse[l] = CoarseSpace(T, self.s[l], self.mask[l], min(p_used, int(np.prod(n))))
        self.Ainv_coarsest = np.linalg.inv(op.dense(self.s[-1], self.mask[-1]))

    def smooth(self, l, u, f):
        s, m = self.s[l], self.mask[l]
        cs = self.coarse[l]
        if cs is None:
            for _ in range(self.nu):
                u = op.jacobi_sweep(u, f, s, m, self.omega)
            return u
        a = self.nu // 2
        b = self.nu - a - 1
        for _ in range(a):
            u = op.jacobi_sweep(u, f, s, m, self.omega)
        u = u + cs.m2(op.residual(u, f, s, m))
        for _ in range(b):
            u = op.jacobi_sweep(u, f, s, m, self.omega)
        return u

    def vcycle(self, l, f):
        if l == self.L:
            return (self.Ainv_coarsest @ np.asarray(f).ravel()).reshape(np.shape(f))
        s, m = self.s[l], self.mask[l]
        u = self.smooth(l, np.zeros_like(f), f)
        r = op.residual(u, f, s, m)
        e = self.vcycle(l + 1, restrict(r, self.mask[l + 1]))
        u = u + prolong(e, f.shape, m)
        return self.smooth(l, u, f)

    def precond(self, r):
        """M(r): one V-cycle from zero (flat in, flat out)."""
        shape = self.s[0].shape
        return self.vcycle(0, np.asarray(r).reshape(shape)).ravel()
