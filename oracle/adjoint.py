"""Adjoint gradient of a receiver misfit with respect to k^2 (oracle).

The scattering problem of §2 (eq. 1) maps the wave-number field to the
wave field: A(k^2) u = f.  With receivers on one grid plane (the observation
operator P picks the plane's nodes) and data d, the misfit is

    L(k^2) = 1/2 || P u - d ||_2^2 .

Differentiating A u = f at an unmasked node p, where the only entry of A
that depends on k^2_p is the diagonal -k^2_p (1 + i alpha_p), gives
A du = (1 + i alpha_p) u_p e_p dk^2_p, so

    dL/dk^2_p = Re( conj(lam_p) (1 + i alpha_p) u_p ),   A^H lam = P^T (P u - d),

and 0 on masked nodes (their rows are the identity and carry no k^2).  A^H
is the conjugate transpose of the assembled matrix; no property of A (such
as its complex symmetry) is used here.  Solves use a sparse LU of the
matrix assembled node by node from the definition (a library factorisation
as one step).

Readings: the plane wave enters as a sheet source on a grid plane (the
paper's incident Neumann data on the top face); nodes of the receiver plane
that lie in the scatterer observe u = 0 and their misfit does not depend on
k^2.

TEST INFRASTRUCTURE ONLY, like the rest of this package.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def sparse(s, mask) -> sp.csc_matrix:
    """A (§2 eq. 1, Dirichlet nodes eliminated as in App. D) as a sparse
    matrix built from the definition: an unmasked row p has sum_a 2/h_a^2 - s_p
    on the diagonal and -1/h_a^2 for every unmasked interior neighbour; a
    masked row is the identity row."""
    shape = np.shape(s)
    dim = len(shape)
    n = list(reversed(shape))
    N = int(np.prod(shape))
    sf = np.asarray(s, dtype=np.complex128).ravel()
    mf = np.asarray(mask).astype(bool).ravel()
    idx = np.unravel_index(np.arange(N), shape)          # numpy axes: z, y, x
    rows, cols, vals = [], [], []
    diag = np.zeros(N, dtype=np.complex128)
    strides = [1]
    for a in range(1, dim):
        strides.append(strides[-1] * n[a - 1])
    for a in range(dim):
        w = float(n[a] + 1) ** 2                         # 1 / h_a^2
        diag += 2.0 * w
        ia = idx[dim - 1 - a]
        for step in (-1, 1):
            ok = (ia + step >= 0) & (ia + step < n[a])
            p = np.nonzero(ok)[0]
            q = p + step * strides[a]
            keep = ~mf[p] & ~mf[q]
            rows.append(p[keep])
            cols.append(q[keep])
            vals.append(np.full(int(keep.sum()), -w, dtype=np.complex128))
    diag = diag - sf
    diag[mf] = 1.0
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return A.tocsc()


def solve(s, mask, f) -> np.ndarray:
    """u = A^{-1} f (sparse LU)."""
    A = sparse(s, mask)
    return spla.splu(A).solve(np.asarray(f, dtype=np.complex128).ravel()).reshape(np.shape(f))


def adjoint_solve(s, mask, g) -> np.ndarray:
    """lam = A^{-H} g: the conjugate-transpose system, factored as such."""
    AH = sparse(s, mask).conj().T.tocsc()
    return spla.splu(AH).solve(np.asarray(g, dtype=np.complex128).ravel()).reshape(np.shape(g))


def plane_index(n_axis: int, x: float) -> int:
    """Index of the grid plane nearest coordinate x on an axis with n_axis
    interior nodes at (i + 1) / (n_axis + 1)."""
    return int(min(max(round(x * (n_axis + 1)) - 1, 0), n_axis - 1))


def observe(u, axis: int, index: int) -> np.ndarray:
    """P u: the values on the plane {i_axis = index}; grid axis a is numpy
    axis dim - 1 - a, so the result keeps the remaining axes in x-fastest
    order."""
    u = np.asarray(u)
    return np.take(u, index, axis=u.ndim - 1 - axis)


def misfit(u, d, axis: int, index: int, mask):
    """L = 1/2 ||P u - d||^2 and g = P^T (P u - d) with g zeroed on masked
    nodes (u is identically 0 there, so L does not depend on them)."""
    u = np.asarray(u, dtype=np.complex128)
    r = observe(u, axis, index) - np.asarray(d, dtype=np.complex128)
    L = 0.5 * float(np.sum(np.abs(r) ** 2))
    g = np.zeros_like(u)
    sl = [slice(None)] * u.ndim
    sl[u.ndim - 1 - axis] = index
    g[tuple(sl)] = r
    g[np.asarray(mask).astype(bool)] = 0.0
    return L, g


def ksq_gradient(lam, u, alpha, mask) -> np.ndarray:
    """dL/dk^2_p = Re(conj(lam_p) (1 + i alpha_p) u_p), 0 on masked nodes."""
    gr = np.real(np.conj(lam) * (1.0 + 1j * np.asarray(alpha, dtype=np.float64)) * u)
    return np.where(np.asarray(mask).astype(bool), 0.0, gr)


def loss_and_gradient(ksq, alpha, mask, f, d, axis: int, index: int):
    """Forward solve, misfit, adjoint solve and gradient.  Returns
    (L, dL/dk^2, u, lam).  One sparse LU of A serves both solves: the
    adjoint one is its conjugate-transpose solve (pinned against
    ``adjoint_solve``, which factors A^H itself)."""
    s = np.asarray(ksq, dtype=np.float64) * (1.0 + 1j * np.asarray(alpha, dtype=np.float64))
    lu = spla.splu(sparse(s, mask))
    u = lu.solve(np.asarray(f, dtype=np.complex128).ravel()).reshape(np.shape(f))
    L, g = misfit(u, d, axis, index, mask)
    lam = lu.solve(g.ravel(), trans="H").reshape(np.shape(f))
    return L, ksq_gradient(lam, u, alpha, mask), u, lam


def loss(ksq, alpha, mask, f, d, axis: int, index: int) -> float:
    """L(k^2) alone (forward solve and misfit), for finite differences."""
    s = np.asarray(ksq, dtype=np.float64) * (1.0 + 1j * np.asarray(alpha, dtype=np.float64))
    return misfit(solve(s, mask, f), d, axis, index, mask)[0]
