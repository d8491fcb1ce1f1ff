"""Discrete Helmholtz operator and the point relaxations (oracle).

Problem (§2, eq. 1) in the finite-difference form used here:

    -Delta_h u - k^2 (1 + i alpha) u = f    on unmasked nodes,
    u = 0                                   on scatterer (masked) nodes.

Reading of the paper for this discretisation (the paper uses FEM with
Sommerfeld boundaries; the grid form below replaces it):

* interior nodes x_i = (i+1) h, h = 1/(n+1); ghost nodes behind the sponge
  carry u = 0;
* the Dirichlet scatterer is eliminated symmetrically: a masked row is the
  identity row, and masked neighbours of an unmasked node contribute 0
  (App. D shows the residual of such rows vanishes);
* per node the axis differences are summed in the order x-, x+, y-, y+, z-,
  z+, each axis scaled by 1/h_a^2, then s_p x_p is subtracted, where
  s = k^2 (1 + i alpha).

Fields are numpy arrays of shape (nz, ny, nx) / (ny, nx); numpy axis
``dim - 1 - a`` is grid axis ``a`` (a = 0 is x).
"""
from __future__ import annotations

import numpy as np


def spacing(shape) -> list:
    """h_a for grid axes a = 0 (x), 1 (y), 2 (z) of a field of numpy shape."""
    n = list(reversed(shape))
    return [1.0 / (na + 1) for na in n]


def coefficient(ksq, alpha) -> np.ndarray:
    """s = k^2 (1 + i alpha) (§2, eq. 1 with the sponge damping)."""
    return np.asarray(ksq, dtype=np.float64) * (1.0 + 1j * np.asarray(alpha, dtype=np.float64))


def _shift(x, axis, step):
    """x_{p - step e_axis} with zero ghosts: result[p] = x[p - step]."""
    y = np.zeros_like(x)
    src = [slice(None)] * x.ndim
    dst = [slice(None)] * x.ndim
    if step > 0:
        dst[axis] = slice(step, None)
        src[axis] = slice(None, -step)
    else:
        dst[axis] = slice(None, step)
        src[axis] = slice(-step, None)
    y[tuple(dst)] = x[tuple(src)]
    return y


def apply(x, s, mask) -> np.ndarray:
    """y = A x for the masked Helmholtz operator (§2, eq. 1; App. D)."""
    x = np.asarray(x, dtype=np.complex128)
    m = np.asarray(mask).astype(bool)
    xn = np.where(m, 0.0, x)                 # masked neighbours count as zero
    h = spacing(x.shape)
    acc = np.zeros_like(x)
    for a in range(x.ndim):
        ax = x.ndim - 1 - a
        minus = _shift(xn, ax, 1)            # x_{p - e_a}
        plus = _shift(xn, ax, -1)            # x_{p + e_a}
        acc = acc + ((x - minus) + (x - plus)) * (1.0 / h[a] ** 2)
    y = acc - s * x
    return np.where(m, x, y)


def diagonal(s, mask) -> np.ndarray:
    """D_p = sum_a 2/h_a^2 - s_p on unmasked nodes, 1 on masked ones."""
    h = spacing(np.shape(s))
    d = sum(2.0 / ha ** 2 for ha in h) - s
    return np.where(np.asarray(mask).astype(bool), 1.0 + 0j, d)


def residual(u, f, s, mask) -> np.ndarray:
    """r = f - A u (eq. 2)."""
    return np.asarray(f, dtype=np.complex128) - apply(u, s, mask)


def jacobi_sweep(u, f, s, mask, omega) -> np.ndarray:
    """One damped Jacobi step u + omega D^{-1} (f - A u): eq. 2 with M taken
    from the diagonal of A (§3.1.1)."""
    return u + omega * residual(u, f, s, mask) / diagonal(s, mask)


def colour(shape) -> np.ndarray:
    """(i + j + l) mod 2 of every node; 0 is 'red' and is updated first."""
    idx = np.indices(shape)
    return (sum(idx) % 2).astype(np.int8)


def rbgs_sweep(u, f, s, mask, omega) -> np.ndarray:
    """One red-black Gauss-Seidel (SOR for omega != 1) sweep: eq. 2 with M
    from the lower-triangular part of A (§3.1.1) in red-then-black order.
    Nodes of one colour are coupled only to the other colour, so each
    colour's update uses the current values of the other."""
    u = np.array(u, dtype=np.complex128)
    c = colour(u.shape)
    d = diagonal(s, mask)
    for col in (0, 1):
        r = residual(u, f, s, mask)
        sel = c == col
        u[sel] = u[sel] + omega * r[sel] / d[sel]
    return u


def dense(s, mask) -> np.ndarray:
    """The matrix of A assembled node by node from the definition (not from
    ``apply``): for the cross-check pins and the direct reference solve."""
    shape = np.shape(s)
    dim = len(shape)
    n = list(reversed(shape))
    h = [1.0 / (na + 1) for na in n]
    N = int(np.prod(shape))
    sf = np.asarray(s).ravel()
    mf = np.asarray(mask).astype(bool).ravel()
    A = np.zeros((N, N), dtype=np.complex128)
    strides = [1]
    for a in range(1, dim):
        strides.append(strides[-1] * n[a - 1])
    for p in range(N):
        if mf[p]:
            A[p, p] = 1.0
            continue
        idx = [(p // strides[a]) % n[a] for a in range(dim)]
        diag = 0.0
        for a in range(dim):
            w = 1.0 / h[a] ** 2
            diag += 2.0 * w
            for step in (-1, 1):
                q_a = idx[a] + step
                if 0 <= q_a < n[a]:
                    q = p + step * strides[a]
                    if not mf[q]:
                        A[p, q] -= w
        A[p, p] = diag - sf[p]
    return A


def direct_solve(f, s, mask) -> np.ndarray:
    """u* = A^{-1} f by dense LU with partial pivoting (the direct reference
    of §4.1), for small grids only."""
    A = dense(s, mask)
    return np.linalg.solve(A, np.asarray(f, dtype=np.complex128).ravel()).reshape(np.shape(f))
