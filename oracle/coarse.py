"""Trunk-basis coarse correction (oracle), App. C.

The trunk matrix T (n x p) is evaluated at the grid nodes; the first
``p_used`` columns (natural-order selection) form the prolongation P, the
restriction is R = P^*, and the second preconditioner is
M2 = P (R A P)^{-1} R.  P is replaced by the Q factor of its QR
decomposition so that A_c = Q^T A Q is well conditioned.

Readings:

* rows of T at scatterer nodes are zeroed before the QR (the coarse space
  lives on the unknowns; the network is trained without a scatterer, §3.2);
* Q is real (T is real), so R = Q^* = Q^T;
* QR is Householder with positive diag(R); a column whose remaining norm is
  at most ``tau`` times the largest column norm of P is dropped (not
  reflected) and the number of kept columns is the rank used;
* the coarse solve uses LU with partial pivoting;
* optionally the basis is stored in fp32 (``q_round="f32"``): Q is the fp32
  rounding of the QR factor and A_c is the Galerkin matrix of that stored
  basis, so M2 stays the exact Galerkin correction on span(Q) for a basis
  within 1e-7 of the fp64 one.
"""
from __future__ import annotations

import numpy as np

from . import operator as op

TAU_C128 = 1e-7
TAU_C64 = 1e-5


def prolongation(T, mask, p_used):
    """P = first p_used trunk columns, zeroed on scatterer rows."""
    P = np.array(T[:, :p_used], dtype=np.float64)
    P[np.asarray(mask).astype(bool).ravel()] = 0.0
    return P


def householder_qr(P, tau=TAU_C128):
    """Column-dropping Householder QR.  Returns (Q, R, kept) with Q of shape
    (n, r), R (r x r) upper triangular with positive diagonal, and the indices
    of the kept columns of P, so that P[:, kept] = Q R."""
    A = np.array(P, dtype=np.float64)
    n, p = A.shape
    thresh = tau * np.max(np.linalg.norm(A, axis=0)) if p else 0.0
    vs = []
    kept = []
    R = np.zeros((min(n, p), p))
    for j in range(p):
        k = len(kept)
        x = A[k:, j]
        alpha = np.linalg.norm(x)
        if alpha <= thresh or k >= n:
            continue
        # reflector H = I - 2 v v^T / (v^T v) maps x to -sign(x0) alpha e1
        sgn = 1.0 if x[0] >= 0 else -1.0
        v = x.copy()
        v[0] += sgn * alpha
        v /= np.linalg.norm(v)
        A[k:, j:] -= 2.0 * np.outer(v, v @ A[k:, j:])
        vs.append(v)
        kept.append(j)
    r = len(kept)
    R = A[:r, kept].copy()
    R = np.triu(R)
    # Q = H_1 ... H_r [I_r; 0]
    Q = np.zeros((n, r))
    Q[:r, :r] = np.eye(r)
    for k in range(r - 1, -1, -1):
        v = vs[k]
        Q[k:, :] -= 2.0 * np.outer(v, v @ Q[k:, :])
    sg = np.sign(np.diag(R))
    sg[sg == 0] = 1.0
    Q = Q * sg[None, :]
    R = R * sg[:, None]
    return Q, R, kept


def galerkin(Q, s, mask, shape):
    """A_c = Q^T (A Q) (App. C, R A P with R = P^T)."""
    r = Q.shape[1]
    AQ = np.empty((Q.shape[0], r), dtype=np.complex128)
    for j in range(r):
        AQ[:, j] = op.apply(Q[:, j].reshape(shape).astype(np.complex128), s, mask).ravel()
    return Q.T @ AQ


class CoarseSpace:
    """Q, A_c and the coarse correction M2 r = Q A_c^{-1} Q^T r."""

    def __init__(self, T, s, mask, p_used, tau=TAU_C128, q_round=None):
        self.shape = np.shape(s)
        P = prolongation(T, mask, p_used)
        self.Q, self.R, self.kept = householder_qr(P, tau)
        if q_round == "f32":
            self.Q = self.Q.astype(np.float32).astype(np.float64)
        self.rank = self.Q.shape[1]
        self.Ac = galerkin(self.Q, s, mask, self.shape)

    def m2(self, r):
        """M2 r = Q A_c^{-1} Q^T r, with A_c^{-1} by LU with partial pivoting."""
        rf = np.asarray(r, dtype=np.complex128).ravel()
        y = self.Q.T @ rf
        c = np.linalg.solve(self.Ac, y)
        return (self.Q @ c).reshape(np.shape(r))
