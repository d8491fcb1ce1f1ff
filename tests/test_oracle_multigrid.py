"""Pins of the multigrid oracle (§4.3, DeepONet-MG-Krylov): transfer
operators against their closed forms and each other, the V-cycle against
the textbook contraction on the Laplacian and against dense LU, linearity,
and the a-1-b DeepONet-Jacobi smoother against its dense error-propagation
matrix."""
import numpy as np
import pytest

from paper_2405_12380_amd import inputs as I
from oracle import multigrid as mg, operator as op, krylov, meta as meta_or


def _mat(fn, shape_in, dtype=float):
    n = int(np.prod(shape_in))
    cols = []
    for j in range(n):
        e = np.zeros(n, dtype=dtype)
        e[j] = 1
        cols.append(np.asarray(fn(e.reshape(shape_in))).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("shape", [(7, 7, 7), (5, 9), (7, 3, 5)])
def test_prolongation_is_scaled_restriction_transpose(shape):
    dim = len(shape)
    nc = tuple((m + 1) // 2 - 1 for m in shape)
    zf = np.zeros(shape, np.uint8)
    zc = np.zeros(nc, np.uint8)
    R = _mat(lambda r: mg.restrict(r, zc), shape)
    P = _mat(lambda e: mg.prolong(e, shape, zf), nc)
    assert np.abs(P - 2 ** dim * R.T).max() <= 1e-15


def test_prolongation_reproduces_multilinear_functions():
    n = (15, 15, 15)
    nc = mg.coarse_n(n)
    Xc = mg.points(nc)
    f = lambda X: 0.3 + 1.7 * X[:, 0] - 0.4 * X[:, 1] + 2.2 * X[:, 2] + 0.9 * X[:, 0] * X[:, 1] * X[:, 2]
    ec = f(Xc).reshape(tuple(reversed(nc)))
    ef = mg.prolong(ec, tuple(reversed(n)), np.zeros(tuple(reversed(n)), np.uint8))
    ref = f(mg.points(n)).reshape(tuple(reversed(n)))
    inner = tuple(slice(1, m - 1) for m in reversed(n))
    assert np.abs(ef[inner] - ref[inner]).max() <= 1e-13


def test_full_weighting_of_a_quadratic():
    """FW of x^2 at coarse node X is X^2 + h^2 / 2 (h the fine spacing)."""
    n = (15, 7, 9)
    X = mg.points(n)[:, 0].reshape(tuple(reversed(n)))
    rc = mg.restrict(X ** 2, np.zeros(tuple(reversed(mg.coarse_n(n))), np.uint8))
    Xc = mg.points(mg.coarse_n(n))[:, 0].reshape(rc.shape)
    h = 1.0 / 16
    assert np.abs(rc - (Xc ** 2 + h * h / 2)).max() <= 1e-15


def test_vcycle_contracts_on_the_laplacian():
    """V-cycle with 5+5 damped Jacobi sweeps as a stationary iteration on the
    3D Laplacian (k = 0, no sponge, no mask): the error contracts by well under
    0.2 per cycle (classical multigrid behaviour)."""
    n = (15, 15, 15)
    shp = tuple(reversed(n))
    s = np.zeros(shp, complex)
    m = np.zeros(shp, np.uint8)
    H = mg.Hierarchy(s, m, levels=2, omega=0.5, nu=5)
    g = np.random.default_rng(0)
    f = g.standard_normal(shp) + 0j
    u = np.zeros(shp, complex)
    u_star = op.direct_solve(f, s, m)
    errs = []
    for _ in range(4):
        u = u + H.precond(op.residual(u, f, s, m)).reshape(shp)
        errs.append(np.linalg.norm(u - u_star))
    rates = [errs[i + 1] / errs[i] for i in range(3)]
    assert max(rates) < 0.2, rates


def test_exact_coarsest_solve_and_mg_gmres_against_lu():
    P = I.random_problem((7, 7, 7), seed=3, mask_frac=0.05, k=4.0)
    s = op.coefficient(P["ksq"], P["alpha"])
    f = P["f"] * (1 - P["mask"])
    H0 = mg.Hierarchy(s, P["mask"], levels=0)
    assert np.allclose(H0.precond(f.ravel()), op.direct_solve(f, s, P["mask"]).ravel(), rtol=1e-12, atol=1e-14)
    H = mg.Hierarchy(s, P["mask"], levels=2, omega=0.5, nu=5)
    u, info = meta_or.krylov_meta("gmres", f, np.zeros_like(f), s, P["mask"], 30, 1e-12, 300, precond=H.precond)
    assert info["status"] == 0
    assert np.linalg.norm(u - op.direct_solve(f, s, P["mask"])) <= 1e-9 * np.linalg.norm(u)


def test_deeponet_smoother_is_linear_and_differs_from_plain():
    C = I.config2(0, n=(15, 15, 15))
    s = op.coefficient(C["ksq"], C["alpha"])
    Hn = mg.Hierarchy(s, C["mask"], levels=2, omega=0.5, nu=5, trunk=C["trunk"], p_used=32)
    Hp = mg.Hierarchy(s, C["mask"], levels=2, omega=0.5, nu=5)
    g = np.random.default_rng(1)
    x = g.standard_normal(s.size) + 1j * g.standard_normal(s.size)
    y = g.standard_normal(s.size) + 1j * g.standard_normal(s.size)
    a, b = 0.7 - 0.2j, -1.3 + 0.5j
    lhs = Hn.precond(a * x + b * y)
    assert np.linalg.norm(lhs - (a * Hn.precond(x) + b * Hn.precond(y))) <= 1e-12 * np.linalg.norm(lhs)
    assert np.linalg.norm(Hn.precond(x) - Hp.precond(x)) > 1e-3 * np.linalg.norm(Hp.precond(x))
    # zero on scatterer nodes when the input is (Krylov residuals are)
    xm = np.where(C["mask"].ravel().astype(bool), 0, x)
    assert np.all(Hn.precond(xm)[C["mask"].ravel().astype(bool)] == 0)


@pytest.mark.parametrize("nu", [5, 4, 1, 2])
def test_deeponet_smoother_error_propagation(nu):
    """The a-1-b smoother (a = nu // 2 Jacobi sweeps, one trunk-basis
    correction, b = nu - a - 1 sweeps; 2-1-2 for nu = 5) propagates the error
    u - u* by S^b (I - Q A_c^{-1} Q^T A) S^a with S = I - omega D^{-1} A, all
    formed here as dense matrices from the row-by-row assembly of A.  nu = 4
    (a = 2, b = 1) fails if a and b are swapped; nu = 5 fails if the
    correction follows both sweep groups; nu = 1 is the correction alone."""
    C = I.config2(0, n=(7, 7, 7))
    s = op.coefficient(C["ksq"], C["alpha"])
    H = mg.Hierarchy(s, C["mask"], levels=1, omega=0.5, nu=nu, trunk=C["trunk"], p_used=32)
    A = op.dense(s, C["mask"])
    n = A.shape[0]
    S = np.eye(n) - 0.5 * A / np.diag(A)[:, None]
    Q = H.coarse[0].Q
    P = np.eye(n) - Q @ np.linalg.solve(Q.T @ A @ Q, Q.T @ A)
    a = nu // 2
    b = nu - a - 1
    E = np.linalg.matrix_power(S, b) @ P @ np.linalg.matrix_power(S, a)
    g = np.random.default_rng(nu)
    shp = s.shape
    f = (g.standard_normal(shp) + 1j * g.standard_normal(shp)) * (1 - C["mask"])
    u0 = (g.standard_normal(shp) + 1j * g.standard_normal(shp)) * (1 - C["mask"])
    u_star = np.linalg.solve(A, f.ravel())
    got = H.smooth(0, u0, f).ravel()
    ref = u_star + E @ (u0.ravel() - u_star)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)
