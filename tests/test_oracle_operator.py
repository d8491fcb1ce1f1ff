"""Pins of the oracle's operator and relaxations against facts fixed by the
mathematics (CPU only): discrete plane waves, dispersion, an independent
row-by-row assembly, complex symmetry, manufactured-solution convergence order,
sine-mode Jacobi factors and a dense red-black SOR splitting."""
import numpy as np
import pytest

from paper_2405_12380_amd import inputs as I
from oracle import operator as op


def _rand(n, seed, mask_frac=0.1):
    return I.random_problem(n, seed, mask_frac=mask_frac)


def _interior_clear(mask):
    """Nodes whose neighbours are all interior and unmasked, and themselves unmasked."""
    m = np.asarray(mask).astype(bool)
    ok = ~m
    for ax in range(m.ndim):
        for step in (1, -1):
            sh = np.roll(m, step, axis=ax)
            ok &= ~sh
        idx = [slice(None)] * m.ndim
        idx[ax] = 0
        ok[tuple(idx)] = False
        idx[ax] = -1
        ok[tuple(idx)] = False
    return ok


@pytest.mark.parametrize("n", [(9, 7), (8, 6, 5)])
def test_plane_wave_symbol(n):
    """x_p = exp(i kappa . x_p): (A x)_p = (sum_a 4/h_a^2 sin^2(kappa_a h_a / 2) - s_p) x_p
    at nodes away from ghosts and the scatterer (§2 eq. 1, second differences)."""
    P = _rand(n, 0, mask_frac=0.05)
    s = op.coefficient(P["ksq"], P["alpha"])
    X = I.mesh(n)
    kap = np.array([3.1, -1.7, 2.3])[: len(n)]
    x = np.exp(1j * sum(kap[a] * X[a] for a in range(len(n))))
    y = op.apply(x, s, P["mask"])
    h = [1.0 / (na + 1) for na in n]
    symbol = sum(4.0 / h[a] ** 2 * np.sin(kap[a] * h[a] / 2) ** 2 for a in range(len(n)))
    ok = _interior_clear(P["mask"])
    ref = (symbol - s) * x
    assert ok.sum() > 10
    assert np.max(np.abs(y[ok] - ref[ok])) <= 1e-13 * np.max(np.abs(ref[ok]) + symbol)


def test_dispersion_shell_zero():
    """alpha = 0 and kappa on the discrete dispersion shell: A x = 0 at interior nodes."""
    n = (10, 9, 8)
    k = 7.0
    h = [1.0 / (na + 1) for na in n]
    kx, ky = 2.0, 3.0
    rest = k * k - 4 / h[0] ** 2 * np.sin(kx * h[0] / 2) ** 2 - 4 / h[1] ** 2 * np.sin(ky * h[1] / 2) ** 2
    kz = 2.0 / h[2] * np.arcsin(np.sqrt(rest * h[2] ** 2 / 4))
    X = I.mesh(n)
    x = np.exp(1j * (kx * X[0] + ky * X[1] + kz * X[2]))
    s = np.full(I.field_shape(n), k * k) + 0j
    mask = np.zeros(I.field_shape(n), np.uint8)
    y = op.apply(x, s, mask)
    ok = _interior_clear(mask)
    assert np.max(np.abs(y[ok])) <= 1e-10 * k * k


@pytest.mark.parametrize("n", [(6, 5), (5, 4, 3), (4, 4, 4)])
def test_apply_matches_independent_assembly(n):
    P = _rand(n, 1, mask_frac=0.2)
    s = op.coefficient(P["ksq"], P["alpha"])
    A = op.dense(s, P["mask"])
    y = op.apply(P["x"], s, P["mask"]).ravel()
    assert np.max(np.abs(y - A @ P["x"].ravel())) <= 1e-12 * np.max(np.abs(y))


def test_complex_symmetric_and_identity_rows():
    """y^T (A x) = x^T (A y) without conjugation (symmetric elimination of the
    scatterer); masked rows are the identity exactly."""
    n = (7, 6, 5)
    P = _rand(n, 2, mask_frac=0.15)
    s = op.coefficient(P["ksq"], P["alpha"])
    g = np.random.default_rng(1)
    x = P["x"]
    y = g.standard_normal(x.shape) + 1j * g.standard_normal(x.shape)
    lhs = np.sum(y * op.apply(x, s, P["mask"]))
    rhs = np.sum(x * op.apply(y, s, P["mask"]))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    m = P["mask"].astype(bool)
    assert np.array_equal(op.apply(x, s, P["mask"])[m], x[m])
    A = op.dense(s, P["mask"])
    assert np.array_equal(A, A.T)


def _mms(n, k=3.0):
    X = I.mesh(n)
    u = np.sin(np.pi * X[0]) * np.sin(2 * np.pi * X[1]) * np.sin(3 * np.pi * X[2]) * (1 + 0.5j)
    alpha = 0.3 + 0.2 * X[0]
    lap = -(1 + 4 + 9) * np.pi ** 2 * u
    f = -lap - k * k * (1 + 1j * alpha) * u
    return u, f, np.full(u.shape, k * k), alpha


def test_manufactured_solution_second_order():
    """u* = sin(pi x) sin(2 pi y) sin(3 pi z)(1 + i/2) with a smooth alpha; f from
    the continuous operator; the direct solve converges at order 2."""
    errs = []
    hs = []
    for N in (7, 11, 15):
        n = (N, N, N)
        u, f, ksq, alpha = _mms(n)
        s = op.coefficient(ksq, alpha)
        uh = op.direct_solve(f, s, np.zeros(u.shape, np.uint8))
        errs.append(np.linalg.norm(uh - u) / np.linalg.norm(u))
        hs.append(1.0 / (N + 1))
    orders = [np.log(errs[i] / errs[i + 1]) / np.log(hs[i] / hs[i + 1]) for i in range(2)]
    assert all(1.85 <= o <= 2.15 for o in orders), orders


@pytest.mark.parametrize("n", [(9, 8), (6, 5, 4)])
def test_jacobi_sine_mode_factor(n):
    """alpha = 0, no scatterer, homogeneous k: sine modes are eigenvectors, and
    one damped Jacobi step with f = 0 multiplies mode m by 1 - omega lambda_m / D."""
    k, omega = 5.0, 0.7
    X = I.mesh(n)
    h = [1.0 / (na + 1) for na in n]
    m = [2, 3, 1][: len(n)]
    e = np.ones(I.field_shape(n))
    for a in range(len(n)):
        e = e * np.sin(m[a] * np.pi * X[a])
    s = np.full(e.shape, k * k) + 0j
    mask = np.zeros(e.shape, np.uint8)
    lam = sum(4 / h[a] ** 2 * np.sin(m[a] * np.pi * h[a] / 2) ** 2 for a in range(len(n))) - k * k
    D = sum(2 / h[a] ** 2 for a in range(len(n))) - k * k
    u1 = op.jacobi_sweep(e + 0j, np.zeros_like(s), s, mask, omega)
    assert np.max(np.abs(u1 - (1 - omega * lam / D) * e)) <= 1e-13 * np.max(np.abs(e)) * (1 + abs(lam / D))


def test_jacobi_diverges_above_smallest_eigenvalue():
    """k^2 beyond the smallest discrete eigenvalue makes plain Jacobi amplify the
    lowest mode (the paper's relaxation methods diverge on the scattering
    problem)."""
    n = (12, 12)
    X = I.mesh(n)
    h = 1.0 / 13
    e = np.sin(np.pi * X[0]) * np.sin(np.pi * X[1]) + 0j
    lam0 = 2 * 4 / h ** 2 * np.sin(np.pi * h / 2) ** 2
    k2 = lam0 * 1.5
    s = np.full(e.shape, k2) + 0j
    u = e
    for _ in range(50):
        u = op.jacobi_sweep(u, np.zeros_like(e), s, np.zeros(e.shape, np.uint8), 1.0)
    growth = 1 - (lam0 - k2) / (4 / h ** 2 - k2)
    assert growth > 1
    assert np.linalg.norm(u) / np.linalg.norm(e) == pytest.approx(growth ** 50, rel=1e-10)


@pytest.mark.parametrize("omega", [1.0, 1.3])
@pytest.mark.parametrize("n", [(5, 4), (4, 3, 3), (3, 5, 4)])
def test_rbgs_equals_dense_sor_splitting(n, omega):
    """Red-black GS/SOR equals u + omega (D + omega L)^{-1} (f - A u) with A
    ordered red nodes first and L its strictly lower part (brute force)."""
    P = _rand(n, 3, mask_frac=0.2)
    s = op.coefficient(P["ksq"], P["alpha"])
    A = op.dense(s, P["mask"])
    col = op.colour(I.field_shape(n)).ravel()
    perm = np.concatenate([np.flatnonzero(col == 0), np.flatnonzero(col == 1)])
    Ap = A[np.ix_(perm, perm)]
    D = np.diag(np.diag(Ap))
    L = np.tril(Ap, -1)
    u = P["x"].ravel()[perm]
    f = P["f"].ravel()[perm]
    ref_p = u + omega * np.linalg.solve(D + omega * L, f - Ap @ u)
    ref = np.empty_like(ref_p)
    ref[perm] = ref_p
    got = op.rbgs_sweep(P["x"], P["f"], s, P["mask"], omega).ravel()
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_residual_vanishes_on_scatterer():
    """App. D: rows that impose the Dirichlet condition have zero residual for
    any iterate satisfying it; here u = 0 and f = 0 on the scatterer."""
    n = (9, 8, 7)
    P = _rand(n, 4, mask_frac=0.2)
    s = op.coefficient(P["ksq"], P["alpha"])
    m = P["mask"].astype(bool)
    u = P["x"].copy()
    f = P["f"].copy()
    u[m] = 0
    f[m] = 0
    r = op.residual(u, f, s, P["mask"])
    assert np.all(r[m] == 0)
    for sweep in (op.jacobi_sweep, op.rbgs_sweep):
        v = sweep(u, f, s, P["mask"], 0.8)
        assert np.all(v[m] == 0)
