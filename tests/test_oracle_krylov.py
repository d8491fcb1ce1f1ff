"""Pins of the oracle's GMRES(m) (one or two classical Gram-Schmidt passes)
and BiCGStab (CPU only): the GMRES
minimal-residual property against an independent least-squares solve over an
explicitly built Krylov basis, |g| equal to the true residual, finite
termination on matrices with few distinct eigenvalues, agreement with the
dense direct solve, and breakdown detection."""
import numpy as np
import pytest

from paper_2405_12380_amd import inputs as I
from oracle import operator as op, krylov, meta


def _small(n=(6, 5, 4), seed=0):
    P = I.random_problem(n, seed, mask_frac=0.1)
    s = op.coefficient(P["ksq"], P["alpha"])
    m = P["mask"].astype(bool)
    f = P["f"].copy()
    f[m] = 0
    shape = f.shape

    def A(v):
        return op.apply(v.reshape(shape), s, P["mask"]).ravel()
    return P, s, f, A


def test_givens_rotation():
    for a, b in [(3 + 4j, 2.0), (-1e-3 + 2j, 5.0), (0j, 1.5), (2 - 1j, 0.0)]:
        c, s = krylov.givens(a, b)
        G = np.array([[c, s], [-np.conj(s), c]])
        v = G @ np.array([a, b])
        assert abs(v[1]) <= 1e-15 * (abs(a) + b)
        assert np.allclose(G.conj().T @ G, np.eye(2), atol=1e-15)
        assert abs(v[0]) == pytest.approx(np.hypot(abs(a), b), rel=1e-15)


@pytest.mark.parametrize("k", [1, 3, 7, 12])
@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("gs_passes", [1, 2])
def test_gmres_minimal_residual(k, precond, gs_passes):
    """After k < m steps from u0 = 0, GMRES minimises ||f - A M y|| over the
    Krylov space K_k(A M, f); the minimiser is computed here from a QR of the
    explicit power basis, independently of Arnoldi and the Givens rotations."""
    P, s, f, A = _small()
    ff = f.ravel()
    d = np.random.default_rng(7).uniform(0.5, 2.0, ff.size) * np.exp(1j * np.random.default_rng(8).uniform(0, 1, ff.size))
    M = (lambda v: d * v) if precond else None
    AM = (lambda v: A(d * v)) if precond else A
    u, info = krylov.gmres(A, ff, np.zeros_like(ff), 30, 0.0, k, M=M, gs_passes=gs_passes)
    assert info["iters"] == k
    K = [ff]
    for _ in range(k - 1):
        K.append(AM(K[-1]))
    K = np.stack(K, axis=1)
    Qk, _ = np.linalg.qr(K)
    AQ = np.stack([AM(Qk[:, j]) for j in range(Qk.shape[1])], axis=1)
    y, *_ = np.linalg.lstsq(AQ, ff, rcond=None)
    u_ref = Qk @ y
    if precond:
        u_ref = d * u_ref
    r_ref = np.linalg.norm(ff - A(u_ref))
    r_got = np.linalg.norm(ff - A(u))
    assert r_got <= r_ref * (1 + 1e-9) + 1e-14 * np.linalg.norm(ff)
    assert np.linalg.norm(u - u_ref) <= 1e-8 * np.linalg.norm(u_ref)


@pytest.mark.parametrize("gs_passes", [1, 2])
def test_gmres_residual_estimate_matches_true_residual(gs_passes):
    """|g_{j+1}| after j Arnoldi steps equals ||f - A u_j|| of the iterate formed
    from those steps (right preconditioning keeps the true residual)."""
    P, s, f, A = _small()
    ff = f.ravel()
    hist = []
    krylov.gmres(A, ff, np.zeros_like(ff), 40, 0.0, 20, history=hist, gs_passes=gs_passes)
    for j in (1, 5, 11, 20):
        u, info = krylov.gmres(A, ff, np.zeros_like(ff), 40, 0.0, j, gs_passes=gs_passes)
        assert info["rel_res"] == pytest.approx(hist[j], rel=1e-8)
    # monotone within a cycle
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(1, 20))


def test_unrestarted_gmres_terminates_in_n_steps():
    n = (3, 3, 3)
    P, s, f, A = _small(n, 2)
    ff = f.ravel()
    u, info = krylov.gmres(A, ff, np.zeros_like(ff), 40, 1e-12, 40)
    assert info["status"] == krylov.CONVERGED and info["iters"] <= ff.size


def test_few_distinct_eigenvalues_terminate():
    """A with 3 distinct eigenvalues: GMRES converges in 3 steps; BiCGStab (whose
    BiCG part terminates within 3 steps) converges within 2 iterations on 2
    distinct eigenvalues and in 1 on a multiple of the identity."""
    g = np.random.default_rng(3)
    N = 40
    V = g.standard_normal((N, N)) + 1j * g.standard_normal((N, N))
    lam3 = np.repeat([2.0 + 1j, -1.0 + 0.5j, 3.0], [10, 15, 15])
    A3 = V @ np.diag(lam3) @ np.linalg.inv(V)
    b = g.standard_normal(N) + 1j * g.standard_normal(N)
    u, info = krylov.gmres(lambda v: A3 @ v, b, np.zeros(N, complex), 10, 1e-10, 10)
    assert info["status"] == krylov.CONVERGED and info["iters"] == 3
    lam2 = np.repeat([2.0 + 1j, -1.0 + 0.5j], [20, 20])
    A2 = V @ np.diag(lam2) @ np.linalg.inv(V)
    u, info = krylov.bicgstab(lambda v: A2 @ v, b, np.zeros(N, complex), 1e-9, 10)
    assert info["status"] == krylov.CONVERGED and info["iters"] <= 2
    u, info = krylov.bicgstab(lambda v: (2.5 - 1j) * v, b, np.zeros(N, complex), 1e-12, 10)
    assert info["status"] == krylov.CONVERGED and info["iters"] == 1
    assert np.allclose(u, b / (2.5 - 1j), rtol=1e-13)


@pytest.mark.parametrize("kind", ["gmres", "gmres_cgs1", "bicgstab"])
@pytest.mark.parametrize("n", [(8, 7, 6), (12, 12, 12)])
def test_converged_against_direct_solve(kind, n):
    P, s, f, A = _small(n, 4)
    u_star = op.direct_solve(f, s, P["mask"])
    passes = 1 if kind == "gmres_cgs1" else 2
    u, info = meta.krylov_meta(kind.split("_")[0], f, np.zeros_like(f), s, P["mask"], 50, 1e-13, 20000,
                               gs_passes=passes)
    assert info["status"] == krylov.CONVERGED
    assert np.linalg.norm(u - u_star) <= 1e-9 * np.linalg.norm(u_star)
    m = P["mask"].astype(bool)
    assert np.all(u[m] == 0)


def test_bicgstab_breakdown_detected():
    """r_hat^H A p = 0 at the first step (a rotation) is reported as breakdown and
    leaves the iterate untouched."""
    A = np.array([[0.0, 1.0], [-1.0, 0.0]], dtype=complex)
    b = np.array([1.0, 0.0], dtype=complex)
    u, info = krylov.bicgstab(lambda v: A @ v, b, np.zeros(2, complex), 1e-10, 10)
    assert info["status"] == krylov.BREAKDOWN
    assert np.all(u == 0)


def test_gmres_restart_counts_and_nonconvergence():
    P, s, f, A = _small((8, 8, 8), 5)
    ff = f.ravel()
    u, info = krylov.gmres(A, ff, np.zeros_like(ff), 5, 1e-14, 23)
    assert info["status"] == krylov.NOT_CONVERGED and info["iters"] == 23
    assert info["precond_apps"] == 0  # no preconditioner given
    # 4 full cycles of 5 and one of 3: one true residual per cycle start, one at exit
    assert info["matvecs"] == 23 + 5 + 1


def test_golden_bicgstab_counts_match_oracle():
    """The stored count range (tests/golden) was written by the oracle as it
    stands: its unperturbed count is recomputed here."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bicgstab_counts_20cube.json")
    with open(path) as fh:
        ref = json.load(fh)
    C = I.config2(1, n=(20, 20, 20))
    s = op.coefficient(C["ksq"], C["alpha"])
    _, info = meta.krylov_meta("bicgstab", C["f"], np.zeros_like(C["f"]), s, C["mask"], 50, ref["tol"], 5000)
    assert info["iters"] == ref["unperturbed"]
    assert ref["min"] <= ref["unperturbed"] <= ref["max"] and len(ref["counts"]) == 31


@pytest.mark.parametrize("kind", ["gmres", "bicgstab"])
def test_zero_source_uses_the_absolute_residual(kind):
    """f = 0 (relative residual undefined): from u0 != 0 the solvers drive
    ||A u|| below tol itself and report it as rel_res; from u0 = 0 they stop
    at once with u = 0."""
    P, s, f, A = _small((6, 6, 6), 9)
    zero = np.zeros(f.size, complex)
    u0 = np.random.default_rng(3).standard_normal(f.size) * (1 - P["mask"].ravel())
    solve = (lambda b, x, tol: krylov.gmres(A, b, x, 30, tol, 500)) if kind == "gmres" else \
        (lambda b, x, tol: krylov.bicgstab(A, b, x, tol, 500))
    u, info = solve(zero, u0, 1e-9)
    assert info["status"] == krylov.CONVERGED and info["iters"] > 0
    res = np.linalg.norm(A(u))
    assert res <= 1e-9 and info["rel_res"] == pytest.approx(res, rel=1e-12)
    u, info = solve(zero, np.zeros_like(zero), 1e-9)
    assert info["status"] == krylov.CONVERGED and info["iters"] == 0 and not np.any(u)
