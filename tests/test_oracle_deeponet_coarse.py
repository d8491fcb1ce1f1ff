"""Pins of the oracle's DeepONet and trunk-basis coarse space (CPU only):
a hand-computed network, torch float64 layers with the same weights, the
output heads, the positive homogeneity created by the residual scaling,
multilinear resampling, Householder QR with column dropping against LAPACK,
Galerkin orthogonality, M2 A Q = Q, basis invariance, the sine-basis closed
form and the full-basis exactness."""
import math

import numpy as np
import pytest
import torch

from paper_2405_12380_amd import inputs as I
from oracle import operator as op, deeponet as don, coarse, meta, krylov


def test_hand_computed_network():
    """2 -> 3 -> 2 tanh network with weights chosen so each output is a short
    closed form of tanh values."""
    W1 = np.array([[1.0, 0.0, 2.0], [0.0, -1.0, 0.5]])
    b1 = np.array([0.0, 0.25, -1.0])
    W2 = np.array([[1.0, 0.0], [0.0, 2.0], [1.0, -1.0]])
    b2 = np.array([0.5, 0.0])
    x = np.array([[0.3, -0.7]])
    y = don.mlp(x, [(W1, b1), (W2, b2)])
    h = [math.tanh(0.3), math.tanh(0.7 + 0.25), math.tanh(0.6 - 0.35 - 1.0)]
    assert y[0, 0] == pytest.approx(h[0] + h[2] + 0.5, rel=1e-15)
    assert y[0, 1] == pytest.approx(2 * h[1] - h[2], rel=1e-15)


def test_mlp_matches_torch_float64():
    g = np.random.default_rng(0)
    layers = I.glorot_mlp([5, 16, 16, 7], g)
    layers = [(W, g.standard_normal(b.shape) * 0.1) for W, b in layers]
    x = g.standard_normal((11, 5))
    ref = torch.as_tensor(x)
    for li, (W, b) in enumerate(layers):
        lin = torch.nn.Linear(W.shape[0], W.shape[1], dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.as_tensor(W.T))
            lin.bias.copy_(torch.as_tensor(b))
        ref = lin(ref)
        if li < len(layers) - 1:
            ref = torch.tanh(ref)
    assert np.max(np.abs(don.mlp(x, layers) - ref.detach().numpy())) <= 1e-14


def test_split_output_head_closed_form():
    """With T = I and a single linear branch layer W, the head gives
    du = s (W^T x)[:p] + i s (W^T x)[p:] at unmasked nodes (App. B)."""
    n = (4, 3)
    N = 12
    g = np.random.default_rng(1)
    r = g.standard_normal((3, 4)) + 1j * g.standard_normal((3, 4))
    W = g.standard_normal((2 * N, 2 * N)) * 0.3
    T = np.eye(N)
    mask = np.zeros((3, 4), np.uint8)
    mask[1, 2] = 1
    du = don.infer(r, mask, T, [(W, np.zeros(2 * N))], "split_output", N, n)
    s = np.linalg.norm(r) / math.sqrt(N)
    x = np.concatenate([r.real.ravel(), r.imag.ravel()]) / s
    b = x @ W
    ref = s * (b[:N] + 1j * b[N:])
    ref[mask.ravel().astype(bool)] = 0
    assert np.max(np.abs(du.ravel() - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_split_input_head_closed_form():
    n = (4, 3)
    N = 12
    g = np.random.default_rng(2)
    r = g.standard_normal((3, 4)) + 1j * g.standard_normal((3, 4))
    W = g.standard_normal((N, N)) * 0.3
    du = don.infer(r, np.zeros((3, 4), np.uint8), np.eye(N), [(W, np.zeros(N))], "split_input", N, n)
    # one linear layer: du = (Re r) W + i (Im r) W
    ref = r.real.ravel() @ W + 1j * (r.imag.ravel() @ W)
    assert np.max(np.abs(du.ravel() - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_scaling_rule_positive_homogeneity():
    """du = s N(r / s) with s = ||r|| / sqrt(n) makes du(c r) = c du(r) for c > 0
    even for a nonlinear network; du(0) = 0."""
    C = I.config1()
    T = don.trunk_matrix(I.node_points(C["n"]), C["trunk"])
    g = np.random.default_rng(3)
    r = g.standard_normal(I.field_shape(C["n"])) + 1j * g.standard_normal(I.field_shape(C["n"]))
    d1 = don.infer(r, C["mask"], T, C["branch"], "split_input", C["p"], C["n"])
    d2 = don.infer(3.7 * r, C["mask"], T, C["branch"], "split_input", C["p"], C["n"])
    assert np.max(np.abs(d2 - 3.7 * d1)) <= 1e-12 * np.max(np.abs(d2))
    assert np.all(don.infer(0 * r, C["mask"], T, C["branch"], "split_input", C["p"], C["n"]) == 0)
    assert np.all(d1[C["mask"].astype(bool)] == 0)


def test_multilinear_sampling():
    """Resampling reproduces a multilinear field at target nodes whose source
    cell lies between interior nodes, and blends with the zero ghost in the
    boundary cells; identity when the grids agree."""
    n = (9, 7, 5)
    X = I.mesh(n)
    f = 1.0 + 2.0 * X[0] - 0.5 * X[1] + 0.25 * X[2] + X[0] * X[1] * X[2]
    assert np.array_equal(don.sample_to(f, n), f)
    m = (4, 3, 2)
    out = don.sample_to(f, m)
    Y = I.mesh(m)
    exact = 1.0 + 2.0 * Y[0] - 0.5 * Y[1] + 0.25 * Y[2] + Y[0] * Y[1] * Y[2]
    inner = np.ones(out.shape, bool)
    for a, (na, ma) in enumerate(zip(n, m)):
        xt = np.arange(1, ma + 1) / (ma + 1)
        ok = (xt >= 1.0 / (na + 1)) & (xt <= na / (na + 1))
        sh = [1] * 3
        sh[2 - a] = ma
        inner &= ok.reshape(sh)
    assert inner.sum() > 0
    assert np.max(np.abs(out[inner] - exact[inner])) <= 1e-13
    # 1D boundary cell: value = w f(x_0) with w the distance fraction from the ghost
    src = np.ones((1, 1, 4))  # n = (4, 1, 1); target (2, 1, 1): x = 1/3 -> t = 5/3 - 1
    o = don.sample_to(src, (2, 1, 1))
    assert o.ravel() == pytest.approx([1.0, 1.0])
    src = np.arange(1.0, 5.0).reshape(1, 1, 4)  # f(x_i) = i+1 at x_i = (i+1)/5
    o = don.sample_to(src, (9, 1, 1))  # x = 0.1: between ghost (0) and x_0 = 0.2 -> 0.5
    assert o.ravel()[0] == pytest.approx(0.5)


def test_householder_qr_matches_lapack():
    g = np.random.default_rng(4)
    P = g.standard_normal((300, 20))
    Q, R, kept = coarse.householder_qr(P)
    assert kept == list(range(20))
    Qn, Rn = np.linalg.qr(P)
    sg = np.sign(np.diag(Rn))
    Qn, Rn = Qn * sg, Rn * sg[:, None]
    assert np.max(np.abs(Q - Qn)) <= 1e-12
    assert np.max(np.abs(R - Rn)) <= 1e-11
    assert np.all(np.diag(R) > 0)


def test_householder_drops_dependent_columns():
    g = np.random.default_rng(5)
    B = g.standard_normal((200, 6))
    P = np.column_stack([B[:, 0], B[:, 1], B[:, 0] + 2 * B[:, 1], B[:, 2], B[:, 3] * 0.0, B[:, 4], B[:, 5],
                         3 * B[:, 5] - B[:, 2]])
    Q, R, kept = coarse.householder_qr(P, tau=1e-7)
    assert kept == [0, 1, 3, 5, 6]
    assert np.max(np.abs(Q @ R - P[:, kept])) <= 1e-12 * np.max(np.abs(P))
    assert np.max(np.abs(Q.T @ Q - np.eye(5))) <= 1e-13


def _coarse_problem(n=(7, 6, 5), p=20, seed=6):
    P = I.random_problem(n, seed, mask_frac=0.1)
    s = op.coefficient(P["ksq"], P["alpha"])
    g = np.random.default_rng(seed)
    trunk = I.glorot_mlp([3, 32, 32, p], g, first_gain=30.0)
    T = don.trunk_matrix(I.node_points(n), trunk)
    return P, s, T


def test_galerkin_orthogonality_and_exactness_on_span():
    """Q^T (r - A M2 r) = 0 and M2 A Q = Q (App. C: M2 = P (R A P)^{-1} R)."""
    P, s, T = _coarse_problem()
    cs = coarse.CoarseSpace(T, s, P["mask"], 16)
    shape = s.shape
    A = lambda v: op.apply(v.reshape(shape), s, P["mask"]).ravel()
    r = P["f"].ravel()
    z = cs.m2(r.reshape(shape)).ravel()
    assert np.max(np.abs(cs.Q.T @ (r - A(z)))) <= 1e-11 * np.linalg.norm(r)
    for j in range(cs.rank):
        q = cs.Q[:, j].astype(complex)
        back = cs.m2(A(q).reshape(shape)).ravel()
        assert np.max(np.abs(back - q)) <= 1e-10
    assert np.max(np.abs(cs.Q[P["mask"].ravel().astype(bool)])) <= 1e-14


def test_fp32_stored_basis_is_exact_galerkin():
    """With Q rounded to fp32 and A_c built from the rounded Q, M2 is still the
    Galerkin correction on span(Q): Q^T (r - A M2 r) = 0 and M2 A Q = Q."""
    P, s, T = _coarse_problem()
    cs = coarse.CoarseSpace(T, s, P["mask"], 16, q_round="f32")
    assert np.array_equal(cs.Q, cs.Q.astype(np.float32).astype(np.float64))
    shape = s.shape
    A = lambda v: op.apply(v.reshape(shape), s, P["mask"]).ravel()
    r = P["f"].ravel()
    z = cs.m2(r.reshape(shape)).ravel()
    assert np.max(np.abs(cs.Q.T @ (r - A(z)))) <= 1e-11 * np.linalg.norm(r)
    q = cs.Q[:, 3].astype(complex)
    assert np.max(np.abs(cs.m2(A(q).reshape(shape)).ravel() - q)) <= 1e-10


def test_basis_invariance():
    """M2 depends only on span(P): any invertible mixing of the columns gives
    the same correction."""
    P, s, T = _coarse_problem()
    g = np.random.default_rng(7)
    Mx = np.triu(g.standard_normal((16, 16))) + 4 * np.eye(16)
    T2 = T.copy()
    T2[:, :16] = T[:, :16] @ Mx
    c1 = coarse.CoarseSpace(T, s, P["mask"], 16)
    c2 = coarse.CoarseSpace(T2, s, P["mask"], 16)
    r = P["f"]
    assert np.max(np.abs(c1.m2(r) - c2.m2(r))) <= 1e-9 * np.max(np.abs(c1.m2(r)))


def test_sine_basis_diagonal_coarse_matrix():
    """alpha = 0, no scatterer, homogeneous k, T = sine modes: A_c = diag(lambda_m)."""
    n = (8, 7, 6)
    k = 4.0
    X = I.mesh(n)
    h = [1.0 / (na + 1) for na in n]
    modes = [(1, 1, 1), (2, 1, 1), (1, 3, 2), (2, 2, 2), (3, 1, 4)]
    cols, lams = [], []
    for m in modes:
        e = np.ones(I.field_shape(n))
        for a in range(3):
            e = e * np.sin(m[a] * np.pi * X[a])
        cols.append(e.ravel())
        lams.append(sum(4 / h[a] ** 2 * np.sin(m[a] * np.pi * h[a] / 2) ** 2 for a in range(3)) - k * k)
    T = np.stack(cols, axis=1)
    s = np.full(I.field_shape(n), k * k) + 0j
    cs = coarse.CoarseSpace(T, s, np.zeros(I.field_shape(n), np.uint8), len(modes))
    assert cs.rank == len(modes)
    assert np.max(np.abs(cs.Ac - np.diag(lams))) <= 1e-10 * max(abs(l) for l in lams)


def test_full_basis_makes_meta_krylov_exact():
    """p_used = n: M2 = A^{-1}, so DeepONet-GMRES and -BiCGStab converge in one
    iteration, and the relaxation meta-solver with the exact inverse as its
    correction converges at the first correction."""
    n = (4, 4, 4)
    C = I.config2(0, n=n)
    C["mask"][:] = 0
    s = op.coefficient(C["ksq"], C["alpha"])
    T = don.trunk_matrix(I.node_points(n), C["trunk"])
    cs = coarse.CoarseSpace(T, s, C["mask"], 64)
    assert cs.rank == 64
    M = meta.krylov_preconditioner(s, C["mask"], "jacobi", 1, 0.5, cs)
    for kind in ("gmres", "bicgstab"):
        u, info = meta.krylov_meta(kind, C["f"], np.zeros_like(C["f"]), s, C["mask"], 10, 1e-9, 10, precond=M)
        assert info["status"] == krylov.CONVERGED and info["iters"] == 1
    Ad = op.dense(s, C["mask"])
    exact = lambda r: np.linalg.solve(Ad, r.ravel()).reshape(r.shape)
    u, info = meta.relaxation_meta(C["f"], np.zeros_like(C["f"]), s, C["mask"], "jacobi", 0.5, 100, 3, 1e-12,
                                   correction=exact)
    assert info["status"] == krylov.CONVERGED and info["iters"] == 3 and info["corrections"] == 1


def _c1_like(n=20, k=10.0):
    """Config 1's scatterer and source on a smaller 2D grid (k^2 above the
    smallest eigenvalue of the Laplacian: plain Jacobi eventually grows)."""
    nn = (n, n)
    mask = I.box_mask(nn, (0.5, 0.5), 0.1)
    f = I.gaussian_source(nn, (0.25, 0.5), 0.05)
    f[mask.astype(bool)] = 0
    return nn, op.coefficient(np.full(I.field_shape(nn), k * k), I.sponge(nn)), mask, f


def test_relaxation_fallback_reaches_direct_solve():
    """A relaxation meta-solve whose correction makes the residual grow hands
    over to standalone GMRES, which reaches the dense direct solution."""
    nn, s, mask, f = _c1_like()
    u_star = op.direct_solve(f, s, mask)

    def bad(r):  # a correction that amplifies the residual
        return 50.0 * r

    h = []
    u, info = meta.relaxation_meta(f, np.zeros_like(f), s, mask, "jacobi", 0.5, 2000, 5, 1e-12, correction=bad,
                                   history=h, fallback_restart=40)
    assert info["status"] == 0 and info["iters"] == 5 and info["corrections"] == 1
    assert h[0] > 1.0 and info["fallback_iters"] > 0
    assert np.linalg.norm(u - u_star) <= 1e-9 * np.linalg.norm(u_star)
    # without the fallback the same iteration does not converge
    _, info0 = meta.relaxation_meta(f, np.zeros_like(f), s, mask, "jacobi", 0.5, 200, 5, 1e-12, correction=bad)
    assert info0["status"] != 0 and info0["fallback_iters"] == 0


def test_relaxation_fallback_idle_when_contracting():
    """Homogeneous positive-definite case (k^2 below the smallest eigenvalue, no
    sponge, no scatterer): damped Jacobi contracts every residual, the fallback
    never triggers and the result equals the run without it, bit for bit."""
    nn = (16, 16)
    s = op.coefficient(np.full(I.field_shape(nn), 4.0), np.zeros(I.field_shape(nn)))
    mask = np.zeros(I.field_shape(nn), np.uint8)
    f = I.gaussian_source(nn, (0.4, 0.6), 0.1)
    u1, i1 = meta.relaxation_meta(f, np.zeros_like(f), s, mask, "jacobi", 0.5, 300, 10, 0.0, fallback_restart=20)
    u0, i0 = meta.relaxation_meta(f, np.zeros_like(f), s, mask, "jacobi", 0.5, 300, 10, 0.0)
    assert i1["fallback_iters"] == 0 and i1["iters"] == 300
    assert np.array_equal(u1, u0)


def test_relaxation_fallback_restarts_from_last_good_iterate():
    """Plain Jacobi on the C1-like grid decreases the residual for a while and
    then grows.  The fallback must start from the iterate before the first
    growing cycle (not the grown one, not u0): its result equals GMRES started
    from the iterate of a separate relaxation run stopped before that cycle."""
    nn, s, mask, f = _c1_like()
    h = []
    meta.relaxation_meta(f, np.zeros_like(f), s, mask, "jacobi", 0.5, 4000, 25, 0.0, history=h)
    h = np.array(h)
    grow = int(np.argmax(h[1:] > h[:-1])) + 1   # first cycle whose residual exceeds the previous one
    assert h[grow] > h[grow - 1] and np.all(np.diff(h[:grow]) < 0)
    budget = 25 * (grow + 1)
    u_prev, _ = meta.relaxation_meta(f, np.zeros_like(f), s, mask, "jacobi", 0.5, 25 * grow, 25, 0.0)
    u, info = meta.relaxation_meta(f, np.zeros_like(f), s, mask, "jacobi", 0.5, budget, 25, 0.0, fallback_restart=10)
    assert info["fallback_iters"] == budget

    def A(v):
        return op.apply(v.reshape(s.shape), s, mask).ravel()
    ref, _ = krylov.gmres(A, f.ravel(), u_prev.ravel(), 10, 0.0, budget)
    assert np.linalg.norm(u.ravel() - ref) <= 1e-13 * np.linalg.norm(ref)
