"""Parity at the benchmark's full sizes, in the configurations bench.py times,
checked with what the oracle can afford at those sizes: the oracle's own
operator applied to the GPU's solutions (true residuals), the oracle's V-cycle
and training gradients at full size, and finite differences of the adjoint
gradient."""
import numpy as np
import pytest
import torch

from paper_2405_12380_amd import inputs as I
from oracle import operator as op_or, multigrid as mg_or, training as T
from tests.helpers import make_op, rel_err, to_np

pytestmark = pytest.mark.gpu

helm = pytest.importorskip("paper_2405_12380_amd.helm")


def _net(C):
    return helm.DeepONet(helm.C128, C["branch"], C["trunk"], C["p"], head="split_output", branch_grid=(16, 16, 16),
                         k_input=True)


@pytest.mark.parametrize("instance", [0, 2])
def test_headline_solve_64cube(instance):
    """DeepONet-GMRES(50), p = 128, n_r = 3 at 64^3 to 1e-6 (the timed step): the
    oracle's operator confirms the relative residual of the GPU solution."""
    C = I.config2(instance)
    s = op_or.coefficient(C["ksq"], C["alpha"])
    op = make_op(helm, C, helm.C128)
    u = op.field()
    st, stats = helm.meta_solve(op, _net(C), op.field(C["f"]), u, kind="gmres", restart=50, tol=1e-6,
                                max_iters=5000, n_r=3, omega=0.5, p_used=128, k=C["k"])
    assert st == helm.OK
    uh = to_np(u).reshape(C["f"].shape)
    rel = np.linalg.norm(op_or.residual(uh, C["f"], s, C["mask"])) / np.linalg.norm(C["f"])
    assert rel <= 1e-6 and abs(rel - stats["rel_res"]) <= 1e-9
    assert np.all(uh[C["mask"].astype(bool)] == 0)


@pytest.fixture(scope="module")
def headline_instance2():
    """The headline workload's instance 2 (64^3, p = 128 trunk basis, n_r = 3,
    omega 0.5) and the oracle's coarse space and preconditioner for it."""
    from oracle import deeponet as don_or, coarse as co_or, meta as meta_or
    C = I.config2(2)
    s = op_or.coefficient(C["ksq"], C["alpha"])
    T = don_or.trunk_matrix(I.node_points(C["n"]), C["trunk"])
    cs = co_or.CoarseSpace(T, s, C["mask"], 128)
    M = meta_or.krylov_preconditioner(s, C["mask"], "jacobi", 3, 0.5, cs)
    return C, s, cs, M


@pytest.mark.parametrize("gs_passes", [2, 1])
def test_headline_forced_count_64cube(headline_instance2, gs_passes):
    """The timed configuration at full size (64^3, p = 128, c128): 10
    DeepONet-GMRES(50) steps (tol = 0) against the oracle, field parity 1e-10,
    with two and with one classical Gram-Schmidt pass per step."""
    from oracle import meta as meta_or
    C, s, cs, M = headline_instance2
    u_or, info = meta_or.krylov_meta("gmres", C["f"], np.zeros_like(C["f"]), s, C["mask"], 50, 0.0, 10, precond=M,
                                     gs_passes=gs_passes)
    op = make_op(helm, C, helm.C128)
    u = op.field()
    st, stats = helm.meta_solve(op, _net(C), op.field(C["f"]), u, kind="gmres", restart=50, tol=0.0, max_iters=10,
                                n_r=3, omega=0.5, p_used=128, k=C["k"], gs_passes=gs_passes)
    assert stats["iters"] == info["iters"] == 10 and stats["rank_used"] == cs.rank == 128
    assert rel_err(to_np(u), u_or) <= 1e-10


@pytest.mark.parametrize("gs_passes", [2, 1])
def test_headline_to_tolerance_64cube(headline_instance2, gs_passes):
    """The same to 1e-6: iteration count within 2 of the oracle's."""
    from oracle import meta as meta_or
    C, s, cs, M = headline_instance2
    _, info = meta_or.krylov_meta("gmres", C["f"], np.zeros_like(C["f"]), s, C["mask"], 50, 1e-6, 5000, precond=M,
                                  gs_passes=gs_passes)
    op = make_op(helm, C, helm.C128)
    u = op.field()
    st, stats = helm.meta_solve(op, _net(C), op.field(C["f"]), u, kind="gmres", restart=50, tol=1e-6, max_iters=5000,
                                n_r=3, omega=0.5, p_used=128, k=C["k"], gs_passes=gs_passes)
    assert st == helm.OK and info["status"] == 0
    assert abs(stats["iters"] - info["iters"]) <= 2, (stats["iters"], info["iters"])
    assert stats["rel_res"] <= 1e-6


def test_batch_first_problems_true_residuals():
    """The batched workload's first four problems (their real grids) to 1e-6."""
    Ps = I.config4(count=4)
    C0 = I.config2(0, n=(8, 8, 8))
    ops = [make_op(helm, P, helm.C128) for P in Ps]
    fs = [op.field(P["f"]) for op, P in zip(ops, Ps)]
    us = [op.field() for op in ops]
    st, stats = helm.meta_solve_batch(ops, _net(C0), fs, us, tol=1e-6, max_iters=20000, n_r=3, omega=0.5, p_used=128)
    assert st == helm.OK
    for P, u in zip(Ps, us):
        s = op_or.coefficient(P["ksq"], P["alpha"])
        uh = to_np(u).reshape(P["f"].shape)
        assert np.linalg.norm(op_or.residual(uh, P["f"], s, P["mask"])) <= 1e-6 * np.linalg.norm(P["f"])


def test_vcycle_63cube():
    """One DeepONet-MG V-cycle on the multigrid comparison's grid (63^3, 4 levels)."""
    C = I.config2(0, n=(63, 63, 63))
    C["ksq"] = np.full_like(C["ksq"], 144.0)
    s = op_or.coefficient(C["ksq"], C["alpha"])
    op = make_op(helm, C, helm.C128)
    g = np.random.default_rng(2)
    r = g.standard_normal(C["f"].shape) + 1j * g.standard_normal(C["f"].shape)
    r[C["mask"].astype(bool)] = 0
    z = to_np(helm.meta_precond(op, _net(C), op.field(r), p_used=32, omega=0.5, mg_levels=4, mg_nu=5))
    H = mg_or.Hierarchy(s, C["mask"], 4, omega=0.5, nu=5, trunk=C["trunk"], p_used=32)
    assert rel_err(z, H.precond(r.ravel())) <= 1e-10


def test_training_gradients_full_size():
    """One training step at the training workload's shapes (48^3 points, the
    8193-wide branch, the 4x256 trunk, p = 128, batch 64) against the oracle
    with the same bf16 rounding."""
    n = (48, 48, 48)
    X = I.node_points(n)
    w = np.random.default_rng([2405, 3, 1])
    branch = I.glorot_mlp([2 * 16 ** 3 + 1, 256, 256, 256, 256, 256], w)
    trunk = I.glorot_mlp([3, 256, 256, 256, 256, 128], w)
    net = helm.DeepONet(helm.C128, branch, trunk, 128, head="split_output", branch_grid=(16, 16, 16), k_input=True)
    g = np.random.default_rng(8)
    S = 64
    F = g.standard_normal((S, 8193)).astype(np.float32)
    Y = (g.standard_normal((S, X.shape[0])) + 1j * g.standard_normal((S, X.shape[0]))).astype(np.complex64)
    tr = helm.Trainer(net, X, batch=S, max_steps=1)
    tr.data(torch.as_tensor(F).cuda(), torch.as_tensor(Y).cuda())
    loss, gr = tr.grad(np.arange(S))
    f32 = lambda L: [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for W, b in L]
    L_or, gb, gt, _ = T.loss_and_grads(F.astype(np.float64), X, Y.T.astype(np.complex128), f32(branch), f32(trunk),
                                       rnd=T.bf16)
    assert abs(loss - L_or) <= 1e-3 * L_or
    for (dW, db), (eW, eb) in zip(tr.unflatten(gr, 0, 5) + tr.unflatten(gr, 1, 5), gb + gt):
        assert rel_err(dW, eW) <= 1e-2
        assert rel_err(db, eb) <= 1e-2


def test_adjoint_gradient_64cube_finite_differences():
    """The adjoint workload's pipeline on 64^3 (same recipe as 128^3): gradient
    against central differences on two directions (step 1e-4 k^2: at 1e-3 the
    O(step^2) term of this near-resonant grid is 1e-3 of the derivative)."""
    from paper_2405_12380_amd import adjoint as AD
    C = I.config5(n=(64, 64, 64))
    op = make_op(helm, C, helm.C128)
    sv = AD.Solver(op, _net(C), kind="gmres", restart=50, tol=1e-12, max_iters=40000, n_r=3, omega=0.5, p_used=128,
                   k=C["k"])
    axis, index = C["receiver"]
    f = op.field(C["f"])
    with torch.no_grad():
        ut = AD.solve(torch.as_tensor(C["ksq_true"].ravel()).cuda(), f, sv)
        d = ut.reshape(64, 64, 64)[:, :, index].contiguous().reshape(-1)
    k0 = torch.as_tensor(C["ksq"].ravel()).cuda()
    ksq = k0.clone().requires_grad_(True)
    AD.misfit(AD.solve(ksq, f, sv), d, op, axis, index).backward()
    eps = 1e-4 * 400.0
    for v in I.directions(C["n"], 2):
        vt = torch.as_tensor(v.ravel()).cuda()
        with torch.no_grad():
            Lp = AD.misfit(AD.solve(k0 + eps * vt, f, sv), d, op, axis, index).item()
            Lm = AD.misfit(AD.solve(k0 - eps * vt, f, sv), d, op, axis, index).item()
        an = float(torch.dot(ksq.grad, vt))
        assert abs((Lp - Lm) / (2 * eps) - an) <= 1e-4 * abs(an)
