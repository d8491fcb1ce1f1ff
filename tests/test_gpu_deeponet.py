"""GPU parity of the DeepONet rows: trunk evaluation (MFMA GEMMs) and the full
correction du = s N(r / s) with both output heads and branch resampling."""
import numpy as np
import pytest

from paper_2405_12380_amd import inputs as I
from oracle import deeponet as don_or
from tests.helpers import make_op, rel_err, stored_layers, to_np

pytestmark = pytest.mark.gpu

helm = pytest.importorskip("paper_2405_12380_amd.helm")


@pytest.mark.parametrize("dtype", [helm.C128, helm.C64])
def test_trunk_c1(dtype):
    C = I.config1()
    op = make_op(helm, C, dtype)
    net = helm.DeepONet(dtype, C["branch"], C["trunk"], C["p"], head="split_input", branch_grid=C["n"])
    T = to_np(net.trunk(op)).reshape(-1, C["p"])
    # fp64 arithmetic for both dtypes; C64 stores fp32 weights and rounds T once
    ref = don_or.trunk_matrix(I.node_points(C["n"]), stored_layers(C["trunk"], dtype == helm.C64))
    assert rel_err(T, ref) <= (1e-13 if dtype == helm.C128 else 1e-6)


@pytest.mark.parametrize("n", [(24, 24, 24), (33, 17, 9)])
def test_trunk_3d_config_shape(n):
    """3-256x4-128 trunk (first-layer gain 30), ragged node count (not a
    multiple of the 64-row tile)."""
    C = I.config2(0, n=n)
    op = make_op(helm, C, helm.C128)
    net = helm.DeepONet(helm.C128, C["branch"], C["trunk"], C["p"], head="split_output", branch_grid=(16, 16, 16),
                        k_input=True)
    T = to_np(net.trunk(op)).reshape(-1, C["p"])
    ref = don_or.trunk_matrix(I.node_points(C["n"]), C["trunk"])
    assert rel_err(T, ref) <= 1e-12


@pytest.mark.parametrize("widths", [[3, 38, 22, 10], [3, 37, 29, 12]])
def test_trunk_ragged_widths(widths):
    """Layer widths that are not multiples of the GEMM tiles or of the 16-deep
    k chunk: even widths (rows 16-byte aligned) take the register-A product
    with a partial last k chunk and partial column tiles, odd widths the
    LDS-staged one; nonzero biases.  Against the oracle's trunk matrix."""
    n = (21, 13, 11)
    C = I.config2(0, n=n)
    g = np.random.default_rng(11)
    trunk = [(W, g.standard_normal(W.shape[1]) * 0.1) for W, _ in I.glorot_mlp(widths, g, first_gain=3.0)]
    p = widths[-1]
    branch = I.glorot_mlp([2 * 16 ** 3 + 1, 24, 2 * p], g)
    op = make_op(helm, C, helm.C128)
    net = helm.DeepONet(helm.C128, branch, trunk, p, head="split_output", branch_grid=(16, 16, 16), k_input=True)
    T = to_np(net.trunk(op)).reshape(-1, p)
    ref = don_or.trunk_matrix(I.node_points(C["n"]), trunk)
    assert rel_err(T, ref) <= 1e-13


@pytest.mark.parametrize("dtype", [helm.C128, helm.C64])
def test_full_split_input_c1(dtype):
    C = I.config1()
    op = make_op(helm, C, dtype)
    net = helm.DeepONet(dtype, C["branch"], C["trunk"], C["p"], head="split_input", branch_grid=C["n"])
    g = np.random.default_rng(5)
    r = (g.standard_normal(I.field_shape(C["n"])) + 1j * g.standard_normal(I.field_shape(C["n"]))) * 3.0
    r[C["mask"].astype(bool)] = 0
    if dtype == helm.C64:
        r = r.astype(np.complex64).astype(np.complex128)
    du = to_np(net.full(op, op.field(r)))
    lo = dtype == helm.C64
    T = don_or.trunk_matrix(I.node_points(C["n"]), stored_layers(C["trunk"], lo))
    ref = don_or.infer(r, C["mask"], T, stored_layers(C["branch"], lo), "split_input", C["p"], C["n"])
    assert rel_err(du, ref) <= (1e-12 if dtype == helm.C128 else 1e-6)
    assert np.all(du[C["mask"].ravel().astype(bool)] == 0)


@pytest.mark.parametrize("n,bg", [((20, 20, 20), (8, 8, 8)), ((13, 11, 9), (6, 5, 4)), ((8, 8, 8), (8, 8, 8))])
def test_full_split_output_sampled(n, bg):
    g = np.random.default_rng(11)
    p = 16
    m = int(np.prod(bg))
    branch = I.glorot_mlp([2 * m + 1, 32, 2 * p], g)
    trunk = I.glorot_mlp([3, 32, p], g, first_gain=5.0)
    P = I.random_problem(n, 12, mask_frac=0.1)
    op = make_op(helm, P, helm.C128)
    net = helm.DeepONet(helm.C128, branch, trunk, p, head="split_output", branch_grid=bg, k_input=True)
    r = P["x"] * 2.5
    du = to_np(net.full(op, op.field(r), k=7.5))
    T = don_or.trunk_matrix(I.node_points(n), trunk)
    ref = don_or.infer(r, P["mask"], T, branch, "split_output", p, bg, k=7.5, k_input=True)
    assert rel_err(du, ref) <= 1e-12


def test_full_zero_residual():
    C = I.config1()
    op = make_op(helm, C, helm.C128)
    net = helm.DeepONet(helm.C128, C["branch"], C["trunk"], C["p"], head="split_input", branch_grid=C["n"])
    du = to_np(net.full(op, op.field()))
    assert np.all(du == 0)


def test_load_rejects_bad_shapes():
    C = I.config1()
    with pytest.raises(helm.HelmError):
        helm.DeepONet(helm.C128, C["branch"], C["trunk"], C["p"] + 1, head="split_input", branch_grid=C["n"])
    with pytest.raises(helm.HelmError):
        helm.DeepONet(helm.C128, C["branch"], C["trunk"], C["p"], head="split_output", branch_grid=C["n"])
