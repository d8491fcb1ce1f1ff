"""GPU parity of the DeepONet training row: bf16-MFMA loss and gradients
against the oracle's backpropagation with the same bf16 operand rounding,
Adam against the oracle's Adam, loss decrease on a learnable task, and the
export of trained weights back into the network.

Tolerances: the GPU and the oracle round the same operands to bf16; the
remaining differences are fp32 against fp64 accumulation (about 1e-6
relative over these sizes) and the rare operand whose fp32 and fp64 values
round to neighbouring bf16 numbers (one bf16 ulp, 2^-8 relative, on a small
fraction of elements).  Norm-wise gradient agreement within 5e-3 and loss
agreement within 1e-3 leave room for those and fail on any wrong term,
index or transpose (which give O(1) differences)."""
import numpy as np
import pytest
import torch

from paper_2405_12380_amd import inputs as I
from oracle import training as T, deeponet as don_or
from tests.helpers import rel_err, to_np

pytestmark = pytest.mark.gpu

helm = pytest.importorskip("paper_2405_12380_amd.helm")

NPTS = (16, 16, 16)


def _net_and_data(seed=0, n=128, P=None, npts=NPTS, trunk_w=(64, 64, 64)):
    g = np.random.default_rng([77, seed])
    branch = I.glorot_mlp([129, 64, 64, 128], g)
    trunk = I.glorot_mlp([3, *trunk_w], g, first_gain=4.0)
    X = I.node_points(npts)
    F = g.standard_normal((n, 129)).astype(np.float32)
    Y = (g.standard_normal((n, X.shape[0])) + 1j * g.standard_normal((n, X.shape[0]))).astype(np.complex64)
    return branch, trunk, X, F, Y


def _load(branch, trunk, dtype=None):
    return helm.DeepONet(dtype or helm.C128, branch, trunk, 64, head="split_output", branch_grid=(4, 4, 4),
                         k_input=True)


def _f32(layers):
    return [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for W, b in layers]


@pytest.mark.parametrize("npts,trunk_w", [(NPTS, (64, 64, 64)), ((12, 12, 12), (128, 192, 64))])
def test_grad_parity_with_bf16_oracle(npts, trunk_w):
    """Loss and every gradient against the oracle with the same bf16 roundings;
    the second case has a point count that leaves the last 128-row block half
    full and trunk layers of 128 and 192 outputs."""
    branch, trunk, X, F, Y = _net_and_data(npts=npts, trunk_w=trunk_w)
    net = _load(branch, trunk)
    tr = helm.Trainer(net, X, batch=64, max_steps=4)
    tr.data(torch.as_tensor(F).cuda(), torch.as_tensor(Y).cuda())
    idx = np.random.default_rng(5).permutation(128)[:64]
    loss, g = tr.grad(idx)
    L_or, gb, gt, _ = T.loss_and_grads(F[idx].astype(np.float64), X, Y[idx].T.astype(np.complex128),
                                       _f32(branch), _f32(trunk), rnd=T.bf16)
    assert abs(loss - L_or) <= 1e-3 * L_or
    gb_gpu = tr.unflatten(g, 0, 3)
    gt_gpu = tr.unflatten(g, 1, 3)
    for (dW, db), (eW, eb) in zip(gb_gpu + gt_gpu, gb + gt):
        assert rel_err(dW, eW) <= 5e-3, rel_err(dW, eW)
        assert rel_err(db, eb) <= 5e-3, rel_err(db, eb)
    # padded input rows carry no gradient
    flat = to_np(g)
    K, Kp, N, oW, _ = tr.layout(1, 0)
    assert np.all(flat[oW + K * N:oW + Kp * N] == 0)


def test_adam_parity():
    branch, trunk, X, F, Y = _net_and_data(1)
    net = _load(branch, trunk)
    tr = helm.Trainer(net, X, batch=64, max_steps=4, lr=1e-3)
    tr.data(torch.as_tensor(F).cuda(), torch.as_tensor(Y).cuda())
    params = T.flat_params(_f32(branch), _f32(trunk))
    params = [p.copy() for p in params]
    opt = T.Adam(params, lr=1e-3)
    g = np.random.default_rng(9)
    for step in range(3):
        grads = [g.standard_normal(p.shape) * 10.0 ** g.integers(-4, 0) for p in params]
        nb = len(branch)
        gbr = [(grads[2 * i], grads[2 * i + 1]) for i in range(nb)]
        gtr = [(grads[2 * nb + 2 * i], grads[2 * nb + 2 * i + 1]) for i in range(len(trunk))]
        tr.apply(tr.flatten([(a.astype(np.float32), b.astype(np.float32)) for a, b in gbr],
                            [(a.astype(np.float32), b.astype(np.float32)) for a, b in gtr]))
        opt.step(params, [q.astype(np.float32).astype(np.float64) for q in grads])
    got = tr.unflatten(tr.params(), 0, 3) + tr.unflatten(tr.params(), 1, 3)
    for (W, b), i in zip(got, range(0, len(params), 2)):
        assert rel_err(W, params[i]) <= 1e-6
        assert rel_err(b, params[i + 1]) <= 1e-6


def test_training_reduces_loss_on_a_teacher_task():
    """Labels from a teacher network of the same shape: the student's loss
    must fall over 48 Adam steps."""
    branch, trunk, X, F, _ = _net_and_data(2)
    gt = np.random.default_rng(3)
    tb = I.glorot_mlp([129, 64, 64, 128], gt)
    tt = I.glorot_mlp([3, 64, 64, 64], gt, first_gain=4.0)
    Tm = T.mlp_forward(X, tt)[-1]
    Bm = T.mlp_forward(F.astype(np.float64), tb)[-1]
    Y = (Tm @ Bm[:, :64].T + 1j * (Tm @ Bm[:, 64:].T)).T.astype(np.complex64)
    net = _load(branch, trunk)
    tr = helm.Trainer(net, X, batch=64, max_steps=48, lr=2e-3)
    tr.data(torch.as_tensor(F).cuda(), torch.as_tensor(Y).cuda())
    rng = np.random.default_rng(4)
    idx = np.concatenate([rng.permutation(128) for _ in range(24)])[:48 * 64]
    losses = tr.steps(idx)
    assert np.all(np.isfinite(losses))
    assert losses[-6:].mean() < 0.7 * losses[:6].mean(), losses
    ev = tr.eval(np.arange(128))
    assert ev.mean() < losses[:6].mean()


def test_export_updates_inference_and_invalidates_caches():
    branch, trunk, X, F, Y = _net_and_data(3)
    net = _load(branch, trunk)
    tr = helm.Trainer(net, X, batch=64, max_steps=4)
    tr.data(torch.as_tensor(F).cuda(), torch.as_tensor(Y).cuda())
    tr.steps(np.arange(128))
    P2 = I.random_problem(NPTS, seed=2)
    op = helm.Op(NPTS, helm.C128, P2["ksq"], P2["alpha"], P2["mask"])
    r0, Ac0 = helm.coarse_info(op, net, p_used=16)
    tr.export(net)
    Tg = to_np(net.trunk(op)).reshape(-1, 64)
    trained = tr.unflatten(tr.params(), 1, 3)
    assert rel_err(Tg, don_or.trunk_matrix(X, trained)) <= 1e-12
    r1, Ac1 = helm.coarse_info(op, net, p_used=16)
    assert rel_err(Ac1, Ac0) > 1e-6    # rebuilt from the new trunk


def test_branch_input_mode_matches_oracle_sampling():
    """DON_BRANCH_INPUT returns r/s resampled on the branch grid, then k."""
    C = I.config2(0, n=(12, 12, 12))
    net = helm.DeepONet(helm.C128, C["branch"], C["trunk"], C["p"], head="split_output", branch_grid=(16, 16, 16),
                        k_input=True)
    op = helm.Op(C["n"], helm.C128, C["ksq"], C["alpha"], C["mask"])
    x = to_np(net.branch_input(op, op.field(C["f"]), k=7.5))
    s = np.linalg.norm(C["f"]) / np.sqrt(C["f"].size)
    smp = don_or.sample_to(C["f"] / s, (16, 16, 16))
    ref = np.concatenate([smp.real.ravel(), smp.imag.ravel(), [7.5]])
    assert rel_err(x, ref) <= 1e-13


def test_trainer_rejects_unsupported_networks():
    """Trainer creation checks what the fused kernels assume: widths after the
    input multiples of 64 and <= 256, at most 8 trunk layers, p a multiple of
    64; each violation is HELM_E_INVAL."""
    g = np.random.default_rng([77, 9])
    X = I.node_points(NPTS)
    branch = I.glorot_mlp([129, 64, 64, 128], g)
    cases = [I.glorot_mlp([3] + [64] * 9 + [64], g),   # 10 trunk layers
             I.glorot_mlp([3, 96, 64], g),             # width not a multiple of 64
             I.glorot_mlp([3, 320, 64], g)]            # width above 256
    for trunk in cases:
        net = _load(branch, trunk)
        with pytest.raises(helm.HelmError) as e:
            helm.Trainer(net, X, batch=64, max_steps=2)
        assert e.value.status == helm.E_INVAL


def test_new_data_after_captured_steps():
    """Training steps are replayed from captured graphs; replacing the data
    (a larger set, new labels) must record them again: the first loss on the
    new data equals the oracle's loss at the trainer's current parameters."""
    branch, trunk, X, F, Y = _net_and_data(2, n=128)
    net = _load(branch, trunk)
    tr = helm.Trainer(net, X, batch=64, max_steps=8)
    tr.data(torch.as_tensor(F).cuda(), torch.as_tensor(Y).cuda())
    tr.steps(np.random.default_rng(1).integers(0, 128, size=64 * 8))   # captures the one- and eight-step graphs
    _, _, _, F2, Y2 = _net_and_data(3, n=256)
    tr.data(torch.as_tensor(F2).cuda(), torch.as_tensor(Y2).cuda())
    flat = tr.params()
    b_now, t_now = tr.unflatten(flat, 0, 3), tr.unflatten(flat, 1, 3)
    idx = np.random.default_rng(4).permutation(256)[:64]
    idx[0] = 255                                                            # beyond the old data
    losses = tr.steps(idx)
    L_or, _, _, _ = T.loss_and_grads(F2[idx].astype(np.float64), X, Y2[idx].T.astype(np.complex128),
                                     b_now, t_now, rnd=T.bf16)
    assert abs(losses[0] - L_or) <= 1e-3 * L_or
