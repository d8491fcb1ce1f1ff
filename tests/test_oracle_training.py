"""Pins of the training oracle (App. B network, mean relative L2 loss,
Adam): bf16 rounding against torch's conversion, every gradient against
central finite differences, Adam against its closed-form steps, the forward
against the inference oracle."""
import numpy as np
import pytest
import torch

from oracle import training as tr, deeponet as don


def _tiny(seed=0, S=3, P=7):
    g = np.random.default_rng(seed)
    def layers(widths):
        return [(g.standard_normal((a, b)) * 0.7, g.standard_normal(b) * 0.3) for a, b in zip(widths[:-1], widths[1:])]
    branch = layers([5, 4, 4, 6])
    trunk = layers([3, 4, 3])
    F = g.standard_normal((S, 5))
    X = g.random((P, 3))
    Y = g.standard_normal((P, S)) + 1j * g.standard_normal((P, S))
    return F, X, Y, branch, trunk


def test_bf16_rounding_matches_torch():
    g = np.random.default_rng(1)
    x = np.concatenate([g.standard_normal(10000) * 10.0 ** g.integers(-6, 6, 10000),
                        1.0 + np.arange(0, 16) * 2.0 ** -12,          # includes exact ties at 2^-8 steps
                        [0.0, -0.0, 1.0, -3.5, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(tr.bf16(x), ref)


def test_gradients_against_central_differences():
    F, X, Y, branch, trunk = _tiny()
    L, gb, gt, _ = tr.loss_and_grads(F, X, Y, branch, trunk)
    params = tr.flat_params(branch, trunk)
    grads = tr.flat_grads(gb, gt)
    eps = 1e-6
    worst = 0.0
    for p, gp in zip(params, grads):
        for idx in np.ndindex(p.shape):
            old = p[idx]
            p[idx] = old + eps
            Lp = tr.loss_and_grads(F, X, Y, branch, trunk)[0]
            p[idx] = old - eps
            Lm = tr.loss_and_grads(F, X, Y, branch, trunk)[0]
            p[idx] = old
            worst = max(worst, abs((Lp - Lm) / (2 * eps) - gp[idx]))
    scale = max(np.abs(g).max() for g in grads)
    assert worst <= 1e-7 * scale


def test_adam_closed_form_steps():
    g = np.random.default_rng(2)
    p = [g.standard_normal((4, 3)), g.standard_normal(3)]
    grads = [g.standard_normal((4, 3)), g.standard_normal(3)]
    opt = tr.Adam([q.copy() for q in p], lr=1e-3)
    cur = [q.copy() for q in p]
    for t in range(5):
        before = [q.copy() for q in cur]
        opt.step(cur, grads)
        # constant gradient: m_hat = g and v_hat = g^2 at every step
        for b, a, gg in zip(before, cur, grads):
            assert np.allclose(a - b, -1e-3 * gg / (np.abs(gg) + 1e-8), rtol=1e-12, atol=1e-18)


def test_forward_matches_inference_oracle_and_exact_labels():
    F, X, Y, branch, trunk = _tiny(3)
    hs = tr.mlp_forward(X, trunk)
    assert np.abs(hs[-1] - don.trunk_matrix(X, trunk)).max() <= 1e-15
    T = hs[-1]
    B = tr.mlp_forward(F, branch)[-1]
    U = T @ B[:, :3].T + 1j * (T @ B[:, 3:].T)
    assert tr.relative_l2(F, X, U, branch, trunk) == 0.0
    # scale invariance of the relative loss in (U, Y) jointly
    L1 = tr.loss_and_grads(F, X, Y, branch, trunk)[0]
    assert L1 > 0


def test_rounded_gradients_close_to_exact():
    """With bf16 operands the gradients move by the bf16 unit roundoff scale only."""
    F, X, Y, branch, trunk = _tiny(4, S=4, P=40)
    _, gb, gt, _ = tr.loss_and_grads(F, X, Y, branch, trunk)
    _, gb2, gt2, _ = tr.loss_and_grads(F, X, Y, branch, trunk, rnd=tr.bf16)
    for a, b in zip(tr.flat_grads(gb, gt), tr.flat_grads(gb2, gt2)):
        assert np.linalg.norm(a - b) <= 0.05 * np.linalg.norm(a) + 1e-12
