"""DeepONet training step (oracle), App. B.

The network of App. B (branch MLP on the sampled source plus k, trunk MLP on
the node coordinates, branch output split into the groups that give the real
and the imaginary part) is trained on pairs (f, u) of non-scattering solves
with the mean relative L2 loss and Adam.

Definitions (batch of S samples, P points, p trunk outputs):

* forward: T = trunk(X) (P x p), B = branch(F) (S x 2p);
  U_re = T B[:, :p]^T, U_im = T B[:, p:]^T (P x S each);
* loss L = (1/S) sum_s ||U_s - Y_s||_2 / ||Y_s||_2 over the complex values
  of sample s;
* gradients by the chain rule (backpropagation), written out per layer;
* Adam (Kingma & Ba): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
  theta <- theta - lr m_hat / (sqrt(v_hat) + eps) with m_hat = m / (1 - b1^t),
  v_hat = v / (1 - b2^t).

``rnd`` (optional) is applied wherever a tensor becomes a matrix-product
operand, mirroring a kernel that multiplies in a narrower format: for
bfloat16 operands with fp32 accumulation pass ``bf16``; the products and
everything else are fp64 here.

Readings: hidden layers tanh, linear output layers, biases on every layer,
no output bias; the loss is the relative L2 norm per sample (not squared),
averaged over the batch.

TEST INFRASTRUCTURE ONLY, like the rest of this package.
"""
from __future__ import annotations

import numpy as np


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (round to nearest, ties to even) through fp32, and
    return the values as float64."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = x32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = ((bits + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return bits.view(np.float32).astype(np.float64)


def _id(x):
    return np.asarray(x, dtype=np.float64)


def mlp_forward(x, layers, rnd=None):
    """Returns the list of layer inputs H_0..H_L (H_L = output).  Hidden
    layers: H_{l+1} = tanh(H_l W_l + b_l); last layer linear."""
    r = rnd or _id
    hs = [r(x)]
    for li, (W, b) in enumerate(layers):
        z = r(hs[-1]) @ r(W) + b
        hs.append(r(np.tanh(z)) if li < len(layers) - 1 else r(z))
    return hs


def mlp_backward(hs, layers, d_out, rnd=None):
    """Gradients (dW, db) of every layer given dL/d(output); hs from
    mlp_forward.  The derivative of tanh is 1 - tanh^2, taken at the stored
    activation."""
    r = rnd or _id
    grads = [None] * len(layers)
    dz = r(d_out)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        grads[li] = (r(hs[li]).T @ dz, dz.sum(axis=0))
        if li > 0:
            dh = dz @ r(W).T
            dz = r(dh * (1.0 - hs[li] ** 2))
    return grads


def loss_and_grads(F, X, Y, branch, trunk, rnd=None):
    """Mean relative L2 loss of a batch and its gradients.

    F: S x K_b branch inputs; X: P x d trunk inputs; Y: P x S complex labels.
    Returns (L, branch grads, trunk grads, U) with U the P x S prediction."""
    r = rnd or _id
    hb = mlp_forward(F, branch, rnd)
    ht = mlp_forward(X, trunk, rnd)
    T, B = ht[-1], hb[-1]
    S = B.shape[0]
    p = T.shape[1]
    Bc = np.concatenate([B[:, :p], B[:, p:]], axis=0)          # 2S x p: Re rows, then Im rows
    Uc = r(T) @ r(Bc).T                                          # P x 2S
    U = Uc[:, :S] + 1j * Uc[:, S:]
    D = U - Y
    dn = np.linalg.norm(D, axis=0)
    yn = np.linalg.norm(Y, axis=0)
    L = float(np.mean(dn / yn))
    w = 1.0 / (S * dn * yn)
    dUc = np.concatenate([D.real * w, D.imag * w], axis=1)      # dL/dUc
    dUr = r(dUc)
    dT = dUr @ r(Bc)                                             # P x p
    dBc = dUr.T @ r(T)                                           # 2S x p
    dB = np.concatenate([dBc[:S], dBc[S:]], axis=1)              # S x 2p
    gb = mlp_backward(hb, branch, dB, rnd)
    gt = mlp_backward(ht, trunk, dT, rnd)
    return L, gb, gt, U


def relative_l2(F, X, Y, branch, trunk):
    """Mean relative L2 error of the network on (F, Y), fp64."""
    T = mlp_forward(X, trunk)[-1]
    B = mlp_forward(F, branch)[-1]
    p = T.shape[1]
    U = T @ B[:, :p].T + 1j * (T @ B[:, p:].T)
    return float(np.mean(np.linalg.norm(U - Y, axis=0) / np.linalg.norm(Y, axis=0)))


class Adam:
    """Adam on a list of arrays (updated in place)."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.b1
            m += (1.0 - self.b1) * g
            v *= self.b2
            v += (1.0 - self.b2) * g * g
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


def flat_params(branch, trunk):
    """The trainable arrays in a fixed order: branch (W, b) per layer, then trunk."""
    out = []
    for W, b in list(branch) + list(trunk):
        out += [W, b]
    return out


def flat_grads(gb, gt):
    out = []
    for dW, db in list(gb) + list(gt):
        out += [dW, db]
    return out
