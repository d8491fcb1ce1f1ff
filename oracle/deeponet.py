"""DeepONet branch/trunk inference (oracle).

Architecture (App. B): a branch network acting on the sampled input
functions and a trunk network acting on coordinates; the branch output is
split into two groups whose inner products with the trunk output give the
real and the imaginary part of the solution.

Readings taken where the paper is silent or does not match the workloads:

* both networks are MLPs, ``h <- act(h W + b)`` on hidden layers and a
  linear last layer, no scalar output bias; ``act`` is tanh in the
  workloads (the paper's CNN branch and ReLU/LeakyReLU activations belong
  to its trained networks, which are not available);
* ``split_output`` is the paper's head: branch output b in R^{2p},
  N = T b[:p] + i T b[p:];
* ``split_input`` is used when the branch output width equals p (the 2D
  workload): N = T branch(Re r) + i T branch(Im r);
* the network acts on the residual scaled to unit RMS:
  du = s N(r / s), s = ||r||_2 / sqrt(n), du = 0 when r = 0, and du is set to
  zero on scatterer nodes;
* the branch samples the (scaled) residual on its own grid: identity when
  the grids agree, otherwise trilinear interpolation at the branch grid's
  interior nodes (j+1)/(m+1) with zero ghosts (§4.2: fields are linearly
  interpolated between meshes); the wave number is appended raw when the
  network takes it.
"""
from __future__ import annotations

import numpy as np


def activation(name):
    if name == "tanh":
        return np.tanh
    if name == "relu":
        return lambda x: np.maximum(x, 0.0)
    if name == "leaky":
        return lambda x: np.where(x > 0, x, 0.01 * x)
    raise ValueError(name)


def mlp(x, layers, act="tanh"):
    """Forward pass of a fully connected network, batch-major rows."""
    f = activation(act)
    h = np.asarray(x, dtype=np.float64)
    for li, (W, b) in enumerate(layers):
        h = h @ W + b
        if li < len(layers) - 1:
            h = f(h)
    return h


def trunk_matrix(points, trunk, act="tanh"):
    """[T]_ij = T_j(x_i): the trunk evaluated at the node coordinates
    (App. C, definition of the trunk matrix)."""
    return mlp(points, trunk, act)


def sample_to(field, grid_to):
    """Interpolate a field (numpy shape) onto another grid's interior nodes,
    multilinearly, with zero ghosts.  Identity when the grids agree."""
    src = np.asarray(field)
    n_src = list(reversed(src.shape))
    if tuple(n_src) == tuple(grid_to):
        return src.copy()
    out = src
    for a in range(src.ndim):
        ax = src.ndim - 1 - a
        ns, nt = n_src[a], grid_to[a]
        xt = np.arange(1, nt + 1) / (nt + 1)
        t = xt * (ns + 1) - 1.0                      # fractional source index
        i0 = np.floor(t).astype(int)
        w = t - i0
        pad = [(0, 0)] * out.ndim
        pad[ax] = (1, 1)
        padded = np.pad(out, pad)                  # zero ghosts at -1 and ns
        lo = np.take(padded, i0 + 1, axis=ax)
        hi = np.take(padded, i0 + 2, axis=ax)
        shp = [1] * out.ndim
        shp[ax] = nt
        w = w.reshape(shp)
        out = (1.0 - w) * lo + w * hi
    return out


def infer(r, mask, T, branch, head, p, branch_grid, k=None, k_input=False, act="tanh"):
    """Full DeepONet correction du = s N(r / s) on the grid of ``r``."""
    r = np.asarray(r, dtype=np.complex128)
    nn = r.size
    s = np.linalg.norm(r) / np.sqrt(nn)
    if s == 0.0:
        return np.zeros_like(r)
    rh = r / s
    re = sample_to(rh.real, branch_grid).ravel()
    im = sample_to(rh.imag, branch_grid).ravel()
    if head == "split_input":
        b = mlp(np.stack([re, im]), branch, act)       # (2, p)
        N = T @ b[0] + 1j * (T @ b[1])
    elif head == "split_output":
        x = np.concatenate([re, im, [k]]) if k_input else np.concatenate([re, im])
        b = mlp(x[None, :], branch, act)[0]             # (2p,)
        N = T @ b[:p] + 1j * (T @ b[p:])
    else:
        raise ValueError(head)
    du = s * N.reshape(r.shape)
    du[np.asarray(mask).astype(bool)] = 0.0
    return du
