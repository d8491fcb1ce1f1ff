"""Seeded synthetic inputs for the Helmholtz scattering workloads.

This module generates *data only*: grid coordinates, the wave-number and
sponge coefficient fields, scatterer masks, source terms and network weights.
It holds none of the solver's arithmetic and is the one module that both the
GPU path (through tests and the benchmark) and the CPU oracle's tests draw
their inputs from.

Conventions (shared by every consumer):

* A grid is described by ``n = (nx, ny)`` or ``(nx, ny, nz)`` interior nodes.
  Node ``i`` on axis ``a`` sits at ``x = (i + 1) * h_a`` with
  ``h_a = 1 / (n_a + 1)``; the nodes ``i = -1`` and ``i = n_a`` are zero
  ghosts behind the sponge.
* Fields are numpy arrays of shape ``(nz, ny, nx)`` (3D) or ``(ny, nx)`` (2D)
  in C order, so flattening gives the x-fastest node order
  ``p = i + nx * (j + ny * l)``.
* Random streams come from ``numpy.random.default_rng([2405, config, instance])``.
"""
from __future__ import annotations

import os

import numpy as np

SPONGE_WIDTH = 8
SPONGE_ALPHA_MAX = 1.0
MASK_SLACK = 1e-12


def rng_for(config_id: int, instance: int = 0) -> np.random.Generator:
    return np.random.default_rng([2405, int(config_id), int(instance)])


def field_shape(n) -> tuple:
    """numpy shape (z, y, x) / (y, x) of a grid with interior sizes ``n`` (x first)."""
    return tuple(int(v) for v in reversed(tuple(n)))


def axis_coords(n) -> list:
    """Interior node coordinates per axis, x first: ``(i + 1) / (n_a + 1)``."""
    return [np.arange(1, na + 1, dtype=np.float64) / (na + 1) for na in n]


def mesh(n) -> list:
    """Coordinate arrays (X, Y[, Z]) each of the field shape."""
    c = axis_coords(n)
    grids = np.meshgrid(*reversed(c), indexing="ij")  # z, y, x order
    return list(reversed(grids))  # X, Y, Z


def node_points(n) -> np.ndarray:
    """(N, dim) array of node coordinates in flattened x-fastest order."""
    return np.stack([g.ravel() for g in mesh(n)], axis=1)


def sponge(n, width: int = SPONGE_WIDTH, amax: float = SPONGE_ALPHA_MAX) -> np.ndarray:
    """Absorbing-layer profile alpha(x).

    With ``d`` the smallest index distance of a node to the outermost interior
    layer, ``d = min_a min(i_a, n_a - 1 - i_a)``, alpha is
    ``amax * ((width - d) / width)**2`` for ``d < width`` and 0 inside.  It is
    ``amax`` on the outermost nodes and decays quadratically inward.
    """
    dist = None
    for a, na in enumerate(n):
        i = np.arange(na)
        da = np.minimum(i, na - 1 - i)
        shape = [1] * len(n)
        shape[len(n) - 1 - a] = na
        da = da.reshape(shape)
        dist = da if dist is None else np.minimum(dist, da)
    dist = np.broadcast_to(dist, field_shape(n)).astype(np.float64)
    return np.where(dist < width, amax * ((width - dist) / width) ** 2, 0.0)


def box_mask(n, center, half) -> np.ndarray:
    """uint8 indicator of the closed axis-aligned box |x_a - c_a| <= half_a."""
    X = mesh(n)
    half = np.broadcast_to(np.asarray(half, dtype=np.float64), (len(n),))
    m = np.ones(field_shape(n), dtype=bool)
    for a in range(len(n)):
        m &= np.abs(X[a] - center[a]) <= half[a] + MASK_SLACK
    return m.astype(np.uint8)


def ellipsoid_mask(n, center, semi) -> np.ndarray:
    X = mesh(n)
    q = sum(((X[a] - center[a]) / semi[a]) ** 2 for a in range(len(n)))
    return (q <= 1.0 + MASK_SLACK).astype(np.uint8)


def capsule_sail_mask(n, x_range=(0.2, 0.8), radius=0.08, axis_yz=(0.5, 0.5),
                      sail=((0.45, 0.55), (0.48, 0.52), (0.58, 0.66))) -> np.ndarray:
    """Submarine-like body: a capsule along x (cylinder plus hemispherical caps)
    and a box sail on top."""
    X, Y, Z = mesh(n)
    r2 = (Y - axis_yz[0]) ** 2 + (Z - axis_yz[1]) ** 2
    xc = np.clip(X, x_range[0], x_range[1])
    d2 = (X - xc) ** 2 + r2
    m = d2 <= radius ** 2 + MASK_SLACK
    (x0, x1), (y0, y1), (z0, z1) = sail
    m |= ((X >= x0 - MASK_SLACK) & (X <= x1 + MASK_SLACK) & (Y >= y0 - MASK_SLACK)
          & (Y <= y1 + MASK_SLACK) & (Z >= z0 - MASK_SLACK) & (Z <= z1 + MASK_SLACK))
    return m.astype(np.uint8)


def gaussian_source(n, x0, sigma) -> np.ndarray:
    X = mesh(n)
    r2 = sum((X[a] - x0[a]) ** 2 for a in range(len(n)))
    return np.exp(-r2 / (2.0 * sigma ** 2)).astype(np.complex128)


def grf(n, length: float, rng: np.random.Generator, workers: int | None = None) -> np.ndarray:
    """Zero-mean, unit-variance Gaussian random field with covariance
    ``exp(-r^2 / (2 l^2))`` sampled at the grid's nodes.

    White noise on a periodic grid twice the size (same spacing) is convolved
    with ``exp(-|x|^2 / l^2)``; the autocorrelation of that kernel is the
    target covariance.  The result is divided by the kernel's l2 norm (the
    exact standard deviation) and cropped to the interior nodes.  With
    ``workers`` the FFTs run multi-threaded (scipy.fft; the same field up to
    rounding in the last bits).
    """
    h = [1.0 / (na + 1) for na in n]
    big = [2 * na for na in n]
    shape = tuple(reversed(big))
    noise = rng.standard_normal(shape)
    ker = np.ones(shape)
    for a, (na, ha) in enumerate(zip(big, h)):
        i = np.arange(na)
        d = np.minimum(i, na - i) * ha
        s = [1] * len(n)
        s[len(n) - 1 - a] = na
        ker = ker * np.exp(-(d ** 2) / length ** 2).reshape(s)
    axes = list(range(len(shape)))
    if workers:
        import scipy.fft as sfft
        fld = sfft.irfftn(sfft.rfftn(noise, axes=axes, workers=workers) * sfft.rfftn(ker, axes=axes, workers=workers),
                          s=shape, axes=axes, workers=workers)
    else:
        fld = np.fft.irfftn(np.fft.rfftn(noise, axes=axes) * np.fft.rfftn(ker, axes=axes), s=shape, axes=axes)
    fld /= np.sqrt(np.sum(ker ** 2))
    sl = tuple(slice(0, na) for na in reversed(n))
    return np.ascontiguousarray(fld[sl])


def complex_grf(n, length: float, rng: np.random.Generator, workers: int | None = None) -> np.ndarray:
    """Re and Im drawn independently from the same field (App. B)."""
    re = grf(n, length, rng, workers)
    im = grf(n, length, rng, workers)
    return (re + 1j * im).astype(np.complex128)


def glorot_mlp(widths, rng: np.random.Generator, first_gain: float = 1.0):
    """Layers ``[(W, b), ...]`` with ``W`` of shape (fan_in, fan_out), drawn
    Glorot-uniform ``U(+-sqrt(6 / (fan_in + fan_out)))`` in layer order, zero
    biases.  ``first_gain`` scales the first layer's weights."""
    layers = []
    for li, (fi, fo) in enumerate(zip(widths[:-1], widths[1:])):
        lim = np.sqrt(6.0 / (fi + fo))
        W = rng.uniform(-lim, lim, size=(fi, fo))
        if li == 0:
            W = W * first_gain
        layers.append((W.astype(np.float64), np.zeros(fo, dtype=np.float64)))
    return layers


# --------------------------------------------------------------------------
# Workloads.  Each returns a plain dict of numpy arrays and scalars.
# --------------------------------------------------------------------------

def config1() -> dict:
    """2D parity case: 64 x 64 grid, k = 10, 8-cell sponge, square scatterer of
    side 0.2 at the centre, Gaussian source (sigma 0.05) at (0.25, 0.5), and a
    Glorot-initialised DeepONet (branch 4096-128-128-64, trunk 2-128-128-64,
    tanh, seed 0) whose branch is applied to Re and Im of the residual."""
    n = (64, 64)
    k = 10.0
    mask = box_mask(n, (0.5, 0.5), 0.1)
    alpha = sponge(n)
    ksq = np.full(field_shape(n), k * k)
    f = gaussian_source(n, (0.25, 0.5), 0.05)
    f[mask.astype(bool)] = 0
    g = np.random.default_rng(0)
    branch = glorot_mlp([4096, 128, 128, 64], g)
    trunk = glorot_mlp([2, 128, 128, 64], g)
    return dict(n=n, k=k, ksq=ksq, alpha=alpha, mask=mask, f=f,
                branch=branch, trunk=trunk, head="split_input", p=64,
                branch_grid=n, k_input=False)


def config2(instance: int = 0, n=(64, 64, 64), trunk_gain: float = 30.0) -> dict:
    """3D headline case: 64^3 grid, homogeneous k ~ U[5, 15], 8-cell sponge,
    cube scatterer of side 0.25 centred at c ~ U[0.25, 0.75]^3, complex GRF
    source (l = 0.1) zeroed on the scatterer, trunk 3-256x4-128 (tanh,
    first-layer gain ``trunk_gain``) for the p = 128 trunk basis."""
    g = rng_for(2, instance)
    k = float(g.uniform(5.0, 15.0))
    c = g.uniform(0.25, 0.75, size=3)
    mask = box_mask(n, c, 0.125)
    alpha = sponge(n)
    ksq = np.full(field_shape(n), k * k)
    f = complex_grf(n, 0.1, g)
    f[mask.astype(bool)] = 0
    w = np.random.default_rng([2405, 3, 0])
    branch = glorot_mlp([2 * 16 ** 3 + 1, 256, 256, 256, 256, 256], w)
    trunk = glorot_mlp([3, 256, 256, 256, 256, 128], w, first_gain=trunk_gain)
    return dict(n=tuple(n), k=k, ksq=ksq, alpha=alpha, mask=mask, f=f, center=c,
                branch=branch, trunk=trunk, head="split_output", p=128,
                branch_grid=(16, 16, 16), k_input=True)


def random_problem(n, seed: int, mask_frac: float = 0.05, k=None) -> dict:
    """Generic stress input: random complex fields with U(-1, 1) parts, the
    sponge, a homogeneous k and a random scattered mask."""
    g = np.random.default_rng([2405, 99, seed])
    shp = field_shape(n)
    if k is None:
        k = float(g.uniform(5.0, 15.0))
    mask = (g.random(shp) < mask_frac).astype(np.uint8)
    x = g.uniform(-1, 1, shp) + 1j * g.uniform(-1, 1, shp)
    f = g.uniform(-1, 1, shp) + 1j * g.uniform(-1, 1, shp)
    return dict(n=tuple(n), k=k, ksq=np.full(shp, k * k), alpha=sponge(n), mask=mask,
                x=x.astype(np.complex128), f=f.astype(np.complex128))


def config3(count: int, instance: int = 0, n=(48, 48, 48), k_range=(5.0, 15.0), device="cuda"):
    """Training set of App. B: ``count`` non-scattering problems on one grid
    (48^3), homogeneous k ~ U[5, 15], 8-cell sponge, complex GRF sources
    (l = 0.1) scaled to unit RMS (so a network trained on (f, u) sees the same
    scaling as the meta-solver's r / s).  The many sources are drawn on the
    GPU with torch's seeded generator (the same FFT filtering as ``grf``);
    returns (k array, alpha, f as a count x n complex128 torch tensor)."""
    import torch
    g = rng_for(3, instance)
    ks = g.uniform(*k_range, size=count)
    n = tuple(int(v) for v in n)
    alpha = sponge(n)
    shape = tuple(reversed([2 * a for a in n]))
    h = [1.0 / (a + 1) for a in n]
    ker = np.ones(shape)
    for a, (na, ha) in enumerate(zip([2 * v for v in n], h)):
        i = np.arange(na)
        d = np.minimum(i, na - i) * ha
        sh = [1] * len(n)
        sh[len(n) - 1 - a] = na
        ker = ker * np.exp(-(d ** 2) / 0.1 ** 2).reshape(sh)
    kt = torch.as_tensor(ker, device=device)
    kf = torch.fft.rfftn(kt)
    knorm = float(np.sqrt(np.sum(ker ** 2)))
    tg = torch.Generator(device=device)
    tg.manual_seed(int(g.integers(0, 2 ** 62)))
    out = torch.empty((count,) + tuple(reversed(n)), dtype=torch.complex128, device=device)
    sl = tuple(slice(0, a) for a in reversed(n))
    chunk = 32
    for c0 in range(0, count, chunk):
        c1 = min(count, c0 + chunk)
        for part in (0, 1):
            noise = torch.randn((c1 - c0,) + shape, generator=tg, device=device, dtype=torch.float64)
            fld = torch.fft.irfftn(torch.fft.rfftn(noise, dim=(1, 2, 3)) * kf, s=shape, dim=(1, 2, 3)) / knorm
            fld = fld[(slice(None),) + sl]
            if part == 0:
                out[c0:c1].real = fld
            else:
                out[c0:c1].imag = fld
    rms = torch.sqrt(torch.mean(torch.abs(out.reshape(count, -1)) ** 2, dim=1))
    out /= rms.reshape((count,) + (1,) * len(n))
    return ks, alpha, out.reshape(count, -1)


def config4(count: int = 64, instance: int = 0, n_range=(48, 128), k_range=(5.0, 25.0)) -> list:
    """Batched case: ``count`` independent cubic problems, n ~ U{48..128}
    nodes per axis, homogeneous k ~ U[5, 25], a sponge of max(8, n / 8) cells
    (as in ``config5``: at least 1/8 of the domain, so the k = 25 waves on the
    finest grids are absorbed rather than reflected), a cube
    (half-side ~ U[0.1, 0.3]) or an ellipsoid (semi-axes ~ U[0.1, 0.3]) with
    probability 1/2 each, complex GRF source (l = 0.1) zeroed on the scatterer.

    The centre is drawn per axis so that the scatterer stays out of the sponge
    (nodes with index distance below the sponge width); where that interval is
    empty the centre is 0.5."""
    g = rng_for(4, instance)
    out = []
    for _ in range(count):
        n1 = int(g.integers(n_range[0], n_range[1] + 1))
        n = (n1, n1, n1)
        k = float(g.uniform(*k_range))
        ellipsoid = bool(g.random() < 0.5)
        ext = g.uniform(0.1, 0.3, size=3) if ellipsoid else np.full(3, g.uniform(0.1, 0.3))
        h = 1.0 / (n1 + 1)
        width = max(SPONGE_WIDTH, n1 // 8)
        lo_free, hi_free = (width + 1) * h, (n1 - width) * h
        c = np.empty(3)
        for a in range(3):
            lo, hi = lo_free + ext[a], hi_free - ext[a]
            c[a] = g.uniform(lo, hi) if lo < hi else 0.5
        mask = ellipsoid_mask(n, c, ext) if ellipsoid else box_mask(n, c, ext[0])
        f = complex_grf(n, 0.1, g, workers=min(os.cpu_count() or 1, 16))
        f[mask.astype(bool)] = 0
        out.append(dict(n=n, k=k, ksq=np.full(field_shape(n), k * k), alpha=sponge(n, width=width), mask=mask, f=f,
                        shape="ellipsoid" if ellipsoid else "cube", center=c, extent=ext))
    return out


def config5(n=(128, 128, 128), instance: int = 0, k: float = 20.0, perturb: float = 0.05,
            trunk_gain: float = 30.0, sponge_width=None) -> dict:
    """Adjoint case: homogeneous k = 20, submarine-like scatterer (capsule
    along x plus sail), plane wave incident from the top.

    * The sponge is max(8, n_z / 8) cells wide: at least 8 cells and at least
      1/8 of the domain (an 8-cell layer on a 128^3 grid is too thin to absorb
      the k = 20 wave, and the solves stall on the reflections).

    * The incident wave is a sheet source of real unit amplitude per unit area
      (value 1/h_z) on the first z-plane below the top sponge (index
      n_z - 1 - width), zeroed on the scatterer; it radiates a plane
      wave travelling in -z, the upward half being absorbed by the sponge.
    * Receivers: the x-plane nearest x = 0.9 (``receiver = (axis 0, index)``).
    * ``ksq_true = k^2 (1 + perturb g)`` with g a GRF (l = 0.2) scaled to
      max |g| = 1: the medium that generates the synthetic data.
    * The network is config 2's (same weights stream).
    * ``sponge_width`` overrides the width (for the record of what a thinner
      layer does).
    """
    g = rng_for(5, instance)
    n = tuple(int(v) for v in n)
    shp = field_shape(n)
    mask = capsule_sail_mask(n)
    width = max(SPONGE_WIDTH, n[-1] // 8) if sponge_width is None else int(sponge_width)
    alpha = sponge(n, width=width)
    ksq = np.full(shp, k * k)
    f = np.zeros(shp, dtype=np.complex128)
    zs = n[-1] - 1 - width
    f[zs] = float(n[-1] + 1)
    f[mask.astype(bool)] = 0
    pert = grf(n, 0.2, g)
    pert /= np.max(np.abs(pert))
    ksq_true = ksq * (1.0 + perturb * pert)
    rx = int(min(max(round(0.9 * (n[0] + 1)) - 1, 0), n[0] - 1))
    w = np.random.default_rng([2405, 3, 0])
    branch = glorot_mlp([2 * 16 ** 3 + 1, 256, 256, 256, 256, 256], w)
    trunk = glorot_mlp([3, 256, 256, 256, 256, 128], w, first_gain=trunk_gain)
    return dict(n=n, k=k, ksq=ksq, alpha=alpha, mask=mask, f=f, ksq_true=ksq_true, receiver=(0, rx),
                source_plane=zs, sponge_width=width, branch=branch, trunk=trunk, head="split_output", p=128,
                branch_grid=(16, 16, 16), k_input=True)


def directions(n, count: int, instance: int = 0, length: float = 0.2) -> list:
    """Seeded smooth perturbation directions for finite-difference checks of a
    k^2 gradient: GRFs (length scale ``length``) scaled to max |v| = 1."""
    g = rng_for(55, instance)
    out = []
    for _ in range(count):
        v = grf(tuple(n), length, g)
        out.append(v / np.max(np.abs(v)))
    return out
