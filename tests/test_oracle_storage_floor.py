"""The complex64 path stores every field in fp32 (arithmetic in fp64).  On an
iteration that diverges, each storage rounding is amplified, so the path's
agreement with the complex128 oracle is limited by a floor that no kernel can
beat.  This file measures that floor for the relaxation meta-solver of config
1 (iii) (eq. 3, network correction every 25 sweeps, 200 sweeps): the oracle's
own steps with every stored field (iterate, residual, network input, layer
outputs, trunk matrix, correction) rounded to fp32, against the same steps
unrounded.

* The seeded Glorot network multiplies the residual by about 400 per
  correction and drives |u| to ~1e9: the fp32 floor is about 2e-5 (Jacobi)
  and 1e-4 (red-black Gauss-Seidel), so the GPU's complex64 parity for that
  fixture is bounded by the floor (2e-4), not by the 2e-5 contract.
* The same network with its output layer scaled by 1e-3 keeps the residual
  below 1: the floor is below 1e-6, and the contract's 2e-5 applies."""
import numpy as np
import pytest

from paper_2405_12380_amd import inputs as I
from oracle import operator as op, meta, deeponet as don


def _c64(a):
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


def _r32(a):
    return np.asarray(a).astype(np.float32).astype(np.float64)


def _mlp32(x, layers):
    h = _r32(x)
    for li, (W, b) in enumerate(layers):
        h = h @ W + b
        if li < len(layers) - 1:
            h = np.tanh(h)
        h = _r32(h)
    return h


def storage_floor(kind, out_scale):
    C = I.config1()
    s = _c64(op.coefficient(C["ksq"], C["alpha"]))
    f = _c64(C["f"])
    mask = C["mask"]
    wb = [(_r32(W), _r32(b)) for W, b in C["branch"]]
    wb[-1] = (_r32(wb[-1][0] * out_scale), _r32(wb[-1][1] * out_scale))
    wt = [(_r32(W), _r32(b)) for W, b in C["trunk"]]
    T = don.trunk_matrix(I.node_points(C["n"]), wt)
    exact = meta.deeponet_correction(s, mask, T, dict(branch=wb, head="split_input", p=C["p"], branch_grid=C["n"]))
    u_ex, _ = meta.relaxation_meta(f, np.zeros_like(f), s, mask, kind, 0.5, 200, 25, 0.0, correction=exact)
    T32 = _r32(T)

    def corr32(r):
        sc = np.linalg.norm(r) / np.sqrt(r.size)
        x = r / sc
        br = _mlp32(x.real.ravel()[None, :], wb)[0]
        bi = _mlp32(x.imag.ravel()[None, :], wb)[0]
        du = _c64(sc * (T32 @ br + 1j * (T32 @ bi))).reshape(r.shape)
        du[mask.astype(bool)] = 0
        return du

    u = np.zeros_like(f)
    for _ in range(8):
        for _ in range(25):
            u = _c64(meta.sweep(kind, u, f, s, mask, 0.5))
        u = _c64(u + corr32(_c64(op.residual(u, f, s, mask))))
    return np.linalg.norm(u - u_ex) / np.linalg.norm(u_ex)


@pytest.mark.parametrize("kind", ["jacobi", "rbgs"])
def test_fp32_storage_floor_of_config1_relaxation(kind):
    seeded = storage_floor(kind, 1.0)
    damped = storage_floor(kind, 1e-3)
    assert 1e-5 <= seeded <= 2e-4, seeded      # the divergent fixture's floor: above the contract
    assert damped <= 1e-6, damped              # the damped fixture: far below it
