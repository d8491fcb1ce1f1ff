"""helm_relax_noalloc (static scratch, no allocation) against helm_relax:
the same sweeps bit for bit, on two calls in a row with the second on a
smaller grid, both relaxation kinds and both dtypes, called through the C ABI;
and the size limit of the static scratch."""
import ctypes as C

import numpy as np
import pytest

from paper_2405_12380_amd import inputs as I
from oracle import operator as op_or
from tests.helpers import make_op, rel_err, to_np

pytestmark = pytest.mark.gpu

helm = pytest.importorskip("paper_2405_12380_amd.helm")


def _run(n, seed, dtype, kind, sweeps, omega):
    P = I.random_problem(n, seed)
    op = make_op(helm, P, dtype)
    lo = dtype == helm.C64
    u0 = P["x"].astype(np.complex64).astype(np.complex128) if lo else P["x"]
    f = op.field(P["f"])
    ua = op.field(u0)
    ub = op.field(u0)
    op.relax(kind, omega, sweeps, f, ua)
    op.relax_noalloc(kind, omega, sweeps, f, ub)
    a, b = to_np(ua), to_np(ub)
    assert np.array_equal(a, b)
    # and against the oracle (per-sweep results rounded to the storage precision)
    s = op_or.coefficient(P["ksq"], P["alpha"])
    fr = P["f"]
    if lo:
        s = s.astype(np.complex64).astype(np.complex128)
        fr = fr.astype(np.complex64).astype(np.complex128)
    ref = u0.copy()
    for _ in range(sweeps):
        ref = (op_or.jacobi_sweep if kind == helm.JACOBI else op_or.rbgs_sweep)(ref, fr, s, P["mask"], omega)
        if lo:
            ref = ref.astype(np.complex64).astype(np.complex128)
    assert rel_err(b, ref) <= (1e-13 if dtype == helm.C128 else 1e-6)


@pytest.mark.parametrize("dtype", [helm.C128, helm.C64])
@pytest.mark.parametrize("kind", [0, 1])
def test_noalloc_matches_relax_twice(kind, dtype):
    # the first call on a large grid (odd count: the last sweep lands in the
    # static array and is copied back), the second on a smaller one (even count)
    _run((96, 80, 70), 1, dtype, kind, 3, 0.7)
    _run((33, 17, 9), 2, dtype, kind, 4, 0.9)


def test_noalloc_rejects_fields_beyond_the_scratch():
    n = (256, 256, 65)   # 4.26 Mi nodes: 68 MB of complex128, over the 64 MiB scratch
    op = helm.Op(n, helm.C128, np.full(I.field_shape(n), 25.0), np.zeros(I.field_shape(n)),
                 np.zeros(I.field_shape(n), np.uint8))
    f = op.field()
    u = op.field()
    with pytest.raises(helm.HelmError) as e:
        op.relax_noalloc(helm.JACOBI, 0.5, 1, f, u)
    assert e.value.status == helm.E_INVAL
    # the same grid in complex64 fits (34 MB)
    op32 = helm.Op(n, helm.C64, np.full(I.field_shape(n), 25.0), np.zeros(I.field_shape(n)),
                   np.zeros(I.field_shape(n), np.uint8))
    op32.relax_noalloc(helm.JACOBI, 0.5, 1, op32.field(), op32.field())
