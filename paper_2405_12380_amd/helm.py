"""Python binding of libhelm's C ABI (argument marshalling only).

Every function here converts arguments (torch tensors to device pointers,
Python numbers and lists to C structs), calls the entry point of the same name
in ``libhelm.so`` and converts the results back.  No step of the numerical
method runs in Python.  Importing this module fails loudly when the compiled
library is absent.

torch is imported before the library is loaded so that libhelm binds to the
HIP runtime already loaded by torch (same SONAME), giving one runtime per
process; torch provides device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhelm.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"libhelm.so not found at {_LIB_PATH}: build it with "
                      "`python -m paper_2405_12380_amd.build` (no fallback exists)")
_lib = C.CDLL(_LIB_PATH)

# ---- constants (mirror include/helm.h) --------------------------------------
OK, NOT_CONVERGED = 0, 1
E_INVAL, E_NOMEM, E_HIP, E_BREAKDOWN, E_NONFINITE, E_SINGULAR = -1, -2, -3, -4, -5, -6
C64, C128 = 1, 2
JACOBI, RBGS = 0, 1
DON_TANH, DON_RELU, DON_LEAKY = 0, 1, 2
DON_SPLIT_OUTPUT, DON_SPLIT_INPUT = 0, 1
DON_TRUNK, DON_FULL, DON_BRANCH_INPUT = 0, 1, 2
META_JACOBI, META_GS, META_GMRES, META_BICGSTAB = 0, 1, 2, 3
RB_AUTO, RB_RING, RB_PAIRS = 0, 1, 2

EXPORTED = ["helm_setup", "helm_set_ksq", "helm_tune", "helm_set_rbgs_kernel", "helm_relax_noalloc", "helm_destroy", "helm_size", "helm_apply", "helm_residual",
            "helm_relax", "helm_dot", "helm_nrm2", "deeponet_load", "deeponet_free", "deeponet_infer",
            "meta_solve", "meta_precond", "meta_coarse_info", "meta_solve_adjoint", "meta_solve_batch", "helm_misfit",
            "helm_ksq_gradient", "don_train_create", "don_train_data", "don_train_steps", "don_train_eval",
            "don_train_grad", "don_train_apply", "don_train_nparam", "don_train_layout", "don_train_params",
            "don_train_export", "don_train_free", "helm_kprof_enable", "helm_kprof_read", "helm_stream_copy",
            "helm_strerror", "helm_last_error"]
KP_STENCIL, KP_MULTIDOT, KP_MULTIAXPY, KP_QT, KP_SKINNY, KP_CGS, KP_MFMA = 0, 1, 2, 3, 4, 5, 6
KP_NAMES = {KP_STENCIL: "stencil", KP_MULTIDOT: "multidot", KP_MULTIAXPY: "multi_axpy", KP_QT: "qt_part",
            KP_SKINNY: "skinny_apply", KP_CGS: "cgs_fused", KP_MFMA: "mfma_setup"}


class HelmGrid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3)]


class DonDesc(C.Structure):
    _fields_ = [("n_branch", C.c_int), ("branch_w", C.POINTER(C.c_int)), ("n_trunk", C.c_int),
                ("trunk_w", C.POINTER(C.c_int)), ("act", C.c_int), ("head", C.c_int), ("p", C.c_int),
                ("branch_grid", C.c_int * 3), ("k_input", C.c_int)]


class MetaOpts(C.Structure):
    _fields_ = [("kind", C.c_int), ("restart", C.c_int), ("tol", C.c_double), ("max_iters", C.c_int),
                ("smoother", C.c_int), ("n_r", C.c_int), ("omega", C.c_double), ("nn_every", C.c_int),
                ("p_used", C.c_int), ("k", C.c_double), ("history", C.POINTER(C.c_double)), ("q_fp32", C.c_int),
                ("mg_levels", C.c_int), ("mg_nu", C.c_int), ("no_drop", C.c_int), ("fallback_restart", C.c_int),
                ("gs_passes", C.c_int)]


class MetaStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("matvecs", C.c_int), ("precond_apps", C.c_int), ("converged", C.c_int),
                ("rank_used", C.c_int), ("history_len", C.c_int), ("rel_res", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("cond_Ac_est", C.c_double),
                ("fallback_iters", C.c_int)]


class DonTrainOpts(C.Structure):
    _fields_ = [("n_points", C.c_int), ("batch", C.c_int), ("max_steps", C.c_int), ("lr", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


_vp = C.c_void_p
_sig = {
    "helm_setup": (C.c_int, [C.POINTER(HelmGrid), C.c_int, _vp, _vp, _vp, _vp, C.POINTER(_vp)]),
    "helm_set_ksq": (C.c_int, [_vp, _vp, _vp]),
    "helm_tune": (C.c_int, [_vp, C.c_int, _vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "helm_set_rbgs_kernel": (C.c_int, [_vp, C.c_int]),
    "helm_destroy": (None, [_vp]),
    "helm_size": (C.c_size_t, [_vp]),
    "helm_apply": (C.c_int, [_vp, _vp, _vp, _vp]),
    "helm_residual": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double), _vp]),
    "helm_relax": (C.c_int, [_vp, C.c_int, C.c_double, C.c_int, _vp, _vp, _vp]),
    "helm_relax_noalloc": (C.c_int, [_vp, C.c_int, C.c_double, C.c_int, _vp, _vp, _vp]),
    "helm_dot": (C.c_int, [_vp, _vp, _vp, C.POINTER(C.c_double), _vp]),
    "helm_nrm2": (C.c_int, [_vp, _vp, C.POINTER(C.c_double), _vp]),
    "deeponet_load": (C.c_int, [C.c_int, C.POINTER(DonDesc), C.POINTER(C.POINTER(C.c_double)), C.POINTER(_vp)]),
    "deeponet_free": (None, [_vp]),
    "deeponet_infer": (C.c_int, [_vp, _vp, C.c_int, _vp, C.c_double, _vp, _vp]),
    "meta_solve": (C.c_int, [_vp, _vp, C.POINTER(MetaOpts), _vp, _vp, C.POINTER(MetaStats), _vp]),
    "meta_precond": (C.c_int, [_vp, _vp, C.POINTER(MetaOpts), _vp, _vp, _vp]),
    "meta_coarse_info": (C.c_int, [_vp, _vp, C.POINTER(MetaOpts), C.POINTER(C.c_int), C.POINTER(C.c_double),
                                   C.c_size_t, _vp, C.c_size_t, _vp]),
    "meta_solve_adjoint": (C.c_int, [_vp, _vp, C.POINTER(MetaOpts), _vp, _vp, C.POINTER(MetaStats), _vp]),
    "meta_solve_batch": (C.c_int, [C.c_int, C.POINTER(_vp), _vp, C.POINTER(MetaOpts), C.POINTER(_vp),
                                   C.POINTER(_vp), C.POINTER(MetaStats), _vp]),
    "helm_misfit": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp, C.POINTER(C.c_double), _vp]),
    "helm_ksq_gradient": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "don_train_create": (C.c_int, [_vp, C.POINTER(DonTrainOpts), _vp, C.POINTER(_vp)]),
    "don_train_data": (C.c_int, [_vp, C.c_int, _vp, _vp]),
    "don_train_steps": (C.c_int, [_vp, C.c_int, _vp, C.POINTER(C.c_float), _vp]),
    "don_train_eval": (C.c_int, [_vp, C.c_int, _vp, C.POINTER(C.c_float), _vp]),
    "don_train_grad": (C.c_int, [_vp, _vp, C.POINTER(C.c_float), _vp, _vp]),
    "don_train_apply": (C.c_int, [_vp, _vp, _vp]),
    "don_train_nparam": (C.c_size_t, [_vp]),
    "don_train_layout": (C.c_int, [_vp, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                   C.POINTER(C.c_int), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "don_train_params": (C.c_int, [_vp, _vp, _vp]),
    "don_train_export": (C.c_int, [_vp, _vp, _vp]),
    "don_train_free": (None, [_vp]),
    "helm_kprof_enable": (C.c_int, [C.c_int]),
    "helm_kprof_read": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "helm_stream_copy": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "helm_strerror": (C.c_char_p, [C.c_int]),
    "helm_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class HelmError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.helm_last_error().decode() or _lib.helm_strerror(status).decode()
        super().__init__(f"{where}: {_lib.helm_strerror(status).decode()} ({status}): {msg}")


def _check(status, where, allow=(OK,)):
    if status not in allow:
        raise HelmError(status, where)
    return status


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return _vp(t.data_ptr())


def cdtype(dt: int):
    return torch.complex128 if dt == C128 else torch.complex64


def rdtype(dt: int):
    return torch.float64 if dt == C128 else torch.float32


def _dev(a, dtype, device="cuda"):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous().reshape(-1)
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dtype).reshape(-1)


def _host_or_dev(a, dtype):
    """(owner, pointer): a device tensor as is, anything else as a contiguous
    host array of the dtype (the owner keeps it alive for the call)."""
    if isinstance(a, torch.Tensor) and a.is_cuda:
        t = a.to(dtype=dtype).contiguous().reshape(-1)
        return t, _vp(t.data_ptr())
    h = np.ascontiguousarray(a.cpu().numpy() if isinstance(a, torch.Tensor) else a,
                             dtype=torch.empty(0, dtype=dtype).numpy().dtype).reshape(-1)
    return h, _vp(h.ctypes.data)


class Op:
    """The discrete Helmholtz operator on a grid (``helm_setup``).

    ``n`` is (nx, ny) or (nx, ny, nz); ``ksq``, ``alpha`` (real) and ``mask``
    (uint8) are arrays of the field shape or flat: numpy arrays are passed to
    the library as host arrays, device tensors as device arrays."""

    def __init__(self, n, dtype: int, ksq, alpha, mask, stream=None):
        self.n = tuple(int(v) for v in n)
        self.dim = len(self.n)
        self.dtype = dtype
        g = HelmGrid(self.dim, (C.c_int * 3)(*(list(self.n) + [1] * (3 - self.dim))))
        keep = [_host_or_dev(a, t) for a, t in ((ksq, torch.float64), (alpha, torch.float64), (mask, torch.uint8))]
        h = _vp()
        _check(_lib.helm_setup(C.byref(g), dtype, *[p for _, p in keep], _stream(stream), C.byref(h)), "helm_setup")
        self.h = h
        self.size = int(_lib.helm_size(h))

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.helm_destroy(self.h)
            self.h = None

    __del__ = close

    def field(self, a=None):
        """A device field of this op's complex dtype (zeros, or converted from ``a``)."""
        if a is None:
            return torch.zeros(self.size, dtype=cdtype(self.dtype), device="cuda")
        return _dev(a, cdtype(self.dtype))

    def set_ksq(self, ksq, stream=None):
        k = _dev(ksq, torch.float64)
        _check(_lib.helm_set_ksq(self.h, _ptr(k), _stream(stream)), "helm_set_ksq")

    def tune(self, fixed_ty: int = 0, stream=None):
        """Autotune the stencil tile (``helm_tune``); returns (ty, zb, us per apply)."""
        ty, zb, us = C.c_int(), C.c_int(), C.c_double()
        _check(_lib.helm_tune(self.h, int(fixed_ty), _stream(stream), C.byref(ty), C.byref(zb), C.byref(us)),
               "helm_tune")
        return ty.value, zb.value, us.value

    def set_rbgs_kernel(self, which: int):
        """Choose the red-black sweep kernel (RB_AUTO, RB_RING, RB_PAIRS)."""
        _check(_lib.helm_set_rbgs_kernel(self.h, int(which)), "helm_set_rbgs_kernel")

    def apply(self, x, y=None, stream=None):
        y = self.field() if y is None else y
        _check(_lib.helm_apply(self.h, _ptr(x), _ptr(y), _stream(stream)), "helm_apply")
        return y

    def residual(self, f, u, r=None, norm=False, stream=None):
        r = self.field() if r is None else r
        nv = C.c_double(0.0)
        _check(_lib.helm_residual(self.h, _ptr(f), _ptr(u), _ptr(r), C.byref(nv) if norm else None,
                                  _stream(stream)), "helm_residual")
        return (r, nv.value) if norm else r

    def relax(self, kind: int, omega: float, sweeps: int, f, u, stream=None):
        _check(_lib.helm_relax(self.h, kind, float(omega), int(sweeps), _ptr(f), _ptr(u), _stream(stream)),
               "helm_relax")
        return u

    def relax_noalloc(self, kind: int, omega: float, sweeps: int, f, u, stream=None):
        """``helm_relax`` without device allocation (static scratch)."""
        _check(_lib.helm_relax_noalloc(self.h, kind, float(omega), int(sweeps), _ptr(f), _ptr(u), _stream(stream)),
               "helm_relax_noalloc")
        return u

    def misfit(self, axis: int, index: int, u, d, g=None, loss=True, stream=None):
        """(1/2 ||P u - d||^2 or None, g = P^T (P u - d)) on the plane {i_axis = index}."""
        g = self.field() if g is None else g
        lv = C.c_double()
        _check(_lib.helm_misfit(self.h, int(axis), int(index), _ptr(u), _ptr(d), _ptr(g),
                                C.byref(lv) if loss else None, _stream(stream)), "helm_misfit")
        return (lv.value if loss else None), g

    def ksq_gradient(self, u, lam, grad=None, stream=None):
        """Re(conj(lam) (1 + i alpha) u), 0 on the scatterer (real field)."""
        if grad is None:
            grad = torch.empty(self.size, dtype=rdtype(self.dtype), device="cuda")
        _check(_lib.helm_ksq_gradient(self.h, _ptr(u), _ptr(lam), _ptr(grad), _stream(stream)), "helm_ksq_gradient")
        return grad

    def dot(self, x, y, stream=None) -> complex:
        out = (C.c_double * 2)()
        _check(_lib.helm_dot(self.h, _ptr(x), _ptr(y), out, _stream(stream)), "helm_dot")
        return complex(out[0], out[1])

    def nrm2(self, x, stream=None) -> float:
        out = C.c_double(0.0)
        _check(_lib.helm_nrm2(self.h, _ptr(x), C.byref(out), _stream(stream)), "helm_nrm2")
        return out.value


_ACT = {"tanh": DON_TANH, "relu": DON_RELU, "leaky": DON_LEAKY}
_HEAD = {"split_output": DON_SPLIT_OUTPUT, "split_input": DON_SPLIT_INPUT}


class DeepONet:
    """A DeepONet uploaded to the device (``deeponet_load``).  ``branch`` and
    ``trunk`` are lists of (W, b) numpy arrays, W of shape (fan_in, fan_out)."""

    def __init__(self, dtype: int, branch, trunk, p: int, head="split_output", act="tanh", branch_grid=(1, 1, 1),
                 k_input=False):
        self.dtype = dtype
        self.p = int(p)
        self.head = head
        bw = [int(branch[0][0].shape[0])] + [int(W.shape[1]) for W, _ in branch]
        tw = [int(trunk[0][0].shape[0])] + [int(W.shape[1]) for W, _ in trunk]
        bg = list(branch_grid) + [1] * (3 - len(branch_grid))
        self._bw = (C.c_int * len(bw))(*bw)
        self._tw = (C.c_int * len(tw))(*tw)
        d = DonDesc(len(bw), self._bw, len(tw), self._tw, _ACT[act], _HEAD[head], self.p,
                    (C.c_int * 3)(*bg), 1 if k_input else 0)
        arrays = []
        for W, b in list(branch) + list(trunk):
            arrays.append(np.ascontiguousarray(W, dtype=np.float64))
            arrays.append(np.ascontiguousarray(b, dtype=np.float64))
        ptrs = (C.POINTER(C.c_double) * len(arrays))(*[a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrays])
        h = _vp()
        _check(_lib.deeponet_load(dtype, C.byref(d), ptrs, C.byref(h)), "deeponet_load")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            if _lib is not None:
                _lib.deeponet_free(self.h)
            self.h = None

    __del__ = close

    def trunk(self, op: Op, out=None, stream=None):
        out = torch.empty(op.size * self.p, dtype=rdtype(self.dtype), device="cuda") if out is None else out
        _check(_lib.deeponet_infer(self.h, op.h, DON_TRUNK, None, 0.0, _ptr(out), _stream(stream)), "deeponet_infer")
        return out

    def branch_input(self, op: Op, r, k=0.0, out=None, stream=None):
        """The branch input vector the network would see for r (``DON_BRANCH_INPUT``)."""
        if out is None:
            out = torch.empty(self._bw[0] * (2 if self.head == "split_input" else 1), dtype=rdtype(self.dtype),
                              device="cuda")
        _check(_lib.deeponet_infer(self.h, op.h, DON_BRANCH_INPUT, _ptr(r), float(k), _ptr(out), _stream(stream)),
               "deeponet_infer")
        return out

    def full(self, op: Op, r, k=0.0, out=None, stream=None):
        out = op.field() if out is None else out
        _check(_lib.deeponet_infer(self.h, op.h, DON_FULL, _ptr(r), float(k), _ptr(out), _stream(stream)),
               "deeponet_infer")
        return out


_KIND = {"jacobi": META_JACOBI, "gs": META_GS, "gmres": META_GMRES, "bicgstab": META_BICGSTAB}
_SMOOTH = {"jacobi": JACOBI, "rbgs": RBGS}


def _opts(kind, restart=50, tol=1e-6, max_iters=20000, smoother="jacobi", n_r=3, omega=0.5, nn_every=25,
          p_used=None, k=0.0, history=None, net=None, q_fp32=False, mg_levels=0, mg_nu=5, no_drop=False,
          fallback_restart=0, gs_passes=0):
    pu = p_used if p_used is not None else (net.p if net is not None else 0)
    hp = history.ctypes.data_as(C.POINTER(C.c_double)) if history is not None else None
    return MetaOpts(_KIND[kind] if isinstance(kind, str) else int(kind), int(restart), float(tol), int(max_iters),
                    _SMOOTH[smoother] if isinstance(smoother, str) else int(smoother), int(n_r), float(omega),
                    int(nn_every), int(pu), float(k), hp, 1 if q_fp32 else 0, int(mg_levels), int(mg_nu),
                    1 if no_drop else 0, int(fallback_restart), int(gs_passes))


def meta_solve(op: Op, net: DeepONet | None, f, u, kind="gmres", history=False, stream=None, adjoint=False, **kw):
    """Run ``meta_solve`` (``meta_solve_adjoint`` for A^H u = f when adjoint is
    set); returns (status, stats dict[, history array]).  u is updated in
    place.  Status HELM_NOT_CONVERGED is returned, not raised."""
    hist = np.zeros(int(kw.get("max_iters", 20000)) + 2) if history else None
    o = _opts(kind, history=hist, net=net, **kw)
    st = MetaStats()
    fn, name = (_lib.meta_solve_adjoint, "meta_solve_adjoint") if adjoint else (_lib.meta_solve, "meta_solve")
    s = fn(op.h, net.h if net is not None else None, C.byref(o), _ptr(f), _ptr(u), C.byref(st), _stream(stream))
    _check(s, name, allow=(OK, NOT_CONVERGED, E_BREAKDOWN, E_NONFINITE))
    stats = {name: getattr(st, name) for name, _ in MetaStats._fields_}
    stats["status"] = s
    if history:
        return s, stats, hist[: st.history_len].copy()
    return s, stats


def meta_solve_batch(ops, net: DeepONet | None, fs, us, stream=None, **kw):
    """Run ``meta_solve_batch`` (BiCGStab over all problems at once); returns
    (status, list of stats dicts).  us are updated in place."""
    n = len(ops)
    kw.setdefault("kind", "bicgstab")
    o = _opts(net=net, **kw)
    hops = (_vp * n)(*[op.h for op in ops])
    hf = (_vp * n)(*[_ptr(f) for f in fs])
    hu = (_vp * n)(*[_ptr(u) for u in us])
    st = (MetaStats * n)()
    s = _lib.meta_solve_batch(n, hops, net.h if net is not None else None, C.byref(o), hf, hu, st, _stream(stream))
    _check(s, "meta_solve_batch", allow=(OK, NOT_CONVERGED, E_BREAKDOWN, E_NONFINITE))
    out = []
    for i in range(n):
        d = {name: getattr(st[i], name) for name, _ in MetaStats._fields_}
        out.append(d)
    return s, out


def meta_precond(op: Op, net: DeepONet | None, r, z=None, stream=None, **kw):
    z = op.field() if z is None else z
    o = _opts("gmres", net=net, **kw)
    _check(_lib.meta_precond(op.h, net.h if net is not None else None, C.byref(o), _ptr(r), _ptr(z),
                             _stream(stream)), "meta_precond")
    return z


def coarse_info(op: Op, net: DeepONet, p_used=None, want_q=False, q_fp32=False, stream=None):
    """(rank, A_c as a complex numpy array[, Q as a device tensor n x rank])."""
    o = _opts("gmres", net=net, p_used=p_used, q_fp32=q_fp32)
    rank = C.c_int(0)
    _check(_lib.meta_coarse_info(op.h, net.h, C.byref(o), C.byref(rank), None, 0, None, 0, _stream(stream)),
           "meta_coarse_info")
    r = rank.value
    ac = np.zeros(2 * r * r)
    qdt = torch.float32 if (q_fp32 or op.dtype == C64) else torch.float64
    q = torch.empty(op.size * r, dtype=qdt, device="cuda") if want_q else None
    _check(_lib.meta_coarse_info(op.h, net.h, C.byref(o), C.byref(rank), ac.ctypes.data_as(C.POINTER(C.c_double)),
                                 r * r, _ptr(q), op.size * r if want_q else 0, _stream(stream)), "meta_coarse_info")
    A = ac.view(np.complex128).reshape(r, r)
    return (r, A, q) if want_q else (r, A)


class Trainer:
    """DeepONet trainer (``don_train_*``): bf16 MFMA forward/backward, Adam.

    X: P x d node coordinates (fp64); the dataset is set with ``data``."""

    def __init__(self, net: DeepONet, X, batch=64, max_steps=64, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        Xd = _dev(X, torch.float64)
        self.P = int(np.asarray(X.shape)[0]) if hasattr(X, "shape") else len(X)
        self.S = int(batch)
        self.max_steps = int(max_steps)
        o = DonTrainOpts(self.P, self.S, self.max_steps, lr, beta1, beta2, eps)
        h = _vp()
        _check(_lib.don_train_create(net.h, C.byref(o), _ptr(Xd), C.byref(h)), "don_train_create")
        self.h = h
        self.nparam = int(_lib.don_train_nparam(h))
        self._Y = None

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.don_train_free(self.h)
            self.h = None

    __del__ = close

    def data(self, F, Y):
        """F: n x K_b fp32 device tensor; Y: n x P complex64 device tensor (kept alive here)."""
        F = F.to(torch.float32).contiguous()
        Y = Y.to(torch.complex64).contiguous()
        self._Y = Y
        _check(_lib.don_train_data(self.h, int(F.shape[0]), _ptr(F), _ptr(Y)), "don_train_data")

    def _idx(self, idx):
        return torch.as_tensor(np.asarray(idx, dtype=np.int32) if not torch.is_tensor(idx) else idx,
                               dtype=torch.int32).to("cuda").contiguous()

    def steps(self, idx):
        it = self._idx(idx)
        count = it.numel() // self.S
        out = (C.c_float * count)()
        _check(_lib.don_train_steps(self.h, count, _ptr(it), out, None), "don_train_steps")
        return np.array(out[:], dtype=np.float64)

    def eval(self, idx):
        it = self._idx(idx)
        count = it.numel() // self.S
        out = (C.c_float * count)()
        _check(_lib.don_train_eval(self.h, count, _ptr(it), out, None), "don_train_eval")
        return np.array(out[:], dtype=np.float64)

    def grad(self, idx):
        it = self._idx(idx)
        g = torch.empty(self.nparam, dtype=torch.float32, device="cuda")
        loss = C.c_float()
        _check(_lib.don_train_grad(self.h, _ptr(it), C.byref(loss), _ptr(g), None), "don_train_grad")
        return float(loss.value), g

    def apply(self, grads):
        g = grads.to(device="cuda", dtype=torch.float32).contiguous()
        _check(_lib.don_train_apply(self.h, _ptr(g), None), "don_train_apply")

    def params(self):
        out = torch.empty(self.nparam, dtype=torch.float32, device="cuda")
        _check(_lib.don_train_params(self.h, _ptr(out), None), "don_train_params")
        return out

    def layout(self, which: int, layer: int):
        K, Kp, N = C.c_int(), C.c_int(), C.c_int()
        oW, ob = C.c_size_t(), C.c_size_t()
        _check(_lib.don_train_layout(self.h, which, layer, C.byref(K), C.byref(Kp), C.byref(N), C.byref(oW),
                                     C.byref(ob)), "don_train_layout")
        return K.value, Kp.value, N.value, oW.value, ob.value

    def unflatten(self, flat, which: int, nlayers: int):
        """[(W (K x N), b (N))] numpy arrays of the branch (0) or trunk (1) from a flat vector."""
        f = flat.detach().cpu().numpy() if torch.is_tensor(flat) else np.asarray(flat)
        out = []
        for li in range(nlayers):
            K, Kp, N, oW, ob = self.layout(which, li)
            out.append((f[oW:oW + Kp * N].reshape(Kp, N)[:K].astype(np.float64), f[ob:ob + N].astype(np.float64)))
        return out

    def flatten(self, branch, trunk):
        """Flat fp32 vector (zero padding) from [(W, b)] lists."""
        f = np.zeros(self.nparam, dtype=np.float32)
        for which, layers in ((0, branch), (1, trunk)):
            for li, (W, b) in enumerate(layers):
                K, Kp, N, oW, ob = self.layout(which, li)
                blk = np.zeros((Kp, N), dtype=np.float32)
                blk[:K] = W
                f[oW:oW + Kp * N] = blk.ravel()
                f[ob:ob + N] = b
        return torch.as_tensor(f).to("cuda")

    def export(self, net: DeepONet):
        _check(_lib.don_train_export(self.h, net.h, None), "don_train_export")


def kprof_enable(on: bool = True, kinds=None):
    """Turn per-kernel event timing on for the classes in `kinds` (all when
    None), clearing earlier records, or off."""
    if not on:
        mask = 0
    elif kinds is None:
        mask = -1
    else:
        mask = 0
        for k in kinds:
            mask |= 1 << int(k)
    _check(_lib.helm_kprof_enable(mask), "helm_kprof_enable")


def stream_copy(src, dst, stream=None):
    """dst = src with the library's non-temporal streaming copy (device tensors)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("stream_copy: sizes differ")
    _check(_lib.helm_stream_copy(_ptr(src), _ptr(dst), nb, _stream(stream)), "helm_stream_copy")
    return dst


def kprof_read(kind: int):
    """(launches, total ms, total algorithmic bytes) for one kernel class."""
    n, ms, by = C.c_int(0), C.c_double(0.0), C.c_double(0.0)
    _check(_lib.helm_kprof_read(kind, C.byref(n), C.byref(ms), C.byref(by)), "helm_kprof_read")
    return n.value, ms.value, by.value
