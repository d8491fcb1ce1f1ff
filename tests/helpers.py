"""Shared test helpers: building ops from the seeded inputs and comparing
GPU fields with the oracle.  Holds no arithmetic of the method."""
from __future__ import annotations

import numpy as np

from paper_2405_12380_amd import inputs as I


def rel_err(a, b) -> float:
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def to_np(t):
    return t.detach().cpu().numpy()


def stored(a, dtype_c64: bool):
    """Values as a C64 op stores them (complex64 rounding), else unchanged."""
    a = np.asarray(a)
    return a.astype(np.complex64).astype(np.complex128) if dtype_c64 else a


def stored_layers(layers, dtype_c64: bool):
    """Network weights as a C64 network stores them (fp32 rounding), else unchanged."""
    if not dtype_c64:
        return layers
    return [(np.asarray(W, dtype=np.float32).astype(np.float64), np.asarray(b, dtype=np.float32).astype(np.float64))
            for W, b in layers]


def make_op(helm, P, dtype):
    return helm.Op(P["n"], dtype, P["ksq"], P["alpha"], P["mask"])


def as_field(P, a):
    return np.asarray(a).reshape(I.field_shape(P["n"]))
