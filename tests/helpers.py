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


def make_op(helm, P, dtype):
    return helm.Op(P["n"], dtype, P["ksq"], P["alpha"], P["mask"])


def as_field(P, a):
    return np.asarray(a).reshape(I.field_shape(P["n"]))
