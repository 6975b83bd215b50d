"""Helpers for the GPU parity tests: moving Fortran-ordered numpy data to and
from flat FP64 device tensors, and the error measures used in assertions."""
import sys

import numpy as np


def torch():
    import torch as _t
    return _t


def dev(x) -> "object":
    """numpy tensor (Fortran semantics) or matrix -> flat FP64 device tensor in
    the library layout (index 1 fastest; matrices column-major)."""
    t = torch()
    flat = np.asarray(x, dtype=np.float64).ravel(order="F")
    return t.from_numpy(flat.copy()).to("cuda")


def host(t, dims) -> np.ndarray:
    return t.detach().cpu().numpy().reshape(tuple(dims), order="F")


def rel_err(x, ref) -> float:
    x = np.asarray(x).ravel()
    ref = np.asarray(ref).ravel()
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(x - ref)) / (den if den > 0 else 1.0))


def rel_l2(x, ref) -> float:
    x = np.asarray(x).ravel()
    ref = np.asarray(ref).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (den if den > 0 else 1.0))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
