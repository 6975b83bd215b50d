"""Error measures (test infrastructure only): relative L2 per field, and the
relative infinity norm (the paper measures errors in the infinity norm,
Section 3)."""
from __future__ import annotations

import numpy as np


def rel_l2(x, ref) -> float:
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (den if den > 0 else 1.0))


def rel_inf(x, ref) -> float:
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.max(np.abs(ref)) if ref.size else 0.0
    return float(np.max(np.abs(x - ref)) / (den if den > 0 else 1.0)) if x.size else 0.0
