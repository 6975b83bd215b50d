"""phi-functions of small dense matrices (FP64), from their definition.

Test infrastructure only (see the package docstring).

phi_l(X) = sum_k X^k / (k + l)!  (Section 1).  The oracle evaluates all of
phi_0(X), ..., phi_p(X) at once as the first block row of the exponential of
the block upper-triangular matrix

        [ X  I  0 ... 0 ]
        [ 0  0  I ... 0 ]
    W = [ .        .    ]      ((p+1) n x (p+1) n),
        [ 0  0  0 ... I ]
        [ 0  0  0 ... 0 ]

a standard identity that follows from the series: the (1, j+1) block of
exp(W) is sum_k X^k/(k+j)! = phi_j(X).  The exponential itself is the library
routine scipy.linalg.expm.  This is deliberately an independent method from
the rational Pade / modified squaring construction the GPU library uses.
"""
from __future__ import annotations

from typing import List

import numpy as np
import scipy.linalg


def phi_all(X: np.ndarray, p: int) -> List[np.ndarray]:
    """[phi_0(X), ..., phi_p(X)] for a square FP64 matrix X (real, or complex
    for the complex-coefficient splittings of Table 2)."""
    X = np.asarray(X)
    X = X.astype(np.complex128 if np.iscomplexobj(X) else np.float64)
    n = X.shape[0]
    if X.shape != (n, n):
        raise ValueError("X must be square")
    W = np.zeros(((p + 1) * n, (p + 1) * n), dtype=X.dtype)
    W[:n, :n] = X
    for j in range(p):
        W[j * n:(j + 1) * n, (j + 1) * n:(j + 2) * n] = np.eye(n)
    E = scipy.linalg.expm(W)
    return [E[:n, j * n:(j + 1) * n].copy() for j in range(p + 1)]


def phi(X: np.ndarray, ell: int) -> np.ndarray:
    """phi_ell(X)."""
    return phi_all(X, ell)[ell]
