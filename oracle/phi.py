"""phi-functions of small dense matrices, from their definition.

Test infrastructure only (see the package docstring).

phi_l(X) = sum_k X^k / (k + l)!  (Section 1).  Two evaluations, chosen by the
matrix:

* Scalar multiples of the Neumann second-difference pattern (every matrix the
  workloads build, Section 3): X = a T_n with T_n tridiagonal, interior rows
  (1, -2, 1), first row (-2, 2), last row (2, -2).  T_n has the DCT-I
  eigenvectors v_k[j] = cos(pi j k / (n-1)) and eigenvalues
  lambda_k = -4 sin^2(pi k / (2 (n-1))), and it is self-adjoint for the weights
  w = (1/2, 1, ..., 1, 1/2), so phi_l(X) = V diag(phi_l(a lambda_k)) V^{-1}
  with V^{-1} = diag(1/c_k) V^T diag(w), c_k = sum_j w_j v_k[j]^2.  Writing
  the product of two cosines as half the sum of the cosines of the difference
  and the sum of the angles gives, entry by entry,

      phi_l(X)[i, j] = w_j / 2 (t(|i - j|) + t(i + j)),
      t(m) = sum_k phi_l(a lambda_k) / c_k cos(pi k m / (n-1)).

  The scalars phi_l(a lambda_k) and the sums t(m) are evaluated in long double
  (64-bit significand), angles reduced exactly in integers, and the result is
  rounded to FP64 once.  This is the definition applied to the exact
  eigen-decomposition: it carries no scaling-and-squaring amplification,
  whereas any squaring method in FP64 loses about u ||X|| on the constant
  mode of a stiff X (||X|| reaches 2e5 at the 256^3 workload).

* Every other matrix (and complex X, used by the complex splittings of
  Table 2): the first block row of the exponential of the block upper
  triangular matrix

        [ X  I  0 ... 0 ]
        [ 0  0  I ... 0 ]
    W = [ .        .    ]      ((p+1) n x (p+1) n),
        [ 0  0  0 ... I ]
        [ 0  0  0 ... 0 ]

  a standard identity that follows from the series: the (1, j+1) block of
  exp(W) is sum_k X^k/(k+j)! = phi_j(X).  The exponential is the library
  routine scipy.linalg.expm.

Both are independent of the rational Pade / modified squaring construction of
the GPU library.
"""
from __future__ import annotations

import math
from typing import List, Optional

import numpy as np
import scipy.linalg

_LD = np.longdouble
# pi to more digits than long double holds (parsed by numpy at full precision)
_PI_LD = _LD("3.14159265358979323846264338327950288419716939937510")


def neumann_multiple(X: np.ndarray) -> Optional[float]:
    """a if X equals a T_n entry for entry (the Neumann second-difference
    pattern above, n >= 2), else None."""
    if np.iscomplexobj(X) or X.ndim != 2 or X.shape[0] != X.shape[1] or X.shape[0] < 2:
        return None
    n = X.shape[0]
    a = X[0, 1] / 2.0 if n == 2 else X[1, 0]
    T = np.zeros((n, n))
    if n == 2:
        T[:] = [[-2.0, 2.0], [2.0, -2.0]]
    else:
        i = np.arange(1, n - 1)
        T[i, i - 1], T[i, i], T[i, i + 1] = 1.0, -2.0, 1.0
        T[0, 0], T[0, 1] = -2.0, 2.0
        T[n - 1, n - 2], T[n - 1, n - 1] = 2.0, -2.0
    # a * T is exact in FP64 (entries are a times 1, -2 or 2)
    return float(a) if np.array_equal(X, a * T) else None


def phi_scalar_ld(z: np.ndarray, ell: int) -> np.ndarray:
    """phi_ell(z) elementwise in long double: the series sum_k z^k/(k+ell)!
    for |z| < 1 (40 terms), else (e^z - sum_{k<ell} z^k/k!) / z^ell with
    e^z - 1 from expm1."""
    z = np.asarray(z, dtype=_LD)
    out = np.empty_like(z)
    small = np.abs(z) < 1
    zs = z[small]
    term = np.full_like(zs, _LD(1) / _LD(math.factorial(ell)))
    acc = term.copy()
    for k in range(1, 40):
        term = term * zs / _LD(k + ell)
        acc = acc + term
    out[small] = acc
    zb = z[~small]
    num = np.expm1(zb)                       # e^z - 1
    if ell == 0:
        num = num + 1
    else:
        pw = zb.copy()
        for k in range(1, ell):              # subtract z^k/k!, k = 1..ell-1
            num = num - pw / _LD(math.factorial(k))
            pw = pw * zb
        num = num / pw                       # pw = z^ell
    out[~small] = num
    return out


def _phi_neumann(a: float, n: int, p: int) -> List[np.ndarray]:
    """[phi_0(a T_n), ..., phi_p(a T_n)] from the spectral form above."""
    k = np.arange(n)
    lam = -4 * np.sin(_PI_LD * k.astype(_LD) / _LD(2 * (n - 1))) ** 2
    c = np.full(n, _LD(n - 1) / 2)
    c[0] = c[n - 1] = _LD(n - 1)
    w = np.ones(n, dtype=_LD)
    w[0] = w[n - 1] = _LD(0.5)
    # cos(pi k m / (n-1)) for m = 0 .. 2(n-1), the angle reduced mod 2(n-1)
    m = np.arange(2 * n - 1)
    km = np.mod(np.outer(m, k), 2 * (n - 1)).astype(_LD)
    C = np.cos(_PI_LD * km / _LD(n - 1))                        # (2n-1, n)
    i = np.arange(n)
    dif = np.abs(i[:, None] - i[None, :])
    sm = i[:, None] + i[None, :]
    out = []
    for ell in range(p + 1):
        g = phi_scalar_ld(_LD(a) * lam, ell) / c
        t = C @ g                                                # (2n-1,)
        M = (t[dif] + t[sm]) * (w[None, :] / 2)
        out.append(M.astype(np.float64))
    return out


def _phi_expm(X: np.ndarray, p: int) -> List[np.ndarray]:
    n = X.shape[0]
    W = np.zeros(((p + 1) * n, (p + 1) * n), dtype=X.dtype)
    W[:n, :n] = X
    for j in range(p):
        W[j * n:(j + 1) * n, (j + 1) * n:(j + 2) * n] = np.eye(n)
    E = scipy.linalg.expm(W)
    return [E[:n, j * n:(j + 1) * n].copy() for j in range(p + 1)]


def phi_all(X: np.ndarray, p: int, method: str = "auto") -> List[np.ndarray]:
    """[phi_0(X), ..., phi_p(X)] for a square FP64 matrix X (real, or complex
    for the complex-coefficient splittings of Table 2).  method "auto" takes
    the spectral form when X is a multiple of the Neumann pattern, "expm"
    forces the augmented-matrix exponential."""
    X = np.asarray(X)
    X = X.astype(np.complex128 if np.iscomplexobj(X) else np.float64)
    n = X.shape[0]
    if X.ndim != 2 or X.shape != (n, n):
        raise ValueError("X must be square")
    if method == "auto":
        a = neumann_multiple(X)
        if a is not None:
            return _phi_neumann(a, n, p)
    elif method != "expm":
        raise ValueError(method)
    return _phi_expm(X, p)


def phi(X: np.ndarray, ell: int, method: str = "auto") -> np.ndarray:
    """phi_ell(X)."""
    return phi_all(X, ell, method)[ell]
