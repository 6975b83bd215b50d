"""Directional-splitting coefficients, written from the closed forms of the paper.

Test infrastructure only (see the package docstring).

* Table 1 (two-term, d = 2, l_1 = 1, l_2 = 2): the real columns, with the
  "+" choice of sign in alpha_{1,1} (Section 2.4 fixes that choice); the upper
  signs of a column go together row by row.
* Table 3 (three-term, d > 2, l_1 = l_3 = 1, l_2 = 2): the "+" choice in
  alpha_{1,mu}; alpha is the same for every direction mu and eta_2 carries
  the factor 2^{d-3}.

* Table 1 complex column and Table 2 (two-term, complex coefficients, any
  d >= 2, used by exprk3ds_cplx): the upper signs; the lower signs are the
  complex conjugates and give the same real part of every split action.

Each function returns (ells, eta, alpha) with
    ells  : tuple of the phi indices l_i of the terms,
    eta   : array (nterms,) of eta_{i,d},
    alpha : array (nterms, d) of alpha_{i,mu}  (mu = 1..d along axis 1).
"""
from __future__ import annotations

import math

import numpy as np


def table1_real(ell: int):
    """Table 1, real columns, "+" set, for phi_ell with ell in {1, 2}."""
    if ell == 1:
        r = math.sqrt(10.0)
        eta = [-5.0 / 4.0, 9.0]
        alpha = [[4.0 / 3.0 + 4.0 * r / 15.0, 4.0 / 3.0 - 4.0 * r / 15.0],
                 [16.0 / 9.0 + 2.0 * r / 9.0, 16.0 / 9.0 - 2.0 * r / 9.0]]
    elif ell == 2:
        r = math.sqrt(33.0)
        eta = [-4.0 / 3.0, 22.0 / 3.0]
        alpha = [[9.0 / 8.0 + r / 8.0, 9.0 / 8.0 - r / 8.0],
                 [3.0 / 2.0 + 3.0 * r / 22.0, 3.0 / 2.0 - 3.0 * r / 22.0]]
    else:
        raise ValueError("Table 1 covers ell = 1, 2")
    return (1, 2), np.array(eta), np.array(alpha)


def table3_real(ell: int, d: int):
    """Table 3, "+" set, for phi_ell (ell in {1, 2}) in dimension d >= 3."""
    if d < 3:
        raise ValueError("Table 3 is stated for d > 2")
    scale = 2.0 ** (d - 3)
    if ell == 1:
        r = math.sqrt(2991111.0)
        e1 = 2243.0 / 1350.0 + 440521.0 / (675.0 * r)
        e3 = 2243.0 / 1350.0 - 440521.0 / (675.0 * r)
        e2 = -12544.0 / 675.0 * scale
        a1 = 3.0 * (5161.0 + r) / 15869.0
        a3 = 3.0 * (5161.0 - r) / 15869.0
        a2 = 45.0 / 28.0
    elif ell == 2:
        r = math.sqrt(2391.0)
        e1 = 19.0 / 27.0 + 151.0 / (27.0 * r)
        e3 = 19.0 / 27.0 - 151.0 / (27.0 * r)
        e2 = -196.0 / 27.0 * scale
        a1 = 3.0 * (121.0 + r) / 490.0
        a3 = 3.0 * (121.0 - r) / 490.0
        a2 = 9.0 / 7.0
    else:
        raise ValueError("Table 3 covers ell = 1, 2")
    eta = np.array([e1, e2, e3])
    alpha = np.array([[a1] * d, [a2] * d, [a3] * d])
    return (1, 2, 1), eta, alpha


def table1_complex(ell: int):
    """Table 1, complex column (upper signs), for phi_ell with ell in {1, 2}."""
    if ell == 1:
        s2 = math.sqrt(2.0)
        eta = [7.0 / 4.0 + 1.5 * s2 * 1j, -3.0 - 6.0 * s2 * 1j]
        a1 = 12.0 / 11.0 - 4.0 * s2 / 11.0 * 1j
        a2 = 4.0 / 3.0 - 2.0 * s2 / 3.0 * 1j
    elif ell == 2:
        s3 = math.sqrt(3.0)
        eta = [2.0 / 3.0 + 2.0 * s3 / 3.0 * 1j, -2.0 / 3.0 - 8.0 * s3 / 3.0 * 1j]
        a1 = 3.0 / 4.0 - s3 / 4.0 * 1j
        a2 = 6.0 / 7.0 - 3.0 * s3 / 7.0 * 1j
    else:
        raise ValueError("Table 1 covers ell = 1, 2")
    return (1, 2), np.array(eta), np.array([[a1, a1], [a2, a2]])


def table2_complex(ell: int, d: int):
    """Table 2 (upper signs) for phi_ell (ell in {1, 2}) in dimension d >= 2:
    alpha is the same in every direction, eta_2 carries 2^{d-2}."""
    if d < 2:
        raise ValueError("directional splitting needs d >= 2")
    scale = 2.0 ** (d - 2)
    if ell == 1:
        r = math.sqrt(2.0)
        e1 = 7.0 / 4.0 + 3.0 * r / 2.0 * 1j
        e2 = scale * (-3.0 - 6.0 * r * 1j)
        a1 = 12.0 / 11.0 - 4.0 * r / 11.0 * 1j
        a2 = 4.0 / 3.0 - 2.0 * r / 3.0 * 1j
    elif ell == 2:
        r = math.sqrt(3.0)
        e1 = 2.0 / 3.0 + 2.0 * r / 3.0 * 1j
        e2 = scale * (-2.0 / 3.0 - 8.0 * r / 3.0 * 1j)
        a1 = 3.0 / 4.0 - r / 4.0 * 1j
        a2 = 6.0 / 7.0 - 3.0 * r / 7.0 * 1j
    else:
        raise ValueError("Table 2 covers ell = 1, 2")
    return (1, 2), np.array([e1, e2]), np.array([[a1] * d, [a2] * d])


def split_coefficients_cplx(ell: int, d: int):
    """The complex splitting used by exprk3ds_cplx: Table 1's complex column
    for d = 2, Table 2 for d > 2."""
    if d == 2:
        return table1_complex(ell)
    return table2_complex(ell, d)


def split_coefficients(ell: int, d: int):
    """The real splitting used by exprk3ds_real: Table 1 for d = 2
    (Algorithm 1), Table 3 for d > 2 (Algorithm 2)."""
    if d == 2:
        return table1_real(ell)
    if d >= 3:
        return table3_real(ell, d)
    raise ValueError("directional splitting needs d >= 2")
