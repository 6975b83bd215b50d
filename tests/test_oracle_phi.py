"""Pins for the oracle's phi-functions.

* phi_l(0) = I/l!;
* the Taylor series of Section 1 summed term by term for small ||X||;
* the scalar closed forms phi_1(z) = (e^z - 1)/z, phi_2(z) = (e^z - 1 - z)/z^2
  evaluated in 50-digit arithmetic (mpmath);
* the recurrence phi_l(X) = X phi_{l+1}(X) + I/l!;
* the exact spectral form for the Neumann Laplacian used by every workload:
  D2 v_k = lambda_k v_k with v_k[j] = cos(pi j k/(n-1)) and
  lambda_k = -(4/h^2) sin^2(pi k / (2(n-1))), so
  phi_l(c D2) = V diag(phi_l(c lambda_k)) V^{-1}, evaluated in 40-digit
  arithmetic, including stiff arguments (c ||D2|| up to ~1e5).
"""
import math

import mpmath
import numpy as np
import pytest

import oracle as ophi
from workloads import neumann_d2, random_matrix


def _mp_phi(z, ell):
    """Scalar phi_l in high precision: exact formula away from 0, series near 0."""
    z = mpmath.mpf(z)
    if abs(z) < mpmath.mpf("1e-3"):
        return mpmath.nsum(lambda k: z ** int(k) / mpmath.factorial(int(k) + ell), [0, 60])
    s = mpmath.exp(z)
    for k in range(ell):
        s -= z ** k / mpmath.factorial(k)
    return s / z ** ell


@pytest.mark.parametrize("ell", [0, 1, 2, 3])
def test_phi_at_zero(ell):
    n = 5
    P = ophi.phi(np.zeros((n, n)), ell)
    assert np.allclose(P, np.eye(n) / math.factorial(ell), rtol=0, atol=1e-16)


@pytest.mark.parametrize("ell", [0, 1, 2])
def test_phi_taylor_small_norm(ell):
    X = random_matrix(7, 3, scale=0.05)
    ref = np.zeros_like(X)
    term = np.eye(7)
    for k in range(40):
        ref += term / math.factorial(k + ell)
        term = term @ X
    P = ophi.phi(X, ell)
    assert np.max(np.abs(P - ref)) < 2e-16 * 10


@pytest.mark.parametrize("z", [-1e-6, -0.3, -7.0, -250.0, -1e4, 2.5])
def test_phi_scalar_closed_forms(z):
    for ell in (1, 2):
        got = ophi.phi(np.array([[z]]), ell)[0, 0]
        ref = float(_mp_phi(z, ell))
        tol = 1e-14 if z <= 0 else 5e-14        # expm's relative accuracy grows with e^z
        assert abs(got - ref) <= tol * abs(ref), (z, ell, got, ref)


def test_phi_recurrence():
    X = random_matrix(9, 4, scale=2.0) - 3 * np.eye(9)
    P = ophi.phi_all(X, 3)
    for ell in range(3):
        lhs = P[ell]
        rhs = X @ P[ell + 1] + np.eye(9) / math.factorial(ell)
        assert np.max(np.abs(lhs - rhs)) < 1e-13 * max(1.0, np.max(np.abs(lhs)))


def _spectral_phi(n, c, ell, dps=40):
    mpmath.mp.dps = dps
    h = mpmath.mpf(1) / (n - 1)
    V = mpmath.matrix(n, n)
    lam = []
    for k in range(n):
        lam.append(-4 / h ** 2 * mpmath.sin(mpmath.pi * k / (2 * (n - 1))) ** 2)
        for j in range(n):
            V[j, k] = mpmath.cos(mpmath.pi * j * k / (n - 1))
    Vi = V ** -1
    Dg = mpmath.diag([_mp_phi(c * lk, ell) for lk in lam])
    M = V * Dg * Vi
    return np.array([[float(M[i, j]) for j in range(n)] for i in range(n)])


@pytest.mark.parametrize("n,c", [(9, 1e-3), (16, 4e-3), (24, 0.05), (32, 0.2), (40, 20.0), (64, 25.0)])
def test_phi_neumann_spectral(n, c):
    D2 = neumann_d2(n)
    # phi_l(X) for stiff X is only determined to about u*||X|| by X itself
    # (phi_1'(0) = 1/2 on the constant Neumann mode), so the bound has a
    # conditioning term on top of a few ulps.
    normx = c * np.abs(D2).sum(0).max()
    tol = 5e-14 + 2.2e-16 * normx
    for ell in (1, 2):
        ref = _spectral_phi(n, c, ell)
        got = ophi.phi(c * D2, ell)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err < tol, (n, c, ell, err, normx)
