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
  arithmetic (numerical inverse of the eigenvector matrix), including stiff
  arguments (c ||D2|| up to ~1e5);
* for that family the oracle's own evaluation (closed-form inverse, cosine
  product-to-sum, long double) is further pinned by identities every phi
  satisfies: exact row sums 1/l! (X 1 = 0), the doubling formulas of the
  modified squaring at the stiff workload arguments, the recurrence, and
  agreement with the augmented-matrix exponential where that is accurate.
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
    # the oracle evaluates this family through its spectral form in long
    # double: within an ulp or two of the 40-digit value (a squaring method
    # in FP64 would be off by about u ||X|| here)
    normx = c * np.abs(D2).sum(0).max()
    tol = 4e-16
    for ell in (1, 2):
        ref = _spectral_phi(n, c, ell)
        got = ophi.phi(c * D2, ell)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err < tol, (n, c, ell, err, normx)


# ---- the spectral evaluation used for multiples of the Neumann pattern ----
# Its arithmetic (closed-form inverse eigenvector matrix, product-to-sum of
# the cosines, long double sums) is pinned by identities that any phi must
# satisfy and that reach the stiff arguments of the 256^3 workload, where the
# augmented-matrix exponential itself is off by about u ||X||.

STIFF = [(256, 0.01 / 3 * 1.6071428571428572 * 42.1), (256, 0.01 * 1.3026308281593812 * 42.1),
         (128, 0.02 / 3 * 0.4414417180800575 * 42.1), (97, 3.0), (2, 0.7), (3, 5.0)]


def test_neumann_pattern_detection():
    assert ophi_mod().neumann_multiple(2.5 * neumann_d2(7)) == 2.5 * neumann_d2(7)[1, 0]
    assert ophi_mod().neumann_multiple(neumann_d2(2)) is not None
    X = neumann_d2(7)
    X[3, 3] *= 1 + 1e-15
    assert ophi_mod().neumann_multiple(X) is None
    assert ophi_mod().neumann_multiple(random_matrix(5, 1)) is None


def ophi_mod():
    import importlib
    return importlib.import_module("oracle.phi")


@pytest.mark.parametrize("n,c", [(2, 0.3), (5, 0.01), (16, 1e-4), (33, 2e-4), (64, 1e-5), (256, 2e-7)])
def test_spectral_matches_expm_at_moderate_norm(n, c):
    """Where ||X|| <= ~10 the library exponential is accurate to a few ulps."""
    X = c * neumann_d2(n)
    S = ophi.phi_all(X, 3)
    E = ophi.phi_all(X, 3, method="expm")
    for ell in range(4):
        assert np.max(np.abs(S[ell] - E[ell])) <= 2e-15 * np.max(np.abs(E[ell])), (n, c, ell)


@pytest.mark.parametrize("n,c", STIFF)
def test_spectral_constant_mode(n, c):
    """X 1 = 0, so phi_l(X) 1 = 1/l! exactly; every row sums to 1/l!."""
    P = ophi.phi_all(c * neumann_d2(n), 2)
    for ell in range(3):
        assert np.max(np.abs(P[ell].sum(1) - 1.0 / math.factorial(ell))) < 4e-16, (n, c, ell)


@pytest.mark.parametrize("n,c", STIFF)
def test_spectral_doubling_identities(n, c):
    """phi_0(2Y) = phi_0(Y)^2 and phi_k(2Y) = 2^-k (phi_0(Y) phi_k(Y) + sum_{j=1..k} phi_j(Y)/(k-j)!)
    at the stiff arguments (both sides evaluated, one product in FP64)."""
    X = c * neumann_d2(n)
    Y = ophi.phi_all(0.5 * X, 2)
    P = ophi.phi_all(X, 2)
    for k in range(3):
        rhs = Y[0] @ Y[k]
        for j in range(1, k + 1):
            rhs = rhs + Y[j] / math.factorial(k - j)
        rhs = rhs / 2.0 ** k
        err = np.max(np.abs(P[k] - rhs)) / np.max(np.abs(P[k]))
        assert err < 5e-15, (n, c, k, err)


@pytest.mark.parametrize("n,c", [(40, 0.01), (64, 0.05), (256, 1e-4)])
def test_spectral_recurrence(n, c):
    """phi_l(X) = X phi_{l+1}(X) + I/l! for ||X|| up to ~1e3."""
    X = c * neumann_d2(n)
    P = ophi.phi_all(X, 3)
    for ell in range(3):
        rhs = X @ P[ell + 1] + np.eye(n) / math.factorial(ell)
        err = np.max(np.abs(P[ell] - rhs)) / np.max(np.abs(P[ell]))
        assert err < 1e-15 * max(1.0, np.abs(X).sum(0).max()), (n, c, ell, err)


def test_spectral_stiff_against_expm_bound():
    """At the stiff arguments the two evaluations differ by no more than the
    exponential's own u ||X|| error."""
    for n, c in STIFF[:3]:
        X = c * neumann_d2(n)
        S = ophi.phi_all(X, 2)
        E = ophi.phi_all(X, 2, method="expm")
        nx = np.abs(X).sum(0).max()
        for ell in range(3):
            assert np.max(np.abs(S[ell] - E[ell])) / np.max(np.abs(S[ell])) < 2.2e-16 * nx
