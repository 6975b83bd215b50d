"""Pins for the oracle's second-order split integrator etd2rkds (eq. ETD2RK
with the splitting eq. secondord; the paper's comparison method).

* A = 0: phi_1 = I, phi_2 = I/2, so the step is the explicit trapezoidal
  (Heun) method u + tau/2 (g(u) + g(u + tau g(u))), written out here.
* g = 0 on a separable Neumann eigenmode: one step multiplies the mode by
  R = 1 + tau Lambda prod_mu phi_1(tau lambda_mu) (40-digit scalars).
* Step halving on smooth data: observed order 2.
"""
import math
from functools import reduce

import mpmath
import numpy as np
import pytest

import oracle
from workloads import G_FHN, G_NONE, G_SCHNAKENBERG, neumann_d2, random_tensor, smooth_fields


def _mp_phi1(z):
    z = mpmath.mpf(z)
    if abs(z) < mpmath.mpf("1e-3"):
        return mpmath.nsum(lambda k: z ** int(k) / mpmath.factorial(int(k) + 1), [0, 60])
    return (mpmath.exp(z) - 1) / z


def test_zero_diffusion_is_explicit_trapezoid():
    dims = (5, 4, 3)
    As = [[np.zeros((n, n)) for n in dims] for _ in range(2)]
    U = [random_tensor(dims, 1, 0.5), random_tensor(dims, 2, 0.5)]
    eps, a1, a0 = 0.5, 2.0, 0.1
    tau = 3e-3

    def g(W):
        u, v = W
        return [u - u ** 3 - v, eps * (u - a1 * v - a0)]
    k1 = g(U)
    k2 = g([U[c] + tau * k1[c] for c in range(2)])
    ref = [U[c] + tau / 2 * (k1[c] + k2[c]) for c in range(2)]
    got = oracle.integrate_etd2rkds(U, As, tau, 1, G_FHN, (eps, a1, a0))
    for c in range(2):
        assert np.max(np.abs(got[c] - ref[c])) < 1e-15


@pytest.mark.parametrize("dims,ks", [((9, 7, 8), (1, 3, 2)), ((12, 10), (2, 5))])
def test_eigenmode_amplification_second_order(dims, ks):
    mpmath.mp.dps = 40
    tau = 1e-2
    deltas = (1.0, 42.1)
    As = [[delta * neumann_d2(n) for n in dims] for delta in deltas]
    mode = reduce(np.multiply.outer, [np.cos(np.pi * np.arange(n) * k / (n - 1)) for n, k in zip(dims, ks)])
    U = [np.asfortranarray(mode), np.asfortranarray(-0.3 * mode)]
    got = oracle.integrate_etd2rkds(U, As, tau, 1, G_NONE, ())
    for c, delta in enumerate(deltas):
        lam = [-delta * 4.0 * (n - 1) ** 2 * math.sin(math.pi * k / (2 * (n - 1))) ** 2 for n, k in zip(dims, ks)]
        prod = mpmath.mpf(1)
        for l in lam:
            prod *= _mp_phi1(tau * l)
        R = float(1 + tau * sum(lam) * prod)
        assert np.max(np.abs(got[c] - R * U[c])) < 1e-13 * np.max(np.abs(U[c]))


def test_temporal_order_two():
    dims = (8, 8, 8)
    As = [[delta * neumann_d2(n) for n in dims] for delta in (1.0, 42.1)]
    U0 = smooth_fields(dims)
    T = 0.08
    run = lambda m: oracle.integrate_etd2rkds(U0, As, T / m, m, G_FHN, (0.5, 2.0, 0.0))
    ref = run(512)
    errs = [max(np.max(np.abs(run(m)[c] - ref[c])) for c in range(2)) for m in (8, 16, 32)]
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert 1.7 < rates[-1] < 2.4, (errs, rates)
