"""Pins for the oracle's complex-coefficient splitting (exprk3ds_cplx:
Table 1 complex column for d = 2, Table 2 for d > 2).

* The order conditions, rebuilt from the phi series in complex arithmetic
  (same construction as for Tables 1 and 3).
* Table 2 at d = 2 reduces to Table 1's complex column (stated after
  Theorem 2).
* The real part of the complex split phi action is third order against dense
  phi_l(tau K): error ratio -> 8 when tau halves.
* A_mu = 0: the degree-0 condition makes every split action I/l!, so the
  step is Heun's third-order Runge-Kutta method.
* The conjugate (lower-sign) coefficient set gives the same real part.
* Temporal order 3 by step halving on smooth data (non-stiff diffusion).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import coeffs, etd
from tests.test_oracle_coeffs import _exact_coeff, _multi_indices, _split_coeff
from tests.test_oracle_method import _dense_K, _heun3_step, _taylor_phi, _vec
from workloads import G_FHN, G_SCHNAKENBERG, neumann_d2, random_tensor, smooth_fields


@pytest.mark.parametrize("ell", [1, 2])
@pytest.mark.parametrize("d", [2, 3, 4])
def test_table2_order_conditions(ell, d):
    ells, eta, alpha = coeffs.table2_complex(ell, d)
    assert ells == (1, 2)
    for deg in range(3):
        for m in _multi_indices(d, deg):
            res = _split_coeff(ells, eta, alpha, m) - _exact_coeff(ell, m)
            assert abs(res) < 2e-14 * max(1.0, abs(eta).max()), (ell, d, m, res)


@pytest.mark.parametrize("ell", [1, 2])
def test_table1_complex_order_conditions_and_table2_reduction(ell):
    ells, eta, alpha = coeffs.table1_complex(ell)
    for deg in range(3):
        for m in _multi_indices(2, deg):
            assert abs(_split_coeff(ells, eta, alpha, m) - _exact_coeff(ell, m)) < 1e-14
    e2, eta2, alpha2 = coeffs.table2_complex(ell, 2)
    assert e2 == ells
    assert np.allclose(eta2, eta, rtol=0, atol=1e-15) and np.allclose(alpha2, alpha, rtol=0, atol=1e-15)


def test_complex_sets_are_not_real():
    """Theorem 2: no real solution for d > 2, so the imaginary parts are nonzero."""
    for ell in (1, 2):
        _, eta, alpha = coeffs.table2_complex(ell, 3)
        assert np.all(np.abs(eta.imag) > 0.5) and np.all(np.abs(alpha.imag) > 0.1)


def _split_errors_cplx(dims, ell, taus):
    As = [neumann_d2(n) * 0.02 for n in dims]
    V = random_tensor(dims, 7)
    K = _dense_K(As)
    errs = []
    for tau in taus:
        ref = _taylor_phi(tau * K, ell) @ _vec(V)
        got = etd.PhiBank(As, tau, "cplx").split_apply(ell, "f", V)
        assert got.dtype == np.float64
        errs.append(np.linalg.norm(_vec(got) - ref) / np.linalg.norm(ref))
    return np.array(errs)


@pytest.mark.parametrize("dims", [(3, 4), (3, 4, 5)])
@pytest.mark.parametrize("ell", [1, 2])
def test_split_phi_cplx_third_order(dims, ell):
    taus = [0.4 / 2 ** k for k in range(5)]
    e = _split_errors_cplx(dims, ell, taus)
    ratios = e[:-1] / e[1:]
    assert 6.5 < ratios[-1] < 9.5, (e, ratios)
    assert 6.5 < ratios[-2] < 9.5, (e, ratios)


@pytest.mark.parametrize("kind,params,dims", [(G_FHN, (0.5, 2.0, 0.1), (4, 5, 3)),
                                              (G_SCHNAKENBERG, (100.0, 0.1, 0.9), (6, 5))])
def test_zero_diffusion_cplx_is_heun3(kind, params, dims):
    As = [[np.zeros((n, n)) for n in dims] for _ in range(2)]
    if kind == G_FHN:
        U = [random_tensor(dims, 1, 0.5), random_tensor(dims, 2, 0.5)]
    else:
        U = [1.0 + random_tensor(dims, 1, 0.1), 0.9 + random_tensor(dims, 2, 0.1)]
    tau = 2e-3
    got = etd.etd_step(U, As, etd.make_banks(As, tau, "cplx"), tau, kind, params)
    ref = _heun3_step(U, tau, kind, params)
    for c in range(2):
        assert np.max(np.abs(got[c] - ref[c])) < 1e-13 * max(1.0, np.max(np.abs(ref[c])))


def test_conjugate_set_gives_same_real_part(monkeypatch):
    dims = (5, 4, 3)
    As = [neumann_d2(n) * 0.3 for n in dims]
    V = random_tensor(dims, 4)
    upper = etd.PhiBank(As, 0.05, "cplx").split_apply(1, 3, V)
    orig = coeffs.split_coefficients_cplx

    def conj(ell, d):
        ells, eta, alpha = orig(ell, d)
        return ells, eta.conj(), alpha.conj()

    monkeypatch.setattr(etd, "split_coefficients_cplx", conj)
    lower = etd.PhiBank(As, 0.05, "cplx").split_apply(1, 3, V)
    assert np.max(np.abs(upper - lower)) < 1e-14 * np.max(np.abs(upper))


def test_temporal_order_three_cplx():
    """Classical order on a non-stiff problem (diffusion 0.01 / 0.421 on 8^3;
    with the 1 / 42.1 diffusion of the workloads the observed rate of this
    variant drops to about 2.2-2.4 at these step sizes, order reduction)."""
    dims, params, deltas, T, ms = (8, 8, 8), (0.5, 2.0, 0.0), (0.01, 0.421), 0.08, [4, 8, 16]
    As = [[delta * neumann_d2(n) for n in dims] for delta in deltas]
    U0 = smooth_fields(dims)
    ref = oracle.integrate(U0, As, T / (ms[-1] * 16), ms[-1] * 16, G_FHN, params, variant="cplx")
    errs = []
    for m in ms:
        U = oracle.integrate(U0, As, T / m, m, G_FHN, params, variant="cplx")
        errs.append(max(np.max(np.abs(U[c] - ref[c])) for c in range(2)))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert 2.6 < rates[-1] < 3.6, (errs, rates)
