"""Pins for the oracle's splitting coefficients (Tables 1 and 3).

The order conditions are rebuilt here from the definition of phi_l
(Section 1) rather than retyped from the printed systems: for commuting
scalars z_mu, sum_i eta_i prod_mu phi_{l_i}(alpha_{i,mu} z_mu) must match the
Taylor coefficients of phi_l(z_1 + ... + z_d) up to total degree 2 (the
approximation is O(tau^3)).  For Table 3 the extra degree-3 monomials z_mu^3
and z_mu z_nu z_xi (eq. addcond) must match too.  The Groebner-basis
polynomials printed in the proof of Theorem 3 (tests/golden) must vanish at
the Table 3 values.
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import coeffs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _multi_indices(d, deg):
    return [m for m in itertools.product(range(deg + 1), repeat=d) if sum(m) == deg]


def _split_coeff(ells, eta, alpha, m):
    """Taylor coefficient of z^m in sum_i eta_i prod_mu phi_{l_i}(alpha_{i,mu} z_mu):
    phi_l(x) = sum_k x^k/(k+l)!, so each factor contributes alpha^k/(k+l_i)!."""
    tot = 0.0
    for i, li in enumerate(ells):
        term = eta[i]
        for mu, k in enumerate(m):
            term *= alpha[i, mu] ** k / math.factorial(k + li)
        tot += term
    return tot


def _exact_coeff(ell, m):
    """Taylor coefficient of z^m in phi_l(z_1 + ... + z_d): multinomial/(|m|+l)!."""
    k = sum(m)
    multinom = math.factorial(k) / np.prod([math.factorial(j) for j in m])
    return multinom / math.factorial(k + ell)


@pytest.mark.parametrize("ell", [1, 2])
def test_table1_order_conditions(ell):
    ells, eta, alpha = coeffs.table1_real(ell)
    assert ells == (1, 2)
    for deg in range(3):
        for m in _multi_indices(2, deg):
            res = _split_coeff(ells, eta, alpha, m) - _exact_coeff(ell, m)
            assert abs(res) < 5e-15, (ell, m, res)


@pytest.mark.parametrize("ell", [1, 2])
@pytest.mark.parametrize("d", [3, 4])
def test_table3_order_conditions(ell, d):
    ells, eta, alpha = coeffs.table3_real(ell, d)
    assert ells == (1, 2, 1)
    for deg in range(3):
        for m in _multi_indices(d, deg):
            res = _split_coeff(ells, eta, alpha, m) - _exact_coeff(ell, m)
            assert abs(res) < 5e-14, (ell, d, m, res)
    # eq. (addcond): pure cubes and products of three distinct directions
    for m in _multi_indices(d, 3):
        if max(m) == 3 or max(m) == 1:
            res = _split_coeff(ells, eta, alpha, m) - _exact_coeff(ell, m)
            assert abs(res) < 5e-14, (ell, d, m, res)


def test_table3_is_not_fourth_order():
    """A mixed cubic monomial (z_1^2 z_2) is not matched: the splitting is
    third order, not more (guards against a test that passes vacuously)."""
    ells, eta, alpha = coeffs.table3_real(1, 3)
    m = (2, 1, 0)
    assert abs(_split_coeff(ells, eta, alpha, m) - _exact_coeff(1, m)) > 1e-4


def test_plus_sign_choice():
    """The '+' set of Section 2.4: alpha_{1,1} (resp. alpha_{1,mu}) takes the
    larger root."""
    _, _, a = coeffs.table1_real(1)
    assert a[0, 0] > a[0, 1]
    assert a[0, 0] == pytest.approx(4 / 3 + 4 * math.sqrt(10) / 15, rel=1e-15)
    _, _, a = coeffs.table1_real(2)
    assert a[0, 0] == pytest.approx(9 / 8 + math.sqrt(33) / 8, rel=1e-15)
    _, e, a = coeffs.table3_real(1, 3)
    assert a[0, 0] > a[2, 0] and e[0] > e[2]


def test_swapped_sign_pairing_breaks_conditions():
    """Pairing eta_1 with alpha_3 (mixing the +/- rows) violates the
    conditions, so the row-by-row pairing in the oracle is the right one."""
    ells, eta, alpha = coeffs.table3_real(1, 3)
    alpha_bad = alpha[[2, 1, 0]]
    worst = max(abs(_split_coeff(ells, eta, alpha_bad, m) - _exact_coeff(1, m))
                for m in _multi_indices(3, 1))
    assert worst > 1e-3


def _load_groebner():
    polys = []
    with open(os.path.join(GOLDEN, "groebner_table3.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            ell, expr = line.split("|")
            polys.append((int(ell), expr.strip()))
    return polys


@pytest.mark.parametrize("ell", [1, 2])
def test_groebner_basis_vanishes_at_table3(ell):
    _, eta, alpha = coeffs.table3_real(ell, 3)
    env = dict(eta1=eta[0], eta2=eta[1], eta3=eta[2], a1=alpha[0, 0], a2=alpha[1, 0], a3=alpha[2, 0])
    polys = [p for (l, p) in _load_groebner() if l == ell]
    assert len(polys) == 6
    for expr in polys:
        # scale by the size of the largest monomial so the residual is relative
        terms = expr.replace("- ", "+ -").split("+")
        mag = max(abs(eval(t, {}, env)) for t in terms if t.strip())
        val = eval(expr, {}, env)
        assert abs(val) <= 1e-14 * mag, (ell, expr, val, mag)


def test_d2_uses_table1_and_d3_table3():
    assert coeffs.split_coefficients(1, 2)[0] == (1, 2)
    assert coeffs.split_coefficients(1, 3)[0] == (1, 2, 1)
    _, e3, _ = coeffs.split_coefficients(1, 3)
    _, e4, _ = coeffs.split_coefficients(1, 4)
    assert e4[1] == pytest.approx(2 * e3[1], rel=1e-15)          # eta_2 ~ 2^{d-3}
    assert e3[1] == pytest.approx(-12544 / 675, rel=1e-15)
