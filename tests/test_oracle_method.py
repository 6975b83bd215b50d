"""Pins for the oracle's split phi action and split-ETD3 step.

Each check is fixed by the paper or by mathematics, independently of the
oracle's own code paths:

* eq. (expTucker): exp(tau K) v is exactly one Tucker operator with the
  factors exp(tau A_mu); the dense reference is K assembled with numpy.kron and
  its exponential summed as a Taylor series.
* Sections 2.1-2.3: the split phi_l is a third-order approximation: against
  dense phi_l(c tau K) (Taylor series of the assembled K), the error ratio
  tends to 8 when tau halves; the second-order formula eq. (secondord) gives 4.
* A_mu = 0: S_l = I/l!, so eq. (exprk3) becomes Heun's third-order
  Runge-Kutta method (written out here from the textbook tableau).
* g = 0 on a separable Neumann eigenmode: one step multiplies the mode by
  R = 1 + tau Lambda sum_i eta_i prod_mu phi_{l_i}(tau alpha_{i,mu} lambda_mu)
  (scalar, 40-digit), and |R| <= 1 for the diffusion operators used here.
* Temporal order 3 by step halving on smooth data (Section 3 reports order 3).
* Reaction terms vanish on their nullclines / at the Schnakenberg steady state.
"""
import math
from functools import reduce

import mpmath
import numpy as np
import pytest

import oracle
from oracle import coeffs, etd, tensor
from workloads import G_FHN, G_NONE, G_SCHNAKENBERG, neumann_d2, random_tensor, smooth_fields


def _vec(T):
    return T.ravel(order="F")


def _dense_K(As):
    dims = [A.shape[0] for A in As]
    K = 0
    for mu in range(len(As)):
        mats = [np.eye(n) for n in dims]
        mats[mu] = As[mu]
        K = K + reduce(np.kron, mats[::-1])
    return K


def _taylor_phi(X, ell, terms=60):
    out = np.zeros_like(X)
    term = np.eye(X.shape[0])
    for k in range(terms):
        out += term / math.factorial(k + ell)
        term = term @ X
    return out


def _small_As(dims, scale=1.0):
    return [scale * neumann_d2(n) / (n - 1) ** 2 * 0.25 for n in dims]


def test_exp_tucker_exact():
    dims = (3, 4, 5)
    As = [0.3 * np.random.default_rng(k).standard_normal((n, n)) for k, n in enumerate(dims)]
    V = random_tensor(dims, 2)
    tau = 0.7
    dense = _taylor_phi(tau * _dense_K(As), 0, terms=80) @ _vec(V)
    tuck = _vec(tensor.tucker(V, [oracle.phi(tau * A, 0) for A in As]))
    assert np.max(np.abs(dense - tuck)) < 1e-13 * np.max(np.abs(dense))


def _split_errors(dims, ell, taus, second_order=False):
    As = [neumann_d2(n) * 0.02 for n in dims]           # ||tau K|| <~ 1 at the taus used
    V = random_tensor(dims, 7)
    K = _dense_K(As)
    errs = []
    for tau in taus:
        ref = _taylor_phi(tau * K, ell) @ _vec(V)
        if second_order:
            got = oracle.split2_apply(As, tau, ell, V)
        else:
            bank = etd.PhiBank(As, tau)                   # stage f: c = 1
            got = bank.split_apply(ell, "f", V)
        errs.append(np.linalg.norm(_vec(got) - ref) / np.linalg.norm(ref))
    return np.array(errs)


@pytest.mark.parametrize("dims", [(3, 4), (3, 4, 5)])
@pytest.mark.parametrize("ell", [1, 2])
def test_split_phi_third_order(dims, ell):
    taus = [0.4 / 2 ** k for k in range(5)]
    e = _split_errors(dims, ell, taus)
    ratios = e[:-1] / e[1:]
    assert 6.5 < ratios[-1] < 9.5, (e, ratios)
    assert 6.5 < ratios[-2] < 9.5, (e, ratios)


@pytest.mark.parametrize("dims", [(3, 4), (3, 4, 5)])
def test_second_order_split_control(dims):
    taus = [0.4 / 2 ** k for k in range(5)]
    e = _split_errors(dims, 1, taus, second_order=True)
    ratios = e[:-1] / e[1:]
    assert 3.3 < ratios[-1] < 4.7, (e, ratios)


def _heun3_step(U, tau, kind, params):
    """Heun's third-order RK (tableau 0 | 1/3 1/3 | 2/3 0 2/3 | 1/4 0 3/4), written
    out here with its own copy of the reaction formulas."""
    def f(W):
        u, v = W
        if kind == G_FHN:
            eps, a1, a0 = params
            return [u - u ** 3 - v, eps * (u - a1 * v - a0)]
        gam, a, b = params
        return [gam * (a - u + u ** 2 * v), gam * (b - u ** 2 * v)]
    k1 = f(U)
    k2 = f([U[c] + tau / 3 * k1[c] for c in range(2)])
    k3 = f([U[c] + 2 * tau / 3 * k2[c] for c in range(2)])
    return [U[c] + tau / 4 * k1[c] + 3 * tau / 4 * k3[c] for c in range(2)]


@pytest.mark.parametrize("kind,params,dims", [(G_FHN, (0.5, 2.0, 0.1), (4, 5, 3)),
                                              (G_SCHNAKENBERG, (100.0, 0.1, 0.9), (6, 5))])
def test_zero_diffusion_is_heun3(kind, params, dims):
    As = [[np.zeros((n, n)) for n in dims] for _ in range(2)]
    if kind == G_FHN:
        U = [random_tensor(dims, 1, 0.5), random_tensor(dims, 2, 0.5)]
    else:
        U = [1.0 + random_tensor(dims, 1, 0.1), 0.9 + random_tensor(dims, 2, 0.1)]
    tau = 2e-3
    banks = etd.make_banks(As, tau)
    got = etd.etd_step(U, As, banks, tau, kind, params)
    ref = _heun3_step(U, tau, kind, params)
    for c in range(2):
        assert np.max(np.abs(got[c] - ref[c])) < 1e-14 * max(1.0, np.max(np.abs(ref[c])))


def _mp_phi(z, ell):
    z = mpmath.mpf(z)
    if abs(z) < mpmath.mpf("1e-3"):
        return mpmath.nsum(lambda k: z ** int(k) / mpmath.factorial(int(k) + ell), [0, 60])
    s = mpmath.exp(z)
    for k in range(ell):
        s -= z ** k / mpmath.factorial(k)
    return s / z ** ell


def _mode(n, k):
    return np.cos(np.pi * np.arange(n) * k / (n - 1))


def _lam(n, k, delta):
    h = 1.0 / (n - 1)
    return -delta * 4.0 / h ** 2 * math.sin(math.pi * k / (2 * (n - 1))) ** 2


@pytest.mark.parametrize("dims,ks", [((9, 7, 8), (1, 3, 2)), ((12, 10), (2, 5)), ((9, 9, 9), (8, 0, 4))])
def test_eigenmode_amplification(dims, ks):
    mpmath.mp.dps = 40
    d = len(dims)
    deltas = (1.0, 42.1)
    tau = 1e-2
    As = [[delta * neumann_d2(n) for n in dims] for delta in deltas]
    modes = [_mode(n, k) for n, k in zip(dims, ks)]
    mode = reduce(np.multiply.outer, modes)
    U = [np.asfortranarray(mode), np.asfortranarray(0.5 * mode)]
    banks = etd.make_banks(As, tau)
    got = etd.etd_step(U, As, banks, tau, G_NONE, ())
    ells, eta, alpha = coeffs.split_coefficients(1, d)
    for c, delta in enumerate(deltas):
        lam = [_lam(n, k, delta) for n, k in zip(dims, ks)]
        S1 = mpmath.mpf(0)
        for i, li in enumerate(ells):
            term = mpmath.mpf(eta[i])
            for mu in range(d):
                term *= _mp_phi(tau * alpha[i, mu] * lam[mu], li)
            S1 += term
        R = float(1 + tau * sum(lam) * S1)
        ref = R * U[c]
        assert np.max(np.abs(got[c] - ref)) < 1e-13 * np.max(np.abs(U[c])), (c, R)
        assert abs(R) <= 1.0 + 1e-14


@pytest.mark.parametrize("dims,ks", [((9, 7, 8), (1, 3, 2)), ((12, 10), (2, 5))])
def test_eigenmode_linear_reaction_all_stages(dims, ks):
    """FHN at amplitude 1e-9 on a separable eigenmode: u^3 is 1e-18 relative, so
    g(w) = M w with M = [[1, -1], [eps, -eps a1]] and each S_l(c tau) acts on the
    mode as the scalar s_l(c) = sum_i eta_i prod_mu phi_{l_i}(c tau alpha lambda_mu).
    The step of eq. (exprk3) then reduces to a 2x2 recursion (all three stages,
    both phi_1 and phi_2 splittings), evaluated here in 40 digits."""
    mpmath.mp.dps = 40
    d = len(dims)
    deltas = (1.0, 42.1)
    eps, a1 = 0.5, 2.0
    tau = 1e-2
    As = [[delta * neumann_d2(n) for n in dims] for delta in deltas]
    mode = reduce(np.multiply.outer, [_mode(n, k) for n, k in zip(dims, ks)])
    w0 = [mpmath.mpf("1e-9"), mpmath.mpf("-0.7e-9")]
    U = [np.asfortranarray(float(w0[0]) * mode), np.asfortranarray(float(w0[1]) * mode)]
    banks = etd.make_banks(As, tau)
    got = etd.etd_step(U, As, banks, tau, G_FHN, (eps, a1, 0.0))

    def s(ell, c, comp):
        ells, eta, alpha = coeffs.split_coefficients(ell, d)
        lam = [_lam(n, k, deltas[comp]) for n, k in zip(dims, ks)]
        tot = mpmath.mpf(0)
        for i, li in enumerate(ells):
            term = mpmath.mpf(eta[i])
            for mu in range(d):
                term *= _mp_phi(c * tau * alpha[i, mu] * lam[mu], li)
            tot += term
        return tot

    Lam = [sum(_lam(n, k, deltas[c]) for n, k in zip(dims, ks)) for c in range(2)]
    g = lambda w: [w[0] - w[1], eps * (w[0] - a1 * w[1])]
    T = mpmath.mpf(tau)
    G = g(w0)
    F = [Lam[c] * w0[c] + G[c] for c in range(2)]
    third = mpmath.mpf(1) / 3
    w2 = [w0[c] + T / 3 * s(1, third, c) * F[c] for c in range(2)]
    D2 = [g(w2)[c] - G[c] for c in range(2)]
    w3 = [w0[c] + 2 * T / 3 * s(1, 2 * third, c) * F[c] + 4 * T / 3 * s(2, 2 * third, c) * D2[c]
          for c in range(2)]
    D3 = [g(w3)[c] - G[c] for c in range(2)]
    wn = [w0[c] + T * s(1, 1, c) * F[c] + 3 * T / 2 * s(2, 1, c) * D3[c] for c in range(2)]
    for c in range(2):
        ref = float(wn[c]) * mode
        assert np.max(np.abs(got[c] - ref)) < 1e-13 * float(abs(w0[0])), (c, float(wn[c]))


def test_amplification_bounded_on_grid():
    """|R(z)| <= 1 for z_mu = tau lambda_mu <= 0 on a log grid up to 1e7 (d = 2, 3).
    phi of many scalars at once: phi of the diagonal matrix diag(z)."""
    zs = np.concatenate([[0.0], -np.logspace(-4, 7, 23)])
    for d in (2, 3):
        ells, eta, alpha = coeffs.split_coefficients(1, d)
        S1 = 0.0
        for i, li in enumerate(ells):
            factors = [np.diag(oracle.phi(np.diag(alpha[i, mu] * zs), li)) for mu in range(d)]
            S1 = S1 + eta[i] * reduce(np.multiply.outer, factors)
        Z = reduce(np.add.outer, [zs] * d)
        R = 1 + Z * S1
        assert np.max(np.abs(R)) <= 1 + 1e-9, (d, np.max(np.abs(R)))


def _order_run(dims, kind, params, deltas, T, m):
    As = [[delta * neumann_d2(n) for n in dims] for delta in deltas]
    U0 = smooth_fields(dims)
    if kind == G_SCHNAKENBERG:
        U0 = [1.0 + U0[0], 0.9 + U0[1]]
    return oracle.integrate(U0, As, T / m, m, kind, params)


@pytest.mark.parametrize("case", ["fhn3d", "schnak2d"])
def test_temporal_order_three(case):
    if case == "fhn3d":
        dims, kind, params, deltas, T, ms = (8, 8, 8), G_FHN, (0.5, 2.0, 0.0), (1.0, 42.1), 0.08, [4, 8, 16]
    else:
        dims, kind, params, deltas, T, ms = (16, 16), G_SCHNAKENBERG, (100.0, 0.1, 0.9), (1.0, 10.0), 0.02, [5, 10, 20]
    ref = _order_run(dims, kind, params, deltas, T, ms[-1] * 16)
    errs = []
    for m in ms:
        U = _order_run(dims, kind, params, deltas, T, m)
        errs.append(max(np.max(np.abs(U[c] - ref[c])) for c in range(2)))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert 2.6 < rates[-1] < 3.6, (errs, rates)


def test_reaction_fixed_points():
    u = np.linspace(-1.5, 1.5, 11)
    eps, a1, a0 = 0.5, 2.0, 0.3
    g1, _ = oracle.reaction(G_FHN, [u, u - u ** 3], (eps, a1, a0))
    assert np.max(np.abs(g1)) < 1e-15
    v = np.linspace(-1, 1, 11)
    _, g2 = oracle.reaction(G_FHN, [a1 * v + a0, v], (eps, a1, a0))
    assert np.max(np.abs(g2)) < 1e-15
    a, b = 0.1, 0.9
    gs = oracle.reaction(G_SCHNAKENBERG, [np.array([a + b]), np.array([b / (a + b) ** 2])], (100.0, a, b))
    assert max(abs(gs[0][0]), abs(gs[1][0])) < 1e-12
    # rho scales both FHN components
    g_r = oracle.reaction(G_FHN, [u, 0.3 * u], (eps, a1, a0, 2.5))
    g_1 = oracle.reaction(G_FHN, [u, 0.3 * u], (eps, a1, a0))
    assert np.allclose(g_r[0], 2.5 * g_1[0]) and np.allclose(g_r[1], 2.5 * g_1[1])
