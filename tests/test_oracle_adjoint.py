"""Pins of the oracle's discrete adjoint (oracle/adjoint.py) against central
finite differences of the forward oracle, which share no code with the
adjoint: gradients with respect to the initial field (random directions),
the reaction parameters, and the diffusion scale of each component, for the
d = 2 (Table 1) and d = 3 (Table 3) splittings; and the phi derivative
identity z phi_l'(z) = phi_{l-1}(z) - l phi_l(z) against differences of phi."""
import numpy as np
import pytest

import oracle
from oracle import adjoint
import workloads as wl

H = 1e-6


def _loss(U0, As, tau, n, kind, params, target):
    UT = oracle.integrate(U0, As, tau, n, kind, params)
    return 0.5 * sum(float(np.sum((UT[c] - target[c]) ** 2)) for c in range(2))


def _case(kind):
    if kind == "schnak":
        p = wl.schnakenberg_2d(6, 5, tau=2e-3)
        p.U0 = [x + 0.05 * np.random.default_rng(3 + c).standard_normal(x.shape) for c, x in enumerate(p.U0)]
        return p, 3
    p = wl.fhn_3d(dims=(5, 4, 3))
    p.U0 = [0.3 * np.random.default_rng(5 + c).standard_normal(x.shape) for c, x in enumerate(p.U0)]
    return p, 3


@pytest.fixture(scope="module", params=["schnak", "fhn"])
def setup(request):
    p, n = _case(request.param)
    rng = np.random.default_rng(11)
    target = [x + 0.1 * rng.standard_normal(x.shape) for x in p.U0]
    L, U0bar, pbar, sig = adjoint.loss_and_gradients(p.U0, p.A, p.tau, n, p.g_kind, p.params, target)
    return p, n, target, L, U0bar, pbar, sig


def test_loss_matches_forward(setup):
    p, n, target, L, *_ = setup
    assert abs(L - _loss(p.U0, p.A, p.tau, n, p.g_kind, p.params, target)) <= 1e-14 * max(1.0, abs(L))


def test_gradient_initial_field_vs_central_differences(setup):
    p, n, target, L, U0bar, _, _ = setup
    rng = np.random.default_rng(21)
    for trial in range(3):
        dU = [rng.standard_normal(x.shape) for x in p.U0]
        lp = _loss([p.U0[c] + H * dU[c] for c in range(2)], p.A, p.tau, n, p.g_kind, p.params, target)
        lm = _loss([p.U0[c] - H * dU[c] for c in range(2)], p.A, p.tau, n, p.g_kind, p.params, target)
        fd = (lp - lm) / (2 * H)
        ad = sum(float(np.sum(U0bar[c] * dU[c])) for c in range(2))
        assert abs(fd - ad) <= 1e-6 * max(abs(fd), 1e-8), (trial, fd, ad)


def test_gradient_reaction_parameters_vs_central_differences(setup):
    p, n, target, L, _, pbar, _ = setup
    for k in range(len(p.params)):
        pp = list(p.params)
        pm = list(p.params)
        pp[k] += H
        pm[k] -= H
        fd = (_loss(p.U0, p.A, p.tau, n, p.g_kind, pp, target) - _loss(p.U0, p.A, p.tau, n, p.g_kind, pm, target)) / (2 * H)
        assert abs(fd - pbar[k]) <= 1e-6 * max(abs(fd), 1e-8), (k, fd, pbar[k])


def test_gradient_diffusion_scale_vs_central_differences(setup):
    p, n, target, L, _, _, sig = setup
    for c in range(2):
        Ap = [[M * ((1 + H) if cc == c else 1.0) for M in Ac] for cc, Ac in enumerate(p.A)]
        Am = [[M * ((1 - H) if cc == c else 1.0) for M in Ac] for cc, Ac in enumerate(p.A)]
        fd = (_loss(p.U0, Ap, p.tau, n, p.g_kind, p.params, target)
              - _loss(p.U0, Am, p.tau, n, p.g_kind, p.params, target)) / (2 * H)
        assert abs(fd - sig[c]) <= 2e-6 * max(abs(fd), 1e-8), (c, fd, sig[c])


@pytest.mark.parametrize("ell", [1, 2])
def test_phi_scale_derivative_identity(ell):
    X = -wl.neumann_d2(7) * 0.01 + 0.02 * np.random.default_rng(1).standard_normal((7, 7))
    ph = oracle.phi_all(X, ell)
    dphi = ph[ell - 1] - ell * ph[ell]
    fd = (oracle.phi((1 + H) * X, ell) - oracle.phi((1 - H) * X, ell)) / (2 * H)
    assert np.max(np.abs(dphi - fd)) <= 1e-8 * np.max(np.abs(dphi))


def test_planted_transpose_mistake_is_caught():
    """Using S instead of S^T in the adjoint (a plausible mistake) breaks the
    finite-difference agreement on a non-symmetric problem."""
    p, n = _case("schnak")
    rng = np.random.default_rng(9)
    p.A = [[M + 0.3 * np.triu(rng.standard_normal(M.shape), 1) for M in Ac] for Ac in p.A]
    target = [x + 0.1 * rng.standard_normal(x.shape) for x in p.U0]
    dU = [rng.standard_normal(x.shape) for x in p.U0]
    lp = _loss([p.U0[c] + H * dU[c] for c in range(2)], p.A, p.tau, n, p.g_kind, p.params, target)
    lm = _loss([p.U0[c] - H * dU[c] for c in range(2)], p.A, p.tau, n, p.g_kind, p.params, target)
    fd = (lp - lm) / (2 * H)
    _, U0bar, _, _ = adjoint.loss_and_gradients(p.U0, p.A, p.tau, n, p.g_kind, p.params, target)
    good = sum(float(np.sum(U0bar[c] * dU[c])) for c in range(2))
    assert abs(fd - good) <= 1e-6 * abs(fd)
    orig = adjoint.AdjointBank.apply_t
    try:
        adjoint.AdjointBank.apply_t = adjoint.AdjointBank.apply
        _, U0bad, _, _ = adjoint.loss_and_gradients(p.U0, p.A, p.tau, n, p.g_kind, p.params, target)
    finally:
        adjoint.AdjointBank.apply_t = orig
    bad = sum(float(np.sum(U0bad[c] * dU[c])) for c in range(2))
    assert abs(fd - bad) > 1e-4 * abs(fd)
