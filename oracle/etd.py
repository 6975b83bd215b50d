"""split-ETD3 (exprk3ds_real) time stepping, plain FP64 (test infrastructure only).

Follows the paper's statement of the method step by step:

* the third-order scheme eq. (exprk3): c_2 = 1/3, c_3 = 2/3,
  a_32 = 4/3 phi_2(c_3 .), b_2 = 0, b_3 = 3/2 phi_2(.), for u' = K u + g(u);
* every phi_l(c tau K) v is replaced by its directional split approximation
  S_l(c tau) v = sum_i eta_i^(l) T(V, {phi_{l_i}(c tau alpha_{i,mu}^(l) A_mu)}),
  eq. (split2d) with the Table 1 real coefficients when d = 2 (Algorithm 1)
  and eq. (splitnd3) with Table 3 when d > 2 (Algorithm 2);
* the phi matrices are computed once before time stepping for the stages
  s in {2, 3, f} (argument scale c_s = 1/3, 2/3, 1), phi_1 only for stage 2;
* two components with a block-diagonal K (eq. twocompdisc): K_c is built
  from its own A_mu^(c) and the reaction g couples the components pointwise.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from .coeffs import split_coefficients, split_coefficients_cplx
from .phi import phi
from .tensor import kron_sum_action, tucker

G_NONE = 0
G_SCHNAKENBERG = 1
G_FHN = 2

STAGE_SCALE = {2: 1.0 / 3.0, 3: 2.0 / 3.0, "f": 1.0}
# (stage, ell) pairs of the phi bank, Algorithms 1 and 2.
BANK_ENTRIES = [(2, 1), (3, 1), (3, 2), ("f", 1), ("f", 2)]


def reaction(kind: int, U: Sequence[np.ndarray], params: Sequence[float]) -> List[np.ndarray]:
    """Pointwise nonlinearity g = (g^1, g^2) of the two-component systems.

    None (kind 0): g = 0 (pure linear problem, used by the spectral checks).
    Schnakenberg, params (gamma, a, b): g1 = gamma(a - u + u^2 v), g2 = gamma(b - u^2 v).
    FitzHugh-Nagumo, params (eps, a1, a0[, rho]):
        g1 = rho (u - u^3 - v),  g2 = rho eps (u - a1 v - a0)   (rho = 1 by default).
    """
    u, v = U
    if kind == G_NONE:
        return [np.zeros_like(u), np.zeros_like(v)]
    if kind == G_SCHNAKENBERG:
        gamma, a, b = params[:3]
        u2v = u * u * v
        return [gamma * (a - u + u2v), gamma * (b - u2v)]
    if kind == G_FHN:
        eps, a1, a0 = params[:3]
        rho = params[3] if len(params) > 3 else 1.0
        return [rho * (u - u * u * u - v), rho * eps * (u - a1 * v - a0)]
    raise ValueError("unknown reaction kind %r" % kind)


class PhiBank:
    """P_{i,s}^(l){mu} = phi_{l_i}(c_s tau alpha_{i,mu}^(l) A_mu) for one
    component, with the matching eta_i^(l).

    variant "real": exprk3ds_real (Table 1 real columns for d = 2, Table 3
    for d > 2).  variant "cplx": exprk3ds_cplx (Table 1 complex column for
    d = 2, Table 2 for d > 2): the phi matrices and the sum over the terms are
    complex and a split action returns the real part of that sum (the exact
    phi_l(tau K) v is real; the imaginary part is O(tau^3))."""

    def __init__(self, As: Sequence[np.ndarray], tau: float, variant: str = "real"):
        self.d = len(As)
        self.tau = tau
        self.variant = variant
        coef = split_coefficients if variant == "real" else split_coefficients_cplx
        self.mats: Dict[Tuple, List[np.ndarray]] = {}
        self.eta: Dict[int, np.ndarray] = {}
        self.ells: Dict[int, Tuple[int, ...]] = {}
        cache: Dict[Tuple, np.ndarray] = {}
        for ell in (1, 2):
            ells, eta, _ = coef(ell, self.d)
            self.eta[ell] = eta
            self.ells[ell] = ells
        for (s, ell) in BANK_ENTRIES:
            ells, _, alpha = coef(ell, self.d)
            for i, li in enumerate(ells):
                mats = []
                for mu, A in enumerate(As):
                    z = STAGE_SCALE[s] * tau * alpha[i, mu]
                    key = (A.shape[0], hash(A.tobytes()), z, li)
                    if key not in cache:
                        cache[key] = phi(z * A, li)
                    mats.append(cache[key])
                self.mats[(s, ell, i)] = mats

    def split_apply(self, ell: int, s, V: np.ndarray) -> np.ndarray:
        """S_l(c_s tau) V = sum_i eta_i^(l) T(V, {P_{i,s}^(l){mu}})."""
        out = np.zeros(V.shape, dtype=np.complex128 if self.variant == "cplx" else np.float64)
        for i in range(len(self.ells[ell])):
            out = out + self.eta[ell][i] * tucker(V, self.mats[(s, ell, i)])
        return out.real.copy() if self.variant == "cplx" else out


def etd_step(U: Sequence[np.ndarray], As: Sequence[Sequence[np.ndarray]], banks: Sequence[PhiBank],
             tau: float, kind: int, params: Sequence[float]) -> List[np.ndarray]:
    """One split-ETD3 step (the time-loop body of Algorithms 1 and 2)."""
    nc = len(U)
    G = reaction(kind, U, params)
    F = [kron_sum_action(U[c], As[c]) + G[c] for c in range(nc)]
    U2 = [U[c] + tau / 3.0 * banks[c].split_apply(1, 2, F[c]) for c in range(nc)]
    G2 = reaction(kind, U2, params)
    D2 = [G2[c] - G[c] for c in range(nc)]
    U3 = [U[c] + 2.0 * tau / 3.0 * banks[c].split_apply(1, 3, F[c])
          + 4.0 * tau / 3.0 * banks[c].split_apply(2, 3, D2[c]) for c in range(nc)]
    G3 = reaction(kind, U3, params)
    D3 = [G3[c] - G[c] for c in range(nc)]
    return [U[c] + tau * banks[c].split_apply(1, "f", F[c])
            + 1.5 * tau * banks[c].split_apply(2, "f", D3[c]) for c in range(nc)]


def make_banks(As: Sequence[Sequence[np.ndarray]], tau: float, variant: str = "real") -> List[PhiBank]:
    return [PhiBank(Ac, tau, variant) for Ac in As]


def integrate(U0: Sequence[np.ndarray], As: Sequence[Sequence[np.ndarray]], tau: float, nsteps: int,
              kind: int, params: Sequence[float], banks=None, variant: str = "real") -> List[np.ndarray]:
    """nsteps steps of size tau from U0 (constant step size, as in the
    algorithms); variant "real" (exprk3ds_real) or "cplx" (exprk3ds_cplx)."""
    banks = make_banks(As, tau, variant) if banks is None else banks
    U = [np.array(x, dtype=np.float64, order="F") for x in U0]
    for _ in range(nsteps):
        U = etd_step(U, As, banks, tau, kind, params)
    return U


def split2_apply(As: Sequence[np.ndarray], ctau: float, ell: int, V: np.ndarray) -> np.ndarray:
    """Second-order directional splitting, eq. (secondord):
    phi_l(c tau K) v ~ l!^(d-1) T(V, {phi_l(c tau A_mu)})."""
    d = len(As)
    fact = float(np.prod(np.arange(1, ell + 1))) ** (d - 1)
    return fact * tucker(V, [phi(ctau * A, ell) for A in As])


class Phi2Bank:
    """phi_1(tau A_mu) and phi_2(tau A_mu) for the second-order split integrator."""

    def __init__(self, As: Sequence[np.ndarray], tau: float):
        self.d = len(As)
        self.mats = {ell: [phi(tau * A, ell) for A in As] for ell in (1, 2)}

    def apply(self, ell: int, V: np.ndarray) -> np.ndarray:
        """eq. (secondord) at c = 1: l!^(d-1) T(V, {phi_l(tau A_mu)})."""
        fact = float(np.prod(np.arange(1, ell + 1))) ** (self.d - 1)
        return fact * tucker(V, self.mats[ell])


def etd2rkds_step(U: Sequence[np.ndarray], As: Sequence[Sequence[np.ndarray]], banks: Sequence[Phi2Bank],
                  tau: float, kind: int, params: Sequence[float]) -> List[np.ndarray]:
    """One step of etd2rkds: eq. (ETD2RK),
        u2 = u + tau phi_1(tau K) f(u),  u_new = u2 + tau phi_2(tau K)(g(u2) - g(u)),
    with both phi actions replaced by eq. (secondord)."""
    nc = len(U)
    G = reaction(kind, U, params)
    F = [kron_sum_action(U[c], As[c]) + G[c] for c in range(nc)]
    U2 = [U[c] + tau * banks[c].apply(1, F[c]) for c in range(nc)]
    G2 = reaction(kind, U2, params)
    return [U2[c] + tau * banks[c].apply(2, G2[c] - G[c]) for c in range(nc)]


def integrate_etd2rkds(U0, As, tau: float, nsteps: int, kind: int, params) -> List[np.ndarray]:
    banks = [Phi2Bank(Ac, tau) for Ac in As]
    U = [np.array(x, dtype=np.float64, order="F") for x in U0]
    for _ in range(nsteps):
        U = etd2rkds_step(U, As, banks, tau, kind, params)
    return U
