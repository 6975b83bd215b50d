"""Discrete adjoint of the split-ETD3 step, plain FP64 (test infrastructure only).

The step of eq. (exprk3) with the split phi actions (see etd.py) is a
composition of linear maps (the split actions S_l, the Kronecker-sum action
K) and pointwise evaluations of the reaction g.  Its vector-Jacobian product
is obtained by running that composition backwards:

* a split action S V = sum_i eta_i T(V, {P_{i,mu}}) has the transpose
  S^T W = sum_i eta_i T(W, {P_{i,mu}^T}) (a Tucker operator is a Kronecker
  product of its matrices acting on vec V, Section 2 eq. (krontomu), and the
  transpose of a Kronecker product is the product of the transposes);
* K^T = A_d^T (+) ... (+) A_1^T;
* the reaction contributes its pointwise 2 x 2 Jacobian transpose and the
  derivatives with respect to its parameters.

Derivatives with respect to the size of the diffusion: for a component c the
matrices A_mu^(c) are scaled to sigma_c A_mu^(c) and the gradient at
sigma_c = 1 is returned (for A^(v) = d_v D this is d_v times the derivative
with respect to d_v).  A phi matrix phi_l(z sigma A) changes with sigma as
z A phi_l'(z A), and z phi_l'(z) = phi_{l-1}(z) - l phi_l(z) (differentiate
the series phi_l(z) = sum_k z^k/(k+l)! term by term); functions of one
matrix commute, so the same identity holds for the matrices.  The derivative
of a Tucker operator is the sum over directions of the Tucker operator with
that one matrix replaced by its derivative (product rule).

Parity unpinned by the paper (it has no adjoint); pinned instead by central
finite differences of the forward oracle (tests/test_oracle_adjoint.py).
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from .coeffs import split_coefficients
from .etd import BANK_ENTRIES, G_FHN, G_NONE, G_SCHNAKENBERG, STAGE_SCALE, make_banks, reaction
from .phi import phi_all
from .tensor import kron_sum_action, tucker


def reaction_vjp(kind: int, U: Sequence[np.ndarray], params: Sequence[float], Gbar: Sequence[np.ndarray]):
    """(J_g(U)^T Gbar as two fields, d<Gbar, g(U)>/d params as an array)."""
    u, v = U
    gu, gv = Gbar
    npar = len(params)
    pbar = np.zeros(npar)
    if kind == G_NONE:
        return [np.zeros_like(u), np.zeros_like(v)], pbar
    if kind == G_SCHNAKENBERG:
        gamma, a, b = params[:3]
        uv, uu = u * v, u * u
        ubar = gu * gamma * (2.0 * uv - 1.0) - gv * gamma * 2.0 * uv
        vbar = gu * gamma * uu - gv * gamma * uu
        pbar[0] = np.sum(gu * (a - u + uu * v)) + np.sum(gv * (b - uu * v))
        pbar[1] = gamma * np.sum(gu)
        pbar[2] = gamma * np.sum(gv)
        return [ubar, vbar], pbar
    if kind == G_FHN:
        eps, a1, a0 = params[:3]
        rho = params[3] if npar > 3 else 1.0
        ubar = gu * rho * (1.0 - 3.0 * u * u) + gv * rho * eps
        vbar = -gu * rho - gv * rho * eps * a1
        lin = u - a1 * v - a0
        pbar[0] = rho * np.sum(gv * lin)
        pbar[1] = -rho * eps * np.sum(gv * v)
        pbar[2] = -rho * eps * np.sum(gv)
        if npar > 3:
            pbar[3] = np.sum(gu * (u - u * u * u - v)) + eps * np.sum(gv * lin)
        return [ubar, vbar], pbar
    raise ValueError("unknown reaction kind %r" % kind)


class AdjointBank:
    """For one component: the phi matrices P_{i,s}^(l){mu} of the step, and
    their derivatives with respect to the diffusion scale sigma at 1,
    phi_{l_i - 1}(Z) - l_i phi_{l_i}(Z), Z = c_s tau alpha_{i,mu}^(l) A_mu."""

    def __init__(self, As: Sequence[np.ndarray], tau: float):
        self.d = len(As)
        self.P = {}
        self.dP = {}
        self.eta = {}
        for ell in (1, 2):
            self.eta[ell] = split_coefficients(ell, self.d)[1]
        for (s, ell) in BANK_ENTRIES:
            ells, _, alpha = split_coefficients(ell, self.d)
            for i, li in enumerate(ells):
                P, dP = [], []
                for mu, A in enumerate(As):
                    ph = phi_all(STAGE_SCALE[s] * tau * alpha[i, mu] * A, li)
                    P.append(ph[li])
                    dP.append(ph[li - 1] - li * ph[li])
                self.P[(s, ell, i)] = P
                self.dP[(s, ell, i)] = dP

    def apply(self, ell, s, V):
        return sum(self.eta[ell][i] * tucker(V, self.P[(s, ell, i)]) for i in range(len(self.eta[ell])))

    def apply_t(self, ell, s, W):
        """S_l(c_s tau)^T W."""
        return sum(self.eta[ell][i] * tucker(W, [M.T for M in self.P[(s, ell, i)]])
                   for i in range(len(self.eta[ell])))

    def dsigma(self, ell, s, V):
        """d/dsigma of S_l(c_s tau) V at sigma = 1 (all A_mu scaled by sigma)."""
        out = np.zeros_like(V)
        for i in range(len(self.eta[ell])):
            P = self.P[(s, ell, i)]
            for mu in range(self.d):
                mats = list(P)
                mats[mu] = self.dP[(s, ell, i)][mu]
                out = out + self.eta[ell][i] * tucker(V, mats)
        return out


def make_adjoint_banks(As, tau) -> List[AdjointBank]:
    return [AdjointBank(Ac, tau) for Ac in As]


def etd_step_vjp(U, As, abanks, tau, kind, params, Ubar_next):
    """Given U_n and the adjoint of U_{n+1}, returns (adjoint of U_n,
    parameter gradient, diffusion-scale gradient per component) of one step."""
    nc = len(U)
    # forward recomputation of the stage quantities
    G = reaction(kind, U, params)
    F = [kron_sum_action(U[c], As[c]) + G[c] for c in range(nc)]
    U2 = [U[c] + tau / 3.0 * abanks[c].apply(1, 2, F[c]) for c in range(nc)]
    G2 = reaction(kind, U2, params)
    D2 = [G2[c] - G[c] for c in range(nc)]
    U3 = [U[c] + 2.0 * tau / 3.0 * abanks[c].apply(1, 3, F[c]) + 4.0 * tau / 3.0 * abanks[c].apply(2, 3, D2[c])
          for c in range(nc)]
    G3 = reaction(kind, U3, params)
    D3 = [G3[c] - G[c] for c in range(nc)]
    W = Ubar_next
    sig = np.zeros(nc)
    # U_{n+1} = U + tau S1(f) F + 3tau/2 S2(f) D3
    Ubar = [W[c].copy() for c in range(nc)]
    Fbar = [tau * abanks[c].apply_t(1, "f", W[c]) for c in range(nc)]
    D3bar = [1.5 * tau * abanks[c].apply_t(2, "f", W[c]) for c in range(nc)]
    for c in range(nc):
        sig[c] += tau * np.sum(W[c] * abanks[c].dsigma(1, "f", F[c]))
        sig[c] += 1.5 * tau * np.sum(W[c] * abanks[c].dsigma(2, "f", D3[c]))
    # D3 = g(U3) - G
    U3bar, p3 = reaction_vjp(kind, U3, params, D3bar)
    Gbar = [-D3bar[c] for c in range(nc)]
    # U3 = U + 2tau/3 S1(3) F + 4tau/3 S2(3) D2
    D2bar = []
    for c in range(nc):
        Ubar[c] = Ubar[c] + U3bar[c]
        Fbar[c] = Fbar[c] + 2.0 * tau / 3.0 * abanks[c].apply_t(1, 3, U3bar[c])
        D2bar.append(4.0 * tau / 3.0 * abanks[c].apply_t(2, 3, U3bar[c]))
        sig[c] += 2.0 * tau / 3.0 * np.sum(U3bar[c] * abanks[c].dsigma(1, 3, F[c]))
        sig[c] += 4.0 * tau / 3.0 * np.sum(U3bar[c] * abanks[c].dsigma(2, 3, D2[c]))
    # D2 = g(U2) - G
    U2bar, p2 = reaction_vjp(kind, U2, params, D2bar)
    for c in range(nc):
        Gbar[c] = Gbar[c] - D2bar[c]
    # U2 = U + tau/3 S1(2) F
    for c in range(nc):
        Ubar[c] = Ubar[c] + U2bar[c]
        Fbar[c] = Fbar[c] + tau / 3.0 * abanks[c].apply_t(1, 2, U2bar[c])
        sig[c] += tau / 3.0 * np.sum(U2bar[c] * abanks[c].dsigma(1, 2, F[c]))
    # F = K U + G
    for c in range(nc):
        Ubar[c] = Ubar[c] + kron_sum_action(Fbar[c], [A.T for A in As[c]])
        Gbar[c] = Gbar[c] + Fbar[c]
        sig[c] += np.sum(Fbar[c] * kron_sum_action(U[c], As[c]))
    # G = g(U)
    U1bar, p1 = reaction_vjp(kind, U, params, Gbar)
    for c in range(nc):
        Ubar[c] = Ubar[c] + U1bar[c]
    return Ubar, p1 + p2 + p3, sig


def loss_and_gradients(U0, As, tau, nsteps, kind, params, target):
    """L = 1/2 sum_c ||U_c(T) - target_c||^2 after nsteps steps from U0, and its
    gradients: (L, dL/dU0 per component, dL/dparams, dL/dsigma per component)."""
    from .etd import etd_step
    banks = make_banks(As, tau)
    abanks = make_adjoint_banks(As, tau)
    traj = [[np.array(x, dtype=np.float64) for x in U0]]
    for _ in range(nsteps):
        traj.append(etd_step(traj[-1], As, banks, tau, kind, params))
    UT = traj[-1]
    L = 0.5 * sum(float(np.sum((UT[c] - target[c]) ** 2)) for c in range(len(UT)))
    W = [UT[c] - target[c] for c in range(len(UT))]
    pbar = np.zeros(len(params))
    sig = np.zeros(len(UT))
    for n in range(nsteps - 1, -1, -1):
        W, p, s = etd_step_vjp(traj[n], As, abanks, tau, kind, params, W)
        pbar += p
        sig += s
    return L, W, pbar, sig
