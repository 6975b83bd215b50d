"""GPU parity of exprk3ds_cplx (setd_etd_cplx_step: two complex Tucker terms
per split action, real part kept) against the oracle's complex variant, FP64,
1e-12 relative L2 and inf per field; d = 2 (Table 1 complex column) and d = 3
(Table 2), ragged sizes, the dense-K path, and the graph replay."""
import os

import numpy as np
import pytest

import oracle
from tests.gpu_util import dev, rel_err, rel_l2, say, torch
import workloads as wl

pytestmark = pytest.mark.gpu

import paper_2310_07551_amd as setd   # noqa: E402

TOL = 1e-12


def _run(prob, steps):
    ctx = setd.Context(prob.dims, [[dev(M) for M in Ac] for Ac in prob.A], prob.tau)
    u = torch().from_numpy(prob.u0_flat()).cuda()
    ctx.step_cplx(u, steps, prob.g_kind, prob.params)
    torch().cuda.synchronize()
    out = u.cpu().numpy()
    return [out[c * prob.N:(c + 1) * prob.N].reshape(prob.dims, order="F") for c in range(2)]


def _dense(prob):
    rng = np.random.default_rng(4)
    prob.A = [[M - 3.0 * (lambda E: E @ E.T)(rng.standard_normal(M.shape)) / M.shape[0] for M in Ac]
              for Ac in prob.A]
    return prob


@pytest.mark.parametrize("case", ["schnak64", "schnak_ragged", "fhn_ragged", "fhn48", "dense2d"])
def test_cplx_parity(case):
    if case == "schnak64":
        prob, steps = wl.make("schnakenberg2d_64"), 20
    elif case == "schnak_ragged":
        prob, steps = wl.schnakenberg_2d(37, 50), 10
    elif case == "fhn_ragged":
        prob, steps = wl.fhn_3d(dims=(21, 17, 13)), 5
    elif case == "fhn48":
        prob, steps = wl.fhn_3d(n=48), 4
    else:
        prob, steps = _dense(wl.schnakenberg_2d(24, 30)), 5
    say("cplx", case, prob.dims, steps)
    got = _run(prob, steps)
    ref = oracle.integrate(prob.U0, prob.A, prob.tau, steps, prob.g_kind, prob.params, variant="cplx")
    real = oracle.integrate(prob.U0, prob.A, prob.tau, steps, prob.g_kind, prob.params)
    for c in range(2):
        e2, ei = rel_l2(got[c], ref[c]), rel_err(got[c], ref[c])
        say("  field %d rel_l2 %.3e rel_inf %.3e (cplx vs real method %.2e)" % (c, e2, ei, rel_l2(ref[c], real[c])))
        assert e2 < TOL and ei < TOL


def test_cplx_graph_replay_matches_direct():
    prob = wl.fhn_3d(dims=(20, 16, 12))
    ctx = setd.Context(prob.dims, [[dev(M) for M in Ac] for Ac in prob.A], prob.tau)
    ug = torch().from_numpy(prob.u0_flat()).cuda()
    ctx.step_cplx(ug, 3, prob.g_kind, prob.params)
    torch().cuda.synchronize()
    os.environ["SETD_GRAPH"] = "0"
    try:
        ud = torch().from_numpy(prob.u0_flat()).cuda()
        ctx.step_cplx(ud, 3, prob.g_kind, prob.params)
        torch().cuda.synchronize()
    finally:
        del os.environ["SETD_GRAPH"]
    assert np.array_equal(ug.cpu().numpy(), ud.cpu().numpy())


def test_cplx_and_real_steps_share_a_context():
    """Alternating the two methods on one context keeps each one's result."""
    prob = wl.schnakenberg_2d(32, 40)
    ctx = setd.Context(prob.dims, [[dev(M) for M in Ac] for Ac in prob.A], prob.tau)
    u = torch().from_numpy(prob.u0_flat()).cuda()
    ctx.step(u, 2, prob.g_kind, prob.params)
    ctx.step_cplx(u, 2, prob.g_kind, prob.params)
    ctx.step(u, 1, prob.g_kind, prob.params)
    torch().cuda.synchronize()
    U = oracle.integrate(prob.U0, prob.A, prob.tau, 2, prob.g_kind, prob.params)
    U = oracle.integrate(U, prob.A, prob.tau, 2, prob.g_kind, prob.params, variant="cplx")
    U = oracle.integrate(U, prob.A, prob.tau, 1, prob.g_kind, prob.params)
    out = u.cpu().numpy()
    for c in range(2):
        assert rel_l2(out[c * prob.N:(c + 1) * prob.N], U[c].ravel(order="F")) < TOL
