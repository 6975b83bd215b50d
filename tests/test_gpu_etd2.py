"""GPU parity of the second-order split integrator etd2rkds (setd_etd2_step)
against the oracle, FP64, 1e-12 relative L2 / inf per field (as the
third-order step), and graph replay against direct launches."""
import os

import numpy as np
import pytest

import oracle
from tests.gpu_util import dev, rel_err, rel_l2, say, torch
import workloads as wl

pytestmark = pytest.mark.gpu

import paper_2310_07551_amd as setd   # noqa: E402

TOL = 1e-12


def _gpu(prob, steps, second=True):
    A = [[dev(M) for M in Ac] for Ac in prob.A]
    ctx = setd.Context(prob.dims, A, prob.tau)
    u = torch().from_numpy(prob.u0_flat()).to("cuda")
    (ctx.step2 if second else ctx.step)(u, steps, prob.g_kind, prob.params)
    torch().cuda.synchronize()
    out = u.cpu().numpy()
    return [out[c * prob.N:(c + 1) * prob.N].reshape(prob.dims, order="F") for c in range(2)]


@pytest.mark.parametrize("case", ["schnak64", "fhn_ragged", "fhn64"])
def test_etd2rkds_parity(case):
    if case == "schnak64":
        prob, steps = wl.make("schnakenberg2d_64"), 50
    elif case == "fhn_ragged":
        prob, steps = wl.fhn_3d(dims=(21, 17, 13)), 10
    else:
        prob, steps = wl.fhn_3d(n=64), 5
    say("etd2rkds", case, steps)
    got = _gpu(prob, steps)
    ref = oracle.integrate_etd2rkds(prob.U0, prob.A, prob.tau, steps, prob.g_kind, prob.params)
    for c in range(2):
        e2, ei = rel_l2(got[c], ref[c]), rel_err(got[c], ref[c])
        say("  field %d rel_l2 %.3e rel_inf %.3e" % (c, e2, ei))
        assert e2 < TOL and ei < TOL


def test_graph_replay_matches_direct_launches():
    """The captured step replayed from a hipGraph gives bit-identical results
    to direct launches (same kernels, same order), over several replays with
    host work in between."""
    prob = wl.fhn_3d(dims=(24, 20, 16))
    A = [[dev(M) for M in Ac] for Ac in prob.A]
    ctx = setd.Context(prob.dims, A, prob.tau)
    u_graph = torch().from_numpy(prob.u0_flat()).to("cuda")
    snaps = []
    for k in range(3):
        ctx.step(u_graph, 2, prob.g_kind, prob.params)
        torch().cuda.synchronize()
        snaps.append(u_graph.cpu().numpy().copy())
    os.environ["SETD_GRAPH"] = "0"
    try:
        u_direct = torch().from_numpy(prob.u0_flat()).to("cuda")
        for k in range(3):
            ctx.step(u_direct, 2, prob.g_kind, prob.params)
            torch().cuda.synchronize()
            assert np.array_equal(u_direct.cpu().numpy(), snaps[k]), k
    finally:
        del os.environ["SETD_GRAPH"]
