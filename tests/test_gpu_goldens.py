"""FP64 parity of whole trajectories of the 3D FitzHugh-Nagumo workloads
against stored oracle values (split-ETD3, Algorithm 2 with Table 3).

The oracle needs ~25 s per 256^3 step on 8 host cores, so its values are
stored once by `tests/golden/make_fhn3d_goldens.py` (which calls only the
oracle and the seeded input generators): per field the L2 and max norms of
the whole field and the values at 4096 fixed sample points (corners, edges,
faces, volume).  The library runs the full trajectory in one context and is
compared at every stored step count:

* sample values: relative L2 over the samples and max |x - x_o| / max |x_o|
  over the samples, both below 1e-12 (the FP64 bar);
* whole-field norms: |norm(x) - norm(x_o)| / norm(x_o) below 1e-12 for the L2
  and the max norm.

Both sides evaluate the phi matrices of the stiff directions to within a few
ulps (the oracle through the exact eigen-decomposition, the library in
double-double), so what remains is the rounding of the mode products, stage
sums and reaction.
"""
import glob
import importlib.util
import os

import numpy as np
import pytest

from tests.gpu_util import say, torch
import workloads as wl

pytestmark = pytest.mark.gpu

import paper_2310_07551_amd as setd   # noqa: E402

TOL = 1e-12
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _reader():
    spec = importlib.util.spec_from_file_location("make_fhn3d_goldens", os.path.join(GOLDEN, "make_fhn3d_goldens.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.read_golden


def _marks(n):
    files = sorted(glob.glob(os.path.join(GOLDEN, "fhn3d_%d_step*.txt" % n)))
    assert files, "no stored oracle values for fhn3d_%d" % n
    read = _reader()
    return [read(f) for f in files]


def _compare(u, prob, golden):
    step, norms, idx, vals = golden
    N = prob.N
    host = u.cpu().numpy()
    worst = 0.0
    for c, name in enumerate(("u", "v")):
        x = host[c * N:(c + 1) * N]
        got, ref = x[idx], vals[:, c]
        e2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        ei = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        n2 = abs(np.linalg.norm(x) - norms[(name, "l2")]) / norms[(name, "l2")]
        ninf = abs(np.max(np.abs(x)) - norms[(name, "inf")]) / norms[(name, "inf")]
        say("  step %d field %s: samples rel_l2 %.3e rel_inf %.3e; norms l2 %.3e inf %.3e"
            % (step, name, e2, ei, n2, ninf))
        worst = max(worst, e2, ei, n2, ninf)
    return worst


@pytest.mark.parametrize("n", [128, 256])
def test_fhn3d_trajectory_against_stored_oracle(n):
    """fhn3d_128 (100 steps) and fhn3d_256 (200 steps, the benchmark
    workload), compared at every stored step count."""
    prob = wl.make("fhn3d_%d" % n)
    marks = _marks(n)
    say("fhn %d^3 trajectory, marks" % n, [m[0] for m in marks])
    A = [[torch().from_numpy(M.ravel(order="F").copy()).to("cuda") for M in Ac] for Ac in prob.A]
    ctx = setd.Context(prob.dims, A, prob.tau)
    u = torch().from_numpy(prob.u0_flat()).to("cuda")
    done, worst = 0, []
    for golden in marks:
        ctx.step(u, golden[0] - done, prob.g_kind, prob.params)
        torch().cuda.synchronize()
        done = golden[0]
        worst.append((done, _compare(u, prob, golden)))
    ctx.close()
    for step, w in worst:
        assert w < TOL, (n, step, w)
