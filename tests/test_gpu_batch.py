"""GPU parity of the batched integrator (setd_batch_*) against the oracle run
instance by instance: FP64, 1e-12 relative L2 and inf per field, for every
tile shape the tuner can pick, ragged and non-square grids, per-instance
parameters, the dense-K path, d = 3, one component per instance, graph
replay, and the 64-instance workload at full size (sampled instances)."""
import os

import numpy as np
import pytest

import oracle
from tests.gpu_util import dev, rel_err, rel_l2, say, torch
import workloads as wl

pytestmark = pytest.mark.gpu

import paper_2310_07551_amd as setd   # noqa: E402

TOL = 1e-12


def _make(probs):
    A = [[[dev(M) for M in Ac] for Ac in p.A] for p in probs]
    return setd.Batch([p.dims for p in probs], A, probs[0].tau)


def _state(B, probs):
    u = torch().zeros(B.total, dtype=torch().float64, device="cuda")
    for b, p in enumerate(probs):
        for c in range(len(p.U0)):
            B.field(u, b, c).copy_(torch().from_numpy(np.asarray(p.U0[c]).ravel(order="F").copy()))
    return u


def _fields(B, u, b, p):
    return [B.field(u, b, c).cpu().numpy().reshape(p.dims, order="F") for c in range(len(p.U0))]


def _check(B, u, probs, steps, which=None, params=None):
    for b in (range(len(probs)) if which is None else which):
        p = probs[b]
        ref = oracle.integrate(p.U0, p.A, p.tau, steps, p.g_kind, params[b] if params else p.params)
        got = _fields(B, u, b, p)
        for c in range(len(ref)):
            e2, ei = rel_l2(got[c], ref[c]), rel_err(got[c], ref[c])
            say("  inst %d %s field %d rel_l2 %.3e rel_inf %.3e" % (b, p.dims, c, e2, ei))
            assert e2 < TOL and ei < TOL, (b, p.dims, c)


def _ragged():
    # ragged, non-square, mixed with exact tile multiples; d_v varies
    sizes = [(16, 24), (40, 33), (64, 64), (17, 80), (96, 32), (33, 47), (128, 64), (50, 18)]
    rng = np.random.default_rng(7)
    return [wl.schnakenberg_2d(n1, n2, dv=float(rng.uniform(8, 12)), instance=k, tau=1e-3)
            for k, (n1, n2) in enumerate(sizes)]


@pytest.mark.parametrize("t1,tb", [((2, 2, 0), (2, 2, 0)), ((2, 4, 0), (4, 2, 0)), ((4, 4, 2048), (4, 4, 2048)),
                                   ((4, 2, 8192), (2, 4, 8192))])
def test_batch_parity_every_tile_shape(t1, tb):
    probs = _ragged()
    B = _make(probs)
    B.set_tiles(t1, tb)
    u = _state(B, probs)
    say("batch tiles", t1, tb)
    B.step(u, 8, probs[0].g_kind, [p.params for p in probs])
    torch().cuda.synchronize()
    _check(B, u, probs, 8)


def test_batch_tuned_and_per_instance_params():
    probs = _ragged()
    params = [(100.0 + 10 * k, 0.1, 0.9 - 0.01 * k) for k in range(len(probs))]
    B = _make(probs)
    info = B.tune()
    say("tuned", info)
    assert info["tuned"]
    u = _state(B, probs)
    B.step(u, 4, probs[0].g_kind, params)
    B.step(u, 2, probs[0].g_kind, params)   # same lists and graph, replayed
    torch().cuda.synchronize()
    assert B.info()["launches_per_step"] >= 9
    _check(B, u, probs, 6, params=params)


def test_batch_graph_replay_matches_direct_launches():
    probs = _ragged()[:5]
    B = _make(probs)
    B.set_tiles((2, 4, 0), (4, 2, 0))
    ug = _state(B, probs)
    snaps = []
    for _ in range(3):
        B.step(ug, 2, probs[0].g_kind, [p.params for p in probs])
        torch().cuda.synchronize()
        snaps.append(ug.cpu().numpy().copy())
    os.environ["SETD_GRAPH"] = "0"
    try:
        ud = _state(B, probs)
        for k in range(3):
            B.step(ud, 2, probs[0].g_kind, [p.params for p in probs])
            torch().cuda.synchronize()
            assert np.array_equal(ud.cpu().numpy(), snaps[k]), k
    finally:
        del os.environ["SETD_GRAPH"]


def test_batch_dense_k_path():
    """Non-tridiagonal matrices: the K action runs as batched mu-mode products."""
    probs = []
    for k, (n1, n2) in enumerate([(20, 36), (48, 32), (33, 17)]):
        p = wl.schnakenberg_2d(n1, n2, instance=k)
        rng = np.random.default_rng(100 + k)
        for c in range(2):
            for mu in range(2):
                n = p.dims[mu]
                E = rng.standard_normal((n, n))
                p.A[c][mu] = p.A[c][mu] - 5.0 * (E @ E.T) / n   # dense, symmetric, more dissipative
        probs.append(p)
    B = _make(probs)
    B.set_tiles((2, 2, 0), (2, 2, 0))
    u = _state(B, probs)
    B.step(u, 4, probs[0].g_kind, [p.params for p in probs])
    torch().cuda.synchronize()
    _check(B, u, probs, 4)


@pytest.mark.parametrize("dims_list", [[(24, 20), (17, 33), (40, 9)], [(9, 7, 6), (12, 5, 8)]])
def test_batch_single_component_linear(dims_list):
    """One component per instance and no reaction: the batched G/F body with a
    single component, 2D and 3D, ragged sizes.  The oracle's step takes two
    components, so it runs the field twice (the copy is independent of it)."""
    tau = 1e-3
    As = [[[(1.0 + 0.5 * k) * wl.neumann_d2(n) for n in dims]] for k, dims in enumerate(dims_list)]
    U0s = [wl.random_tensor(dims, 20 + k) for k, dims in enumerate(dims_list)]
    B = setd.Batch(dims_list, [[[dev(M) for M in Ac] for Ac in A] for A in As], tau)
    u = torch().zeros(B.total, dtype=torch().float64, device="cuda")
    for b, U in enumerate(U0s):
        B.field(u, b, 0).copy_(torch().from_numpy(np.asarray(U).ravel(order="F").copy()))
    say("single-component batch", dims_list)
    B.step(u, 4, wl.G_NONE, [])
    torch().cuda.synchronize()
    for b, dims in enumerate(dims_list):
        ref = oracle.integrate([U0s[b], U0s[b]], As[b] + As[b], tau, 4, wl.G_NONE, ())[0]
        got = B.field(u, b, 0).cpu().numpy().reshape(dims, order="F")
        e2, ei = rel_l2(got, ref), rel_err(got, ref)
        say("  inst %d %s rel_l2 %.3e rel_inf %.3e" % (b, dims, e2, ei))
        assert e2 < TOL and ei < TOL, (b, dims)
    B.close()


def test_batch_three_dimensional():
    probs = [wl.fhn_3d(dims=dm) for dm in [(16, 20, 12), (32, 32, 32), (21, 17, 13)]]
    for k, p in enumerate(probs):   # distinct data per instance
        rng = np.random.default_rng(50 + k)
        p.U0 = [x + 0.01 * rng.standard_normal(x.shape) for x in p.U0]
    B = _make(probs)
    u = _state(B, probs)
    B.step(u, 3, probs[0].g_kind, [p.params for p in probs])
    torch().cuda.synchronize()
    _check(B, u, probs, 3)


def test_batch_64_instances_full_size_sampled():
    """The 64-instance workload at full size with tuned tiles: every instance
    finite, the smallest, the largest and a middle instance against the oracle."""
    probs = wl.schnakenberg_batch()
    B = _make(probs)
    say("tuned", B.tune())
    u = _state(B, probs)
    steps = 2
    B.step(u, steps, probs[0].g_kind, [p.params for p in probs])
    torch().cuda.synchronize()
    assert torch().isfinite(u).all()
    sizes = [p.N for p in probs]
    order = np.argsort(sizes, kind="stable")
    _check(B, u, probs, steps, which=[int(order[0]), int(order[len(order) // 2]), int(order[-1])])


def _batch_golden(step):
    import importlib.util
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_batch_goldens", os.path.join(here, "make_batch_goldens.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    path = os.path.join(here, "batch64_step%04d.txt" % step)
    assert os.path.exists(path), path
    return mod.read_golden(path)[1]


def test_batch_64_instances_all_against_stored_oracle():
    """All 64 instances of the batching workload (tuned tiles, graph replay)
    through its 100 steps, against the oracle's stored values of every
    instance at steps 20 and 100 (sampled points and whole-field L2 norms)."""
    probs = wl.schnakenberg_batch()
    B = _make(probs)
    say("tuned", B.tune())
    u = _state(B, probs)
    params = [p.params for p in probs]
    done, worst = 0, 0.0
    for step in (20, 100):
        gold = _batch_golden(step)
        B.step(u, step - done, probs[0].g_kind, params)
        torch().cuda.synchronize()
        done = step
        assert torch().isfinite(u).all()
        for b, p in enumerate(probs):
            dims, norms, idx, vals = gold[b]
            assert tuple(dims) == tuple(p.dims)
            for c in range(2):
                f = B.field(u, b, c).cpu().numpy()
                got, ref = f[idx], vals[:, c]
                e2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
                ei = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
                en = abs(np.linalg.norm(f) - norms[c]) / norms[c]
                worst = max(worst, e2, ei, en)
                assert e2 < TOL and ei < TOL and en < TOL, (step, b, p.dims, c, e2, ei, en)
        say("  step %d: all 64 instances within %.3e" % (step, worst))
