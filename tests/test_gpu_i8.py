"""The error-free int8 slicing form (SETD_PREC_I8X4) against the FP64 oracle.

Each phi row and each tensor fibre is rounded to 30 bits of its largest
entry and the thirteen digit products of order >= 2 are summed exactly, so
each term of a mode product errs by about 2^-29 |x|max |p|max, independent of
any cancellation in the sum.  Kernel checks use 1e-7 relative to the largest
output entry (random data: the sums are ~sqrt(n) |x||p|, so the expected error
is ~sqrt(n) 2^-29 ~ 3e-8 of it).  The integrator is held to the
reduced-precision bar of the benchmark, 1e-5 relative L2 per field, on the
same grids as the FP32 forms, and on the full 200-step 256^3 trajectory
against the oracle's stored values.
"""
import glob
import importlib.util
import os

import numpy as np
import pytest

import oracle
from tests.gpu_util import dev, host, rel_err, rel_l2, say, torch
import workloads as wl

pytestmark = pytest.mark.gpu

import paper_2310_07551_amd as setd   # noqa: E402

I8 = setd.PREC_I8X4
KTOL = 1e-7
TOL = 1e-5


@pytest.mark.parametrize("dims", [(7, 13, 5), (64, 96), (100, 37, 20), (128, 128, 128), (33, 40), (256, 3, 40),
                                  (300, 17), (20, 520), (64, 64, 300), (1, 9, 4)])
def test_tucker_i8(dims):
    """Every mode regime, ragged sizes (not multiples of 64 or of the 32
    columns of a workgroup), contractions beyond one 256-value chunk and
    beyond one 256-row group, alpha and beta."""
    T = wl.random_tensor(dims, 2)
    Ls = [wl.random_matrix(n, 20 + k, scale=1.0 / np.sqrt(n)) for k, n in enumerate(dims)]
    W0 = wl.random_tensor(dims, 3)
    Wd = dev(W0)
    say("tucker i8", dims)
    setd.tucker_apply(dev(T), Wd, dims, [dev(L) for L in Ls], alpha=0.7, beta=1.0, prec=I8)
    ref = 0.7 * oracle.tucker(T, Ls)
    e = rel_err(host(Wd, dims) - W0, ref)
    say("  rel %.3e" % e)
    assert e < KTOL, (dims, e)


def test_single_modes_i8():
    dims = (48, 40, 36)
    T = wl.random_tensor(dims, 5)
    for mu in (1, 2, 3):
        L = wl.random_matrix(dims[mu - 1], 7 + mu, scale=0.2)
        mats = [None] * 3
        mats[mu - 1] = dev(L)
        Wd = torch().empty(int(np.prod(dims)), dtype=torch().float64, device="cuda")
        setd.tucker_apply(dev(T), Wd, dims, mats, prec=I8)
        e = rel_err(host(Wd, dims), oracle.mode_product(T, L, mu))
        assert e < KTOL, (mu, e)


def test_i8_exact_on_representable_operands():
    """Operands that are small integers times powers of two have exact
    digits, so the product is exact (the accumulation rounds nowhere)."""
    dims = (64, 96)
    rng = np.random.default_rng(4)
    T = rng.integers(-1000, 1000, size=dims).astype(np.float64) * 2.0 ** -7
    L = rng.integers(-100, 100, size=(64, 64)).astype(np.float64) * 2.0 ** 3
    Wd = torch().empty(int(np.prod(dims)), dtype=torch().float64, device="cuda")
    setd.tucker_apply(dev(T), Wd, dims, [dev(L), None], prec=I8)
    assert np.array_equal(host(Wd, dims), L @ T)


def test_i8_wide_dynamic_range_and_cancellation():
    """A fibre whose entries span 1e-8 .. 1 and sums that cancel to 1e-6 of
    their terms: the error is bounded by the largest entries, not the result."""
    n = 256
    rng = np.random.default_rng(6)
    T = rng.standard_normal((n, 64)) * 10.0 ** rng.uniform(-8, 0, size=(n, 64))
    L = rng.standard_normal((n, n))
    Wd = torch().empty(n * 64, dtype=torch().float64, device="cuda")
    setd.tucker_apply(dev(T), Wd, (n, 64), [dev(L), None], prec=I8)
    got = host(Wd, (n, 64))
    ref = L @ T
    # per term: two operand roundings of 2^-30 and the three dropped digit pairs (2^-36) of
    # |x|max |p|max, about 2^-29; the bound leaves a factor 8
    bound = n * 2.0 ** -26 * np.abs(L).max(axis=1)[:, None] * np.abs(T).max(axis=0)[None, :]
    assert np.all(np.abs(got - ref) <= bound)


def test_i8_nonfinite_input_propagates():
    dims = (40, 30)
    T = wl.random_tensor(dims, 7)
    T[5, 3] = np.nan
    L = wl.random_matrix(40, 8)
    Wd = torch().empty(int(np.prod(dims)), dtype=torch().float64, device="cuda")
    setd.tucker_apply(dev(T), Wd, dims, [dev(L), None], prec=I8)
    got = host(Wd, dims)
    assert np.all(np.isnan(got[:, 3]))
    assert np.all(np.isfinite(np.delete(got, 3, axis=1)))


def _run(prob, nsteps):
    A = [[dev(M) for M in Ac] for Ac in prob.A]
    ctx = setd.Context(prob.dims, A, prob.tau, prec=I8)
    u = torch().from_numpy(prob.u0_flat()).to("cuda")
    ctx.step(u, nsteps, prob.g_kind, prob.params)
    torch().cuda.synchronize()
    out = u.cpu().numpy()
    return [out[c * prob.N:(c + 1) * prob.N].reshape(prob.dims, order="F") for c in range(2)]


@pytest.mark.parametrize("case", ["schnak64", "fhn_ragged", "fhn128", "fhn_thin256", "fhn256"])
def test_integrator_i8(case):
    if case == "schnak64":
        prob, steps = wl.make("schnakenberg2d_64"), 50
    elif case == "fhn_ragged":
        prob, steps = wl.fhn_3d(dims=(21, 17, 13)), 10
    elif case == "fhn128":
        prob, steps = wl.make("fhn3d_128"), 4
    elif case == "fhn_thin256":
        prob, steps = wl.fhn_3d(dims=(16, 8, 256)), 3
    else:
        prob, steps = wl.make("fhn3d_256"), 1
    say("i8", case, steps)
    got = _run(prob, steps)
    ref = oracle.integrate(prob.U0, prob.A, prob.tau, steps, prob.g_kind, prob.params)
    for c in range(2):
        e = rel_l2(got[c], ref[c])
        say("  field %d rel_l2 %.3e" % (c, e))
        assert e < TOL, (case, c, e)


def test_split_phi_apply_i8():
    prob = wl.fhn_3d(dims=(20, 18, 16))
    A = [[dev(M) for M in Ac] for Ac in prob.A]
    ctx = setd.Context(prob.dims, A, prob.tau, prec=I8)
    bank = oracle.etd.PhiBank(prob.A[0], prob.tau)
    V = wl.random_tensor(prob.dims, 9)
    Wd = torch().zeros(prob.N, dtype=torch().float64, device="cuda")
    ctx.split_phi_apply(0, 2, setd.STAGE_F, dev(V), Wd, scale=1.0, beta=0.0)
    assert rel_l2(host(Wd, prob.dims), bank.split_apply(2, "f", V)) < KTOL * 10


def _stored(n):
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_fhn3d_goldens", os.path.join(here, "make_fhn3d_goldens.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    files = sorted(glob.glob(os.path.join(here, "fhn3d_%d_step*.txt" % n)))
    assert files
    return [mod.read_golden(f) for f in files]


@pytest.mark.parametrize("n", [128, 256])
def test_i8_trajectory_against_stored_oracle(n):
    """The whole trajectory of fhn3d_128 (100 steps) and of the 256^3
    benchmark workload (200 steps) in the int8 form, against the FP64
    oracle's stored values at every stored step count: 1e-5 over the sampled
    points (relative L2 and max) and on the whole-field norms."""
    prob = wl.make("fhn3d_%d" % n)
    A = [[dev(M) for M in Ac] for Ac in prob.A]
    ctx = setd.Context(prob.dims, A, prob.tau, prec=I8)
    u = torch().from_numpy(prob.u0_flat()).to("cuda")
    done = 0
    for step, norms, idx, vals in _stored(n):
        ctx.step(u, step - done, prob.g_kind, prob.params)
        torch().cuda.synchronize()
        done = step
        x = u.cpu().numpy()
        for c, name in enumerate(("u", "v")):
            f = x[c * prob.N:(c + 1) * prob.N]
            got, ref = f[idx], vals[:, c]
            e2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            ei = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
            en = abs(np.linalg.norm(f) - norms[(name, "l2")]) / norms[(name, "l2")]
            say("  step %d field %s: samples rel_l2 %.3e rel_inf %.3e norm %.3e" % (step, name, e2, ei, en))
            assert e2 < TOL and ei < TOL and en < TOL, (n, step, name, e2, ei, en)


@pytest.mark.parametrize("dims", [(100, 256, 7), (64, 128, 5), (256, 256, 3), (37, 256), (130, 128),
                                  (128, 256, 20), (256, 128, 7), (128, 128, 100), (128, 128, 300)])
def test_fused_mode2_digits_i8(dims):
    """Grids whose second side is 128 or 256, where the mode-1 products emit
    the digits of the mode-2 operand directly instead of an FP64
    intermediate: ragged first and third sides, a partial last row panel
    (rows past n1 must not touch other fibres), and the 2D form in which
    mode 2 is also the last mode.  With n1 in {128, 256} too (3D) the
    products run in the order 3, 1, 2 and mode 3 emits the mode-1 digits as
    well (ragged and short third sides, both orders of 128 and 256); a third
    side above 256 keeps the order 1, 2, 3 with a chunked last mode.  Same
    bar as the unfused split action."""
    prob = wl.fhn_3d(dims=dims) if len(dims) == 3 else wl.schnakenberg_2d(dims[0], dims[1])
    A = [[dev(M) for M in Ac] for Ac in prob.A]
    ctx = setd.Context(prob.dims, A, prob.tau, prec=I8)
    bank = oracle.etd.PhiBank(prob.A[1], prob.tau)
    V = wl.random_tensor(prob.dims, 11)
    Wd = torch().zeros(prob.N, dtype=torch().float64, device="cuda")
    say("fused i8", dims)
    ctx.split_phi_apply(1, 2, setd.STAGE_F, dev(V), Wd, scale=1.0, beta=0.0)
    e = rel_l2(host(Wd, prob.dims), bank.split_apply(2, "f", V))
    say("  rel_l2 %.3e" % e)
    assert e < KTOL * 10, (dims, e)


def test_fused_mode2_digits_nonfinite_i8():
    """A NaN in the operand of the fused form: the fibres it reaches get the
    non-finite exponent and every output they feed is NaN, as in the
    oracle."""
    prob = wl.schnakenberg_2d(37, 256)
    A = [[dev(M) for M in Ac] for Ac in prob.A]
    ctx = setd.Context(prob.dims, A, prob.tau, prec=I8)
    bank = oracle.etd.PhiBank(prob.A[0], prob.tau)
    V = wl.random_tensor(prob.dims, 12)
    V[5, 77] = np.nan
    Wd = torch().zeros(prob.N, dtype=torch().float64, device="cuda")
    ctx.split_phi_apply(0, 1, setd.STAGE_F, dev(V), Wd, scale=1.0, beta=0.0)
    got = host(Wd, prob.dims)
    ref = bank.split_apply(1, "f", V)
    assert np.array_equal(np.isnan(got), np.isnan(ref))


def test_fused_order_312_nonfinite_i8():
    """A NaN in the operand of the 3, 1, 2 form: every output it reaches
    through the three products is NaN, the others finite, as in the oracle."""
    prob = wl.fhn_3d(dims=(128, 128, 9))
    A = [[dev(M) for M in Ac] for Ac in prob.A]
    ctx = setd.Context(prob.dims, A, prob.tau, prec=I8)
    bank = oracle.etd.PhiBank(prob.A[0], prob.tau)
    V = wl.random_tensor(prob.dims, 13)
    V[3, 4, 5] = np.nan
    Wd = torch().zeros(prob.N, dtype=torch().float64, device="cuda")
    ctx.split_phi_apply(0, 1, setd.STAGE_F, dev(V), Wd, scale=1.0, beta=0.0)
    assert np.array_equal(np.isnan(host(Wd, prob.dims)), np.isnan(bank.split_apply(1, "f", V)))


@pytest.mark.parametrize("dims", [(256, 256, 3), (128, 256, 20), (256, 128, 7), (128, 128, 100), (100, 256, 7),
                                  (37, 256), (130, 128), (64, 128, 5)])
def test_emitted_digits_equal_sliced_digits_i8(dims, monkeypatch):
    """The digits a product emits for the next mode (the fused forms) are the
    ones the slicing kernel cuts from its FP64 result: with emission off
    (SETD_I8_EMIT=0, same order of the modes) the split action is identical
    to the last bit, on full and ragged row panels and both fibre layouts."""
    prob = wl.fhn_3d(dims=dims) if len(dims) == 3 else wl.schnakenberg_2d(dims[0], dims[1])
    A = [[dev(M) for M in Ac] for Ac in prob.A]
    ctx = setd.Context(prob.dims, A, prob.tau, prec=I8)
    V = dev(wl.random_tensor(prob.dims, 14))
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("SETD_I8_EMIT", flag)
        Wd = torch().zeros(prob.N, dtype=torch().float64, device="cuda")
        ctx.split_phi_apply(1, 2, setd.STAGE_F, V, Wd, scale=1.0, beta=0.0)
        out.append(host(Wd, prob.dims))
    say("emitted == sliced", dims)
    assert np.array_equal(out[0], out[1]), (dims, np.abs(out[0] - out[1]).max())


@pytest.mark.parametrize("dims", [(128, 128, 40), (256, 128, 100), (128, 256, 256)])
def test_fused_stage_slicing_bit_identical_i8(dims, monkeypatch):
    """In the order 3, 1, 2 the stage differences D2 = g(U2) - G and
    D3 = g(U3) - G are cut into their mode-3 digits in the pass that forms
    them, without an FP64 D.  Whole steps agree to the last bit with the
    steps that form D in FP64 and slice it afterwards (SETD_I8_EMIT=0, which
    also turns the digit emission between products off; same order of the
    modes), and stay within the reduced-precision bar of the oracle."""
    prob = wl.fhn_3d(dims=dims)
    runs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("SETD_I8_EMIT", flag)
        runs.append(_run(prob, 3))
    say("fused stage slicing", dims)
    for c in range(2):
        assert np.array_equal(runs[0][c], runs[1][c]), (dims, c, np.abs(runs[0][c] - runs[1][c]).max())
    ref = oracle.integrate(prob.U0, prob.A, prob.tau, 3, prob.g_kind, prob.params)
    for c in range(2):
        assert rel_l2(runs[0][c], ref[c]) < TOL, (dims, c)
