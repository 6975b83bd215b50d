"""GPU parity of the mu-mode product / Tucker kernels and the phi builder
against the oracle (FP64).

Tolerance for FP64 products: 1e-13 relative to the largest output entry.  A
mode product sums n <= 512 products of size O(|x| |L|); with FMA rounding the
error is below n * 2^-53 * sum|x||L| ~ 6e-14 of that scale for these inputs
(uniform entries), so 1e-13 leaves room for the different summation order
and still catches any wrong index (errors O(1)).
"""
import numpy as np
import pytest

import oracle
from tests.gpu_util import dev, host, rel_err, say, torch
from workloads import neumann_d2, random_matrix, random_tensor

pytestmark = pytest.mark.gpu

import paper_2310_07551_amd as setd   # noqa: E402

TOL = 1e-13

MODE_SHAPES = [
    (7, 13, 5), (16, 16, 16), (64, 96), (65, 33), (100, 37, 20), (128, 64, 32), (3, 200), (200, 3),
    (33, 47, 61), (1, 9, 4), (256, 5),
]


@pytest.mark.parametrize("dims", MODE_SHAPES)
def test_single_mode_products(dims):
    T = random_tensor(dims, 1)
    Vd = dev(T)
    for mu in range(1, len(dims) + 1):
        L = random_matrix(dims[mu - 1], 10 + mu)
        mats = [None] * len(dims)
        mats[mu - 1] = dev(L)
        say("mode product", dims, "mode", mu)
        Wd = torch().empty_like(Vd)
        setd.tucker_apply(Vd, Wd, dims, mats)
        got = host(Wd, dims)
        ref = oracle.mode_product(T, L, mu)
        assert rel_err(got, ref) < TOL, (dims, mu, rel_err(got, ref))


@pytest.mark.parametrize("dims", [(7, 13, 5), (64, 96), (100, 37, 20), (128, 128, 128), (2, 3, 4, 5)])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (0.5, 1.0), (-2.0, 0.25)])
def test_tucker_all_modes(dims, alpha, beta):
    T = random_tensor(dims, 2)
    W0 = random_tensor(dims, 3)
    Ls = [random_matrix(n, 20 + k, scale=0.3) for k, n in enumerate(dims)]
    say("tucker", dims, alpha, beta)
    Wd = dev(W0)
    setd.tucker_apply(dev(T), Wd, dims, [dev(L) for L in Ls], alpha=alpha, beta=beta)
    ref = alpha * oracle.tucker(T, Ls) + beta * W0
    assert rel_err(host(Wd, dims), ref) < TOL


@pytest.mark.parametrize("dims", [(256, 192), (224, 128), (192, 320), (256, 64, 3), (192, 64, 2)])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (0.7, 1.0)])
def test_mode1_lds_panel_path(dims, alpha, beta):
    """Mode-1 products on the LDS-panel path (192 <= n1 <= 256, n1 % 32 == 0,
    a multiple of 64 columns): full and partial column groups (waves without
    a tile), the epilogue with and without the FP64 base, the product's scale
    (alpha folded into the last matrix); also inside a full Tucker."""
    T = random_tensor(dims, 6)
    W0 = random_tensor(dims, 7)
    L = random_matrix(dims[0], 31, scale=0.3)
    say("mode-1 LDS path", dims, alpha, beta)
    Wd = dev(W0)
    setd.tucker_apply(dev(T), Wd, dims, [dev(L)] + [None] * (len(dims) - 1), alpha=alpha, beta=beta)
    ref = alpha * oracle.mode_product(T, L, 1) + beta * W0
    assert rel_err(host(Wd, dims), ref) < TOL
    Ls = [L] + [random_matrix(n, 40 + k, scale=0.3) for k, n in enumerate(dims[1:])]
    Wd = dev(W0)
    setd.tucker_apply(dev(T), Wd, dims, [dev(M) for M in Ls], alpha=alpha, beta=beta)
    assert rel_err(host(Wd, dims), alpha * oracle.tucker(T, Ls) + beta * W0) < TOL


@pytest.mark.parametrize("dims,mu", [((64, 256, 2), 2), ((128, 192, 3), 2), ((64, 5, 256), 3), ((64, 192), 2)])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (0.7, 1.0)])
def test_modeB_lds_panel_path(dims, mu, alpha, beta):
    """A single mode product along mode mu >= 2 on the LDS-panel path
    (192 <= n <= 256, n % 64 == 0, a multiple of 64 rows per slab): several
    slabs per workgroup group, partial groups, with and without the FP64
    base; also inside a full Tucker."""
    T = random_tensor(dims, 8)
    W0 = random_tensor(dims, 9)
    L = random_matrix(dims[mu - 1], 33, scale=0.3)
    mats = [None] * len(dims)
    mats[mu - 1] = dev(L)
    say("modes>=2 LDS path", dims, mu, alpha, beta)
    Wd = dev(W0)
    setd.tucker_apply(dev(T), Wd, dims, mats, alpha=alpha, beta=beta)
    ref = alpha * oracle.mode_product(T, L, mu) + beta * W0
    assert rel_err(host(Wd, dims), ref) < TOL
    Ls = [random_matrix(nn, 50 + k, scale=0.3) for k, nn in enumerate(dims)]
    Ls[mu - 1] = L
    Wd = dev(W0)
    setd.tucker_apply(dev(T), Wd, dims, [dev(M) for M in Ls], alpha=alpha, beta=beta)
    assert rel_err(host(Wd, dims), alpha * oracle.tucker(T, Ls) + beta * W0) < TOL


def test_tucker_identity_modes_and_workspace():
    dims = (20, 30, 10)
    T = random_tensor(dims, 4)
    L2 = random_matrix(30, 5)
    ws = torch().empty(setd.tucker_workspace_bytes(dims) // 8 + 1, dtype=torch().float64, device="cuda")
    Wd = torch().zeros(int(np.prod(dims)), dtype=torch().float64, device="cuda")
    setd.tucker_apply(dev(T), Wd, dims, [None, dev(L2), None], workspace=ws)
    assert rel_err(host(Wd, dims), oracle.mode_product(T, L2, 2)) < TOL
    # no matrix at all: W = alpha V + beta W
    W1 = dev(T)
    setd.tucker_apply(dev(T), W1, dims, [None, None, None], alpha=2.0, beta=1.0)
    assert rel_err(host(W1, dims), 3.0 * T) < 1e-15


def test_beta_zero_ignores_nan():
    dims = (8, 9)
    T = random_tensor(dims, 6)
    L = [random_matrix(8, 1), random_matrix(9, 2)]
    Wd = torch().full((72,), float("nan"), dtype=torch().float64, device="cuda")
    setd.tucker_apply(dev(T), Wd, dims, [dev(x) for x in L], beta=0.0)
    assert np.all(np.isfinite(host(Wd, dims)))


def test_sampled_tucker_full_size():
    """256^3 Tucker (the benchmark's mode-product size): sampled outputs
    computed one by one, s = sum_{jkl} L1[i,j] L2[m,k] L3[q,l] X[j,k,l]."""
    n = 256
    dims = (n, n, n)
    X = random_tensor(dims, 8)
    Ls = [random_matrix(n, 30 + k, scale=0.1) for k in range(3)]
    Wd = torch().empty(n ** 3, dtype=torch().float64, device="cuda")
    say("tucker 256^3")
    setd.tucker_apply(dev(X), Wd, dims, [dev(L) for L in Ls])
    got = host(Wd, dims)
    rng = np.random.default_rng(0)
    idx = rng.integers(0, n, size=(64, 3))
    idx[:4] = [[0, 0, 0], [n - 1, n - 1, n - 1], [0, n - 1, 0], [n - 1, 0, n - 1]]
    ref = np.array([np.einsum("j,k,l,jkl->", Ls[0][i], Ls[1][m], Ls[2][q], X) for i, m, q in idx])
    val = np.array([got[i, m, q] for i, m, q in idx])
    assert rel_err(val, ref) < 1e-12


def _phi_tol(X):
    # against the oracle's augmented-matrix exponential (general matrices):
    # that FP64 evaluation carries an error of about u ||X|| itself
    return 1e-13 + 4.4e-16 * np.abs(X).sum(0).max()


# Multiples of the Neumann second difference: the oracle evaluates them
# through the exact eigen-decomposition in long double (within an ulp of the
# 40-digit value, pinned on the CPU), and the library rounds a double-double
# Pade / squaring result once, so the two agree to a few FP64 ulps of the
# largest entry whatever ||X|| is.  An FP64 squaring method would be off by
# about u ||X|| (2e-11 at the stiffest 256-point matrix below).
PHI_NEUMANN_TOL = 1e-15


@pytest.mark.parametrize("n,c", [(1, 0.3), (5, 0.0), (9, 1e-3), (33, 0.05), (64, 2.0), (128, 0.5), (256, 0.67),
                                 (512, 0.1), (1000, 0.02)])
def test_phi_matrices_neumann(n, c):
    A = neumann_d2(max(n, 2))[:n, :n] * 42.1 if n > 1 else np.array([[-3.0]])
    say("phi", n, c)
    got = setd.phi_matrices(dev(A), c, 2).cpu().numpy()
    ref = oracle.phi_all(c * A, 2)
    for k in range(3):
        G = got[k].reshape(n, n, order="F")
        say("  order", k, "err %.3e" % rel_err(G, ref[k]))
        assert rel_err(G, ref[k]) < PHI_NEUMANN_TOL, (n, c, k, rel_err(G, ref[k]))


def _bank_scalars(tau, d=3):
    """Every scalar c_s tau alpha_{i,mu} of the phi bank of Algorithm 2
    (Algorithm 1 for d = 2), and tau itself (second-order splitting)."""
    from oracle import etd as oetd
    from oracle.coeffs import split_coefficients
    out = {tau}
    for s, ell in oetd.BANK_ENTRIES:
        _, _, alpha = split_coefficients(ell, d)
        for z in np.ravel(oetd.STAGE_SCALE[s] * tau * alpha):
            out.add(float(z))
    return sorted(out)


@pytest.mark.parametrize("n", [128, 256])
@pytest.mark.parametrize("diff", [1.0, 42.1])
def test_phi_bank_scalars_stiff(n, diff):
    """phi_0..phi_2 at every bank scalar of the 3D FitzHugh-Nagumo workloads
    (tau = 1e-2, d_u = 1, d_v = 42.1; ||X||_1 up to 1.8e5 at n = 256)."""
    A = diff * neumann_d2(n)
    worst = 0.0
    for z in _bank_scalars(1e-2):
        got = setd.phi_matrices(dev(A), z, 2).cpu().numpy()
        ref = oracle.phi_all(z * A, 2)
        for k in range(3):
            e = rel_err(got[k].reshape(n, n, order="F"), ref[k])
            worst = max(worst, e)
            assert e < PHI_NEUMANN_TOL, (n, diff, z, k, e)
    say("phi bank scalars", n, diff, "worst %.3e" % worst)


@pytest.mark.parametrize("n,scale", [(7, 0.5), (40, 3.0), (100, 0.01)])
def test_phi_matrices_general(n, scale):
    A = random_matrix(n, 9, scale=scale) - scale * np.eye(n)
    for ell in (0, 1, 3):
        got = setd.phi_matrices(dev(A), 1.0, ell).cpu().numpy()
        ref = oracle.phi_all(A, ell)
        for k in range(ell + 1):
            G = got[k].reshape(n, n, order="F")
            assert rel_err(G, ref[k]) < _phi_tol(A) * 10, (n, ell, k, rel_err(G, ref[k]))


@pytest.mark.parametrize("n,norm", [(16, 1 - 1e-12), (96, 0.999), (200, 1 - 1e-12)])
def test_phi_matrices_at_the_scaling_threshold(n, norm):
    """||X||_1 at the scaling threshold 1, where no squaring is applied and the
    bound on ||I - D(X)||_1 that fixes the number of inverse-iteration steps
    is reached; non-normal X, all orders up to 4."""
    A = random_matrix(n, 21, scale=1.0)
    A *= norm / np.abs(A).sum(0).max()
    got = setd.phi_matrices(dev(A), 1.0, 4).cpu().numpy()
    ref = oracle.phi_all(A, 4)
    for k in range(5):
        G = got[k].reshape(n, n, order="F")
        assert rel_err(G, ref[k]) < 1e-13, (n, norm, k, rel_err(G, ref[k]))


def test_phi_rejects_nonfinite():
    A = np.eye(4)
    A[1, 2] = np.nan
    with pytest.raises(setd.SetdError) as ei:
        setd.phi_matrices(dev(A), 0.1, 1)
    assert ei.value.code == -4


def test_field_norms_deterministic():
    x = random_tensor((1000, 77), 1)
    y = x + 1e-3 * random_tensor((1000, 77), 2)
    xd, yd = dev(x), dev(y)
    r1 = setd.field_norms(xd, yd)
    r2 = setd.field_norms(xd, yd)
    assert r1 == r2
    assert abs(r1[0] - np.linalg.norm(x)) < 1e-13 * np.linalg.norm(x)
    assert r1[1] == np.max(np.abs(x))
    assert abs(r1[2] - np.linalg.norm(x - y)) < 1e-12 * np.linalg.norm(x - y)
    assert r1[3] == np.max(np.abs(x - y))
    z = x.copy()
    z[3, 4] = np.nan
    assert np.isnan(setd.field_norms(dev(z))[1])
