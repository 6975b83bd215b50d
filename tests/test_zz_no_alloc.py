"""setd_tucker_apply_noalloc (the Tucker operator with the library's per-GPU
scratch array as workspace, no allocation) against setd_tucker_apply on the
same inputs: identical results in every arithmetic, on two calls in a row
(the second on a smaller tensor, so stale scratch contents from the first
call are present), beta handling, and the size limit."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import dev, host, rel_err, say, torch
from workloads import random_matrix, random_tensor

pytestmark = pytest.mark.gpu

import paper_2310_07551_amd as setd   # noqa: E402
from paper_2310_07551_amd import _lib   # noqa: E402


def _both(dims, prec, alpha, beta, seed):
    T = random_tensor(dims, seed)
    W0 = random_tensor(dims, seed + 1)
    Ls = [random_matrix(n, seed + 2 + k, scale=0.3) for k, n in enumerate(dims)]
    mats = [dev(L) for L in Ls]
    Vd = dev(T)
    Wa, Wb = dev(W0), dev(W0)
    setd.tucker_apply(Vd, Wa, dims, mats, alpha=alpha, beta=beta, prec=prec)
    setd.tucker_apply_noalloc(Vd, Wb, dims, mats, alpha=alpha, beta=beta, prec=prec)
    torch().cuda.synchronize()
    return host(Wa, dims), host(Wb, dims), alpha * oracle.tucker(T, Ls) + beta * W0


@pytest.mark.parametrize("prec", [setd.PREC_F64, setd.PREC_F32, setd.PREC_BF16X3, setd.PREC_I8X4])
def test_noalloc_matches_allocating_entry_point(prec):
    for dims, alpha, beta, seed in (((64, 96, 80), 1.0, 0.0, 10), ((20, 30, 17), 0.7, 0.5, 20)):
        say("noalloc", prec, dims, alpha, beta)
        ref_lib, got, ref_oracle = _both(dims, prec, alpha, beta, seed)
        assert np.array_equal(got, ref_lib), (prec, dims, np.max(np.abs(got - ref_lib)))
        tol = {setd.PREC_F64: 1e-13, setd.PREC_I8X4: 1e-7}.get(prec, 1e-5)
        assert rel_err(got, ref_oracle) < tol, (prec, dims, rel_err(got, ref_oracle))


def test_noalloc_largest_fp64_workload_tensor():
    """128^3 (the 3D FitzHugh-Nagumo grid of the 100-step workload) fits the
    scratch array in FP64, in the bf16 split form and in the int8 slicing
    form (its digit buffer included)."""
    dims = (128, 128, 128)
    for prec in (setd.PREC_F64, setd.PREC_BF16X3, setd.PREC_I8X4):
        assert setd.tucker_workspace_bytes(dims, prec) <= _lib.NOALLOC_SCRATCH_BYTES
        T = random_tensor(dims, 3)
        Ls = [random_matrix(128, 40 + k, scale=0.1) for k in range(3)]
        mats = [dev(L) for L in Ls]
        Wa = torch().zeros(128 ** 3, dtype=torch().float64, device="cuda")
        Wb = torch().full((128 ** 3,), float("nan"), dtype=torch().float64, device="cuda")
        setd.tucker_apply(dev(T), Wa, dims, mats, prec=prec)
        setd.tucker_apply_noalloc(dev(T), Wb, dims, mats, prec=prec)
        assert torch().equal(Wa, Wb), prec


def test_noalloc_rejects_tensors_beyond_the_scratch_array():
    dims = (192, 192, 192)
    assert setd.tucker_workspace_bytes(dims) > _lib.NOALLOC_SCRATCH_BYTES
    V = torch().zeros(192 ** 3, dtype=torch().float64, device="cuda")
    W = torch().full((192 ** 3,), 3.0, dtype=torch().float64, device="cuda")
    M = dev(np.eye(192))
    with pytest.raises(setd.SetdError) as ei:
        setd.tucker_apply_noalloc(V, W, dims, [M, M, M])
    assert ei.value.code == _lib.SETD_EINVAL
    assert "scratch" in str(ei.value)
    torch().cuda.synchronize()
    assert bool((W == 3.0).all())
    # argument errors are still reported as by setd_tucker_apply
    with pytest.raises(setd.SetdError) as ei:
        setd.tucker_apply_noalloc(V, W, (192, 0, 192), [M, M, M])
    assert ei.value.code == _lib.SETD_EINVAL
