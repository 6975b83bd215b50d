"""Host-side logic that needs no GPU: argument checks of the Python binding
(before anything reaches the library), the workload generators' recipes,
and the benchmark's one-GPU contract."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import paper_2310_07551_amd as setd
from paper_2310_07551_amd import autograd as sad
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_binding_rejects_host_tensors():
    A = torch.zeros(16, dtype=torch.float64)
    with pytest.raises(TypeError):
        setd.phi_matrices(A, 0.1, 1)
    with pytest.raises(TypeError):
        setd.Context((4, 4), [[A, A], [A, A]], 0.1)
    with pytest.raises(TypeError):
        setd.Batch([(4, 4)], [[[A, A], [A, A]]], 0.1)


def test_batch_binding_shape_checks():
    A = torch.zeros(16, dtype=torch.float64)
    with pytest.raises(ValueError):
        setd.Batch([], [], 0.1)
    with pytest.raises(ValueError):
        setd.Batch([(4, 4), (4, 4, 4)], [[[A, A]], [[A, A, A]]], 0.1)


def test_autograd_rejects_bad_checkpoint():
    with pytest.raises(ValueError):
        sad.integrate(torch.zeros(4, dtype=torch.float64), torch.zeros(3, dtype=torch.float64),
                      torch.ones(2, dtype=torch.float64), dims=(2,), D=[[None], [None]], g_kind=0, tau=0.1,
                      nsteps=1, checkpoint=0)


def test_neumann_d2_rows_and_spectrum():
    n = 9
    D = wl.neumann_d2(n)
    h = 1.0 / (n - 1)
    assert np.allclose(D.sum(axis=1), 0.0)                      # constants are in the kernel
    assert D[0, 0] == -2 / h ** 2 and D[0, 1] == 2 / h ** 2 and D[-1, -2] == 2 / h ** 2
    lam = np.sort(np.linalg.eigvals(D).real)
    k = np.arange(n)
    ref = np.sort(-4 / h ** 2 * np.sin(np.pi * k / (2 * (n - 1))) ** 2)
    assert np.allclose(lam, ref, rtol=1e-12, atol=1e-9)


def test_workload_recipes():
    p = wl.make("schnakenberg2d_64")
    assert p.dims == (64, 64) and p.tau == 1e-3 and p.nsteps == 50
    assert abs(p.U0[0].mean() - 1.0) < 1e-3 and abs(p.U0[1].mean() - 0.9) < 1e-3
    assert np.max(np.abs(p.U0[0] - 1.0)) <= 0.01
    q = wl.make("fhn3d_128")
    assert q.dims == (128, 128, 128) and q.tau == 1e-2 and q.nsteps == 100
    assert abs(q.U0[0].std() - 0.01) < 2e-4
    assert np.allclose(q.A[1][0], 42.1 * q.A[0][0])
    # the batch: 64 instances, sides from the stated set, d_v in [8, 12], reproducible
    b1, b2 = wl.schnakenberg_batch(), wl.schnakenberg_batch()
    assert len(b1) == 64
    for p1, p2 in zip(b1, b2):
        assert p1.dims == p2.dims and all(s in wl.BATCH_SIDES for s in p1.dims)
        dv = p1.A[1][0][1, 1] / p1.A[0][0][1, 1]
        assert 8.0 <= dv <= 12.0
        assert np.array_equal(p1.U0[0], p2.U0[0])
    assert len({p.dims for p in b1}) > 10                          # uneven, non-square


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single" in r.stderr
