"""Writes the FP64 oracle's reference values for the batching workload: the
64 independent 2D Schnakenberg instances of uneven size of
`workloads.schnakenberg_batch()` (sides from {64, ..., 512}, d_v ~ U(8, 12),
tau = 1e-3), each run alone by the oracle (Algorithm 1 with the Table 1 real
coefficients).

Only `oracle/` and `workloads/` are called.  For every step count in --marks
one text file is written, tests/golden/batch64_step<kkkk>.txt, holding for
every instance the L2 norm of each whole field and the values at 256 sample
points per instance (its four corners, edge points, the rest random; PCG64
seed 20231012 + instance), written with repr() (exact FP64 round trip).

Usage:
    python tests/golden/make_batch_goldens.py --marks 20,100
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import etd as oetd  # noqa: E402
import workloads as wl  # noqa: E402

SAMPLE_SEED = 20231012
NSAMPLES = 256


def sample_points(dims, instance):
    """Flat (Fortran-order) indices of an instance's sample points, sorted."""
    n1, n2 = dims
    rng = np.random.default_rng(SAMPLE_SEED + instance)
    pts = {(0, 0), (n1 - 1, 0), (0, n2 - 1), (n1 - 1, n2 - 1)}
    for e in (0, n1 - 1):
        for j in rng.integers(0, n2, size=8):
            pts.add((e, int(j)))
    for e in (0, n2 - 1):
        for i in rng.integers(0, n1, size=8):
            pts.add((int(i), e))
    while len(pts) < NSAMPLES:
        pts.add((int(rng.integers(0, n1)), int(rng.integers(0, n2))))
    return np.asarray(sorted(i + n1 * j for i, j in pts), dtype=np.int64)


def read_golden(path):
    """{instance: (dims, norms (2,), idx, values (nsamples, 2))} and the step."""
    out, step, cur = {}, None, None
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            p = line.split()
            if p[0] == "step":
                step = int(p[1])
            elif p[0] == "instance":
                cur = int(p[1])
                out[cur] = [(int(p[2]), int(p[3])), (float(p[4]), float(p[5])), [], []]
            else:
                out[cur][2].append(int(p[0]))
                out[cur][3].append((float(p[1]), float(p[2])))
    return step, {k: (v[0], np.asarray(v[1]), np.asarray(v[2], dtype=np.int64), np.asarray(v[3]))
                  for k, v in out.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--marks", default="20,100")
    ap.add_argument("--out-dir", default=HERE)
    a = ap.parse_args()
    marks = sorted(int(m) for m in a.marks.split(","))
    probs = wl.schnakenberg_batch()
    results = {m: {} for m in marks}
    t0 = time.time()
    for b, p in enumerate(probs):
        banks = oetd.make_banks(p.A, p.tau)
        U = [np.array(x, dtype=np.float64, order="F") for x in p.U0]
        for k in range(1, marks[-1] + 1):
            U = oetd.etd_step(U, p.A, banks, p.tau, p.g_kind, p.params)
            if k in marks:
                results[k][b] = [x.ravel(order="F").copy() for x in U]
        print("instance %d %s done, %.0f s" % (b, p.dims, time.time() - t0), flush=True)
    for k in marks:
        path = os.path.join(a.out_dir, "batch64_step%04d.txt" % k)
        with open(path, "w") as f:
            f.write("# FP64 oracle (oracle.etd.etd_step), each instance of workloads.schnakenberg_batch() alone\n")
            f.write("# written by tests/golden/make_batch_goldens.py; per instance: dims, L2 norms of u and v,\n")
            f.write("# then 'index u v' at its sample points\n")
            f.write("step %d\n" % k)
            for b, p in enumerate(probs):
                fu, fv = results[k][b]
                f.write("instance %d %d %d %r %r\n" % (b, p.dims[0], p.dims[1], float(np.linalg.norm(fu)),
                                                     float(np.linalg.norm(fv))))
                for i in sample_points(p.dims, b):
                    f.write("%d %r %r\n" % (int(i), float(fu[i]), float(fv[i])))
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
