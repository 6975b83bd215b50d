"""Writes the FP64 oracle's reference values for the 3D FitzHugh-Nagumo
workloads (128^3, 100 steps; 256^3, 200 steps) at a few step counts.

Only `oracle/` (the step of Algorithm 2, eq. exprk3 with the Table 3
splitting) and `workloads/` (the seeded initial data and matrices) are called;
nothing here comes from the GPU library.  For every step count in --marks one
text file is written:

    tests/golden/fhn3d_<n>_step<kkkk>.txt

holding the per-field L2 and max norms of the whole oracle field and the
oracle's values at a fixed set of sample points (all 8 corners, the 12 edge
midpoints, the 6 face centres, random points on every face and edge, the
rest random in the volume; drawn from PCG64 seed 20231011).  Values are
written with repr(), which round-trips FP64 exactly.

Usage:
    python tests/golden/make_fhn3d_goldens.py --n 128 --marks 1,10,100
    python tests/golden/make_fhn3d_goldens.py --n 256 --marks 1,20,100,200 --state-dir /tmp/fhn256

--state-dir keeps the oracle state every --save-every steps so an
interrupted run continues from its last saved step.
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

SAMPLE_SEED = 20231011
NSAMPLES = 4096


def sample_points(dims):
    """Flat (Fortran-order) indices of the sample points, sorted, unique."""
    n1, n2, n3 = dims
    rng = np.random.default_rng(SAMPLE_SEED)
    pts = set()
    ends = [(0, n1 - 1), (0, n2 - 1), (0, n3 - 1)]
    mids = [(n1 - 1) // 2, (n2 - 1) // 2, (n3 - 1) // 2]
    n = (n1, n2, n3)
    for a in ends[0]:
        for b in ends[1]:
            for c in ends[2]:
                pts.add((a, b, c))
    # edge midpoints and random points along each edge (two coordinates fixed at an end)
    for free in range(3):
        fixed = [m for m in range(3) if m != free]
        for e0 in ends[fixed[0]]:
            for e1 in ends[fixed[1]]:
                for t in [mids[free]] + list(rng.integers(0, n[free], size=8)):
                    p = [0, 0, 0]
                    p[free] = int(t)
                    p[fixed[0]], p[fixed[1]] = e0, e1
                    pts.add(tuple(p))
    # face centres and random points on each face (one coordinate at an end)
    for fixed in range(3):
        free = [m for m in range(3) if m != fixed]
        for e in ends[fixed]:
            ab = [(mids[free[0]], mids[free[1]])] + list(zip(rng.integers(0, n[free[0]], size=64),
                                                             rng.integers(0, n[free[1]], size=64)))
            for a, b in ab:
                p = [0, 0, 0]
                p[fixed] = e
                p[free[0]], p[free[1]] = int(a), int(b)
                pts.add(tuple(p))
    while len(pts) < NSAMPLES:
        pts.add(tuple(int(rng.integers(0, n[m])) for m in range(3)))
    flat = sorted(i + n1 * (j + n2 * k) for (i, j, k) in pts)
    return np.asarray(flat, dtype=np.int64)


def write_mark(path, prob, step, U, idx):
    with open(path, "w") as f:
        f.write("# FP64 oracle (oracle.etd.etd_step) for workloads.%s dims=%s tau=%r params=%r\n"
                % ("fhn_3d", prob.dims, prob.tau, prob.params))
        f.write("# initial data: workloads.fhn_3d seeds 0 (u), 1 (v); written by tests/golden/make_fhn3d_goldens.py\n")
        f.write("step %d\n" % step)
        for c, name in enumerate(("u", "v")):
            x = U[c].ravel(order="F")
            f.write("norm %s l2 %r\n" % (name, float(np.linalg.norm(x))))
            f.write("norm %s inf %r\n" % (name, float(np.max(np.abs(x)))))
        f.write("samples %d\n" % len(idx))
        fu, fv = U[0].ravel(order="F"), U[1].ravel(order="F")
        for i in idx:
            f.write("%d %r %r\n" % (int(i), float(fu[i]), float(fv[i])))


def read_golden(path):
    """(step, norms {('u','l2'): .., ...}, idx, values (nsamples, 2))."""
    norms, rows, step = {}, [], None
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "step":
                step = int(parts[1])
            elif parts[0] == "norm":
                norms[(parts[1], parts[2])] = float(parts[3])
            elif parts[0] == "samples":
                continue
            else:
                rows.append((int(parts[0]), float(parts[1]), float(parts[2])))
    idx = np.asarray([r[0] for r in rows], dtype=np.int64)
    vals = np.asarray([(r[1], r[2]) for r in rows], dtype=np.float64)
    return step, norms, idx, vals


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--marks", required=True)
    ap.add_argument("--state-dir", default=None)
    ap.add_argument("--save-every", type=int, default=10)
    ap.add_argument("--out-dir", default=HERE)
    a = ap.parse_args()
    marks = sorted(int(m) for m in a.marks.split(","))
    prob = wl.make("fhn3d_%d" % a.n)
    idx = sample_points(prob.dims)
    banks = oetd.make_banks(prob.A, prob.tau)
    U = [np.array(x, dtype=np.float64, order="F") for x in prob.U0]
    k0 = 0
    if a.state_dir:
        os.makedirs(a.state_dir, exist_ok=True)
        saved = sorted(int(f[5:11]) for f in os.listdir(a.state_dir) if f.startswith("state") and f.endswith(".npz"))
        if saved:
            k0 = saved[-1]
            with np.load(os.path.join(a.state_dir, "state%06d.npz" % k0), allow_pickle=False) as z:
                U = [np.asfortranarray(z["u"]), np.asfortranarray(z["v"])]
            print("resumed at step", k0, flush=True)
    t0 = time.time()
    for k in range(k0, marks[-1]):
        U = oetd.etd_step(U, prob.A, banks, prob.tau, prob.g_kind, prob.params)
        step = k + 1
        print("step %d  %.0f s" % (step, time.time() - t0), flush=True)
        if step in marks:
            path = os.path.join(a.out_dir, "fhn3d_%d_step%04d.txt" % (a.n, step))
            write_mark(path, prob, step, U, idx)
            print("wrote", path, flush=True)
        if a.state_dir and step % a.save_every == 0:
            tmp = os.path.join(a.state_dir, "tmp.npz")
            np.savez(tmp, u=U[0], v=U[1])
            os.replace(tmp, os.path.join(a.state_dir, "state%06d.npz" % step))
            prev = os.path.join(a.state_dir, "state%06d.npz" % (step - a.save_every))
            if os.path.exists(prev):
                os.remove(prev)


if __name__ == "__main__":
    main()
