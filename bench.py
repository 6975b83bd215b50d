#!/usr/bin/env python3
"""split-ETD3 throughput on one MI355X.

Default workload: 3D FitzHugh-Nagumo on a 256^3 grid (two components, FP64,
tau = 1e-2; seeded N(0, 0.01^2) initial data), the configuration the metric
is quoted on.  W warm-up steps, then exactly K timed steps between two device
synchronisations; the phi bank is built before (its time is reported apart,
as the paper does).  Prints one JSON line on stdout.

The K timed steps run as the library runs them by default: each step a
replay of its captured hipGraph, no per-launch events.  The same K steps are
then run a second time with every library kernel launch bracketed by HIP
events on its launch stream (setd_profile_*; per-launch events and graph
replay exclude each other): the per-class kernel table and the roofline come
from that pass.  The dominant kernel class (by total time) is reported with
its algorithmic flops (2 N n per mode product term) divided by its measured
time, against the MI355X FP64 matrix peak; each reduced-precision form gets
the same against the peak of its own arithmetic.

Accuracy: for the 3D FitzHugh-Nagumo workloads each form also runs a clean
trajectory of the stored step counts from u0 and is compared with the FP64
oracle's stored values (tests/golden, sampled points and whole-field norms)
and, field by field, with the library's FP64 trajectory.

cpu_baseline: the FP64 oracle timed on this host for a bounded sample of the
same workload (one step by default, phi bank excluded), with the host CPU
model and core counts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "split-ETD3 steps/s + Tucker TFLOP/s (%MFMA peak), 3D FHN 256³, FP64 vs split"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2500.0, "bf16x2": 2500.0, "i8x4": 5000.0}
# matrix-core products per algorithmic product (three-piece split: 6, two-piece: 3,
# int8 digit slicing: the thirteen digit pairs of order >= 2)
MFMA_PER_PRODUCT = {"f64": 1, "f32": 1, "bf16x3": 6, "bf16x2": 3, "i8x4": 13}
PEAK_HBM_GBS = 8000.0
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def mode_flops_per_step(dims, nterms, ncomp=2):
    """Algorithmic Tucker flops of one step: ncomp x 5 split actions'
    worth of Tuckers (3 stages of phi_1 on F, phi_2 on D2, phi_2 on D3) x
    nterms x d mode products x 2 N n_mu."""
    N = 1
    for n in dims:
        N *= n
    per_tucker = sum(2.0 * N * n for n in dims)
    return ncomp * 5 * nterms * per_tucker


# FP64 mode-product kernel classes of setd_profile_read (the panel kernel of
# modes >= 2 is timed apart from the register kernel)
F64_MODE_CLASSES = ("mode1_f64", "modeB_f64", "modeB_panel_f64")
KERNEL_SOURCES = {"mode1_f64": "paper_2310_07551_amd/csrc/mode_f64.hip",
                  "modeB_f64": "paper_2310_07551_amd/csrc/mode_f64.hip",
                  "modeB_panel_f64": "paper_2310_07551_amd/csrc/mode_f64.hip",
                  "mode1_lp": "paper_2310_07551_amd/csrc/mode_lp.hip",
                  "modeB_lp": "paper_2310_07551_amd/csrc/mode_lp.hip",
                  "pointwise": "paper_2310_07551_amd/csrc/pointwise.hip"}


def source_sha1(kernel):
    import hashlib
    with open(os.path.join(ROOT, KERNEL_SOURCES[kernel]), "rb") as fh:
        return hashlib.sha1(fh.read()).hexdigest()


def counted_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    profiles/traffic_<kernel>_<workload>.txt (FETCH_SIZE + WRITE_SIZE per
    dispatch, scaled by the same counters on a copy of known size); None when
    there is no summary or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha1") != source_sha1(kernel):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(mbytes, reps=5):
    """A plain device copy of known size, for scaling the HBM counters."""
    import torch
    n = int(mbytes * 1e6) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    log("copy probe: %d launches of a %d-byte read + %d-byte write" % (reps, n * 8, n * 8))


def library_gemm(n=256, reps=20):
    """The vendor library's FP64 GEMM (torch.matmul: hipBLASLt / rocBLAS) at the
    mode-product shapes of an n^3 grid, as a reference point for the
    library's own kernels (not part of the split-ETD3 path)."""
    import torch
    dev = "cuda"

    def rate(f, flops, it=reps):
        for _ in range(3):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(it):
            f()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / it
        return {"tflops": round(flops / (ms * 1e-3) / 1e12, 2), "ms": round(ms, 4)}

    g = torch.Generator(device=dev).manual_seed(0)
    N = n ** 3
    P = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
    X1 = torch.randn(n, N // n, dtype=torch.float64, device=dev, generator=g)
    Y1 = torch.empty_like(X1)
    XB = torch.randn(N // n, n, dtype=torch.float64, device=dev, generator=g)
    YB = torch.empty_like(XB)
    XM = torch.randn(n, n, n, dtype=torch.float64, device=dev, generator=g)
    YM = torch.empty_like(XM)
    PT = P.t().contiguous()
    out = {"what": "torch.matmul FP64 at the mode-product shapes of a %d^3 grid (2 N n flops each)" % n,
           "mode1_P_X": rate(lambda: torch.matmul(P, X1, out=Y1), 2.0 * N * n),
           "last_mode_X_Pt": rate(lambda: torch.matmul(XB, PT, out=YB), 2.0 * N * n),
           "middle_mode_batched": rate(lambda: torch.matmul(P, XM, out=YM), 2.0 * N * n)}
    m = 8192
    A = torch.randn(m, m, dtype=torch.float64, device=dev, generator=g)
    B = torch.randn(m, m, dtype=torch.float64, device=dev, generator=g)
    out["square_8192"] = rate(lambda: torch.matmul(A, B), 2.0 * m ** 3, it=5)
    print(json.dumps(out), flush=True)


def host_cpu():
    """(model name, physical cores, logical CPUs) of this host from /proc/cpuinfo."""
    model, phys = "unknown", set()
    try:
        cur = {}
        with open("/proc/cpuinfo") as fh:
            for line in fh.read().splitlines() + [""]:
                if not line.strip():
                    if "core id" in cur:
                        phys.add((cur.get("physical id", "0"), cur["core id"]))
                    cur = {}
                    continue
                k, _, v = line.partition(":")
                cur[k.strip()] = v.strip()
                if k.strip() == "model name":
                    model = v.strip()
    except OSError:
        pass
    logical = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = logical
    return model, (len(phys) or None), logical, avail


def read_golden(n, step):
    """Stored FP64 oracle values of fhn3d_<n> at `step` (tests/golden, written
    by tests/golden/make_fhn3d_goldens.py): (norms, sample indices, values)."""
    import numpy as np
    path = os.path.join(GOLDEN_DIR, "fhn3d_%d_step%04d.txt" % (n, step))
    if not os.path.exists(path):
        return None
    norms, rows = {}, []
    for line in open(path):
        if line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "norm":
            norms[(f[1], f[2])] = float(f[3])
        elif f[0] not in ("step", "samples"):
            rows.append((int(f[0]), float(f[1]), float(f[2])))
    idx = np.asarray([r[0] for r in rows], dtype=np.int64)
    vals = np.asarray([(r[1], r[2]) for r in rows])
    return norms, idx, vals


def golden_errors(u, N, golden):
    """Per field: relative L2 and max error over the stored sample points, and
    the relative error of the whole-field L2 norm, against the oracle."""
    import numpy as np
    norms, idx, vals = golden
    x = u.detach().cpu().numpy()
    out = {}
    for c, name in enumerate(("u", "v")):
        f = x[c * N:(c + 1) * N]
        got, ref = f[idx], vals[:, c]
        out[name] = dict(samples_rel_l2=float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                         samples_rel_inf=float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))),
                         norm_l2_rel=float(abs(np.linalg.norm(f) - norms[(name, "l2")]) / norms[(name, "l2")]))
    return out


def cpu_baseline(prob, nsteps):
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(p.get("num_threads", 1)) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    model, phys, logical, avail = host_cpu()
    banks = oracle.make_banks(prob.A, prob.tau)
    U = [np.array(x) for x in prob.U0]
    t0 = time.perf_counter()
    for _ in range(nsteps):
        U = oracle.etd_step(U, prob.A, banks, prob.tau, prob.g_kind, prob.params)
    dt = time.perf_counter() - t0
    return dict(value=nsteps / dt, unit="steps/s", cores=threads, kind="oracle",
                sample="%d step(s) of %s %s (numpy FP64, phi bank excluded), %.1f s" %
                (nsteps, prob.name, "x".join(map(str, prob.dims)), dt),
                cpu_model=model, physical_cores=phys, logical_cpus=logical, cpus_available=avail,
                threads_note="cores = BLAS threads the oracle's products ran on")


def run_batch(torch, setd, wl, warmup=3, serial_steps=10):
    """Batching form: 64 independent 2D Schnakenberg instances of uneven size
    (sides from {64, ..., 512}, d_v ~ U(8, 12)), FP64, tau = 1e-3, 100 steps.
    Timed with graph replay (no kernel events), then once more with kernel
    events for the per-class rates, then the same instances stepped one
    context at a time for comparison."""
    probs = wl.schnakenberg_batch()
    nsteps = probs[0].nsteps
    dev = torch.device("cuda:0")
    A = [[[torch.from_numpy(M.ravel(order="F").copy()).to(dev) for M in Ac] for Ac in p.A] for p in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B = setd.Batch([p.dims for p in probs], A, probs[0].tau)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    info = B.tune()
    tune_s = time.perf_counter() - t0
    u0 = torch.zeros(B.total, dtype=torch.float64, device=dev)
    for b, p in enumerate(probs):
        for c in range(2):
            B.field(u0, b, c).copy_(torch.from_numpy(p.U0[c].ravel(order="F").copy()))
    params = [p.params for p in probs]
    u = u0.clone()
    B.step(u, warmup, probs[0].g_kind, params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.step(u, nsteps, probs[0].g_kind, params)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = bool(torch.isfinite(u).all())
    # per-class rates (direct launches with events)
    setd.profile_enable(True)
    setd.profile_read(reset=True)
    B.step(u, 5, probs[0].g_kind, params)
    torch.cuda.synchronize()
    prof = setd.profile_read(reset=True)
    setd.profile_enable(False)
    info = B.info()
    B.close()
    flops = sum(mode_flops_per_step(p.dims, 2) for p in probs)
    mode_ms = sum(prof[k]["ms"] for k in F64_MODE_CLASSES) / 5
    # the same instances one context at a time (graph replay per context)
    ctxs = [setd.Context(p.dims, A[b], p.tau) for b, p in enumerate(probs)]
    us = [torch.cat([B.field(u0, b, 0), B.field(u0, b, 1)]).clone() for b in range(len(probs))]
    for b, p in enumerate(probs):
        ctxs[b].step(us[b], 1, p.g_kind, p.params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, p in enumerate(probs):
        ctxs[b].step(us[b], serial_steps, p.g_kind, p.params)
    torch.cuda.synchronize()
    dts = time.perf_counter() - t0
    for c in ctxs:
        c.close()
    res = dict(workload="schnakenberg2d_batch64", instances=len(probs), steps=nsteps, finite=ok,
               steps_per_s=round(nsteps / dt, 3), ms_per_step=round(dt / nsteps * 1e3, 4),
               instance_steps_per_s=round(len(probs) * nsteps / dt, 1),
               tucker_flops_per_step=flops, tucker_tflops=round(flops / (dt / nsteps) / 1e12, 3),
               mode_kernel_tflops=round(flops / (mode_ms * 1e-3) / 1e12, 3) if mode_ms > 0 else None,
               launches_per_step=info["launches_per_step"], tiles=dict(mode1=info["mode1"], modeB=info["modeB"]),
               packed_sets=info["packed_sets"], setup_s=round(setup, 3), tune_s=round(tune_s, 3),
               one_context_at_a_time_steps_per_s=round(serial_steps / dts, 3),
               speedup_vs_one_context_at_a_time=round((nsteps / dt) / (serial_steps / dts), 2))
    log("batch: %.1f steps/s (%d instances), %.2f x one context at a time" %
        (res["steps_per_s"], len(probs), res["speedup_vs_one_context_at_a_time"]))
    return res


def run_methods(torch, setd, prob, A, u0, f64_step_s, steps=20):
    """The other two integrators on the same workload and context type:
    exprk3ds_cplx (two complex Tuckers per split action) and etd2rkds (one
    Tucker per phi action, second order)."""
    out = {}
    for name in ("exprk3ds_cplx", "etd2rkds"):
        ctx = setd.Context(prob.dims, A, prob.tau)
        u = u0.clone()
        fn = ctx.step_cplx if name == "exprk3ds_cplx" else ctx.step2
        fn(u, 2, prob.g_kind, prob.params)          # set-up and warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(u, steps, prob.g_kind, prob.params)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.close()
        out[name] = dict(steps_per_s=round(steps / dt, 3), ms_per_step=round(dt / steps * 1e3, 4),
                         time_vs_exprk3ds_real=round((dt / steps) / f64_step_s, 3), steps=steps)
        log("%s: %.2f steps/s" % (name, steps / dt))
    return out


def run_adjoint(torch, setd, wl, nsteps=200, checkpoint=20):
    """Differentiation form: L = 1/2 ||u(T) - u_target||^2 on 3D FHN 128^3 after
    200 steps (u_target from eps = 0.55, a1 = 2.1), gradients with respect to
    u0, (eps, a1, a0) and d_v through the checkpointed adjoint (one
    checkpoint every 20 steps)."""
    from paper_2310_07551_amd import autograd as sad
    p = wl.make("fhn3d_128")
    dev = torch.device("cuda:0")
    D = [[torch.from_numpy(wl.neumann_d2(m).ravel(order="F").copy()).to(dev) for m in p.dims] for _ in range(2)]
    dv = float(p.A[1][0][1, 1] / wl.neumann_d2(p.dims[0])[1, 1])
    u0 = torch.from_numpy(p.u0_flat()).to(dev)
    kw = dict(dims=p.dims, D=D, g_kind=p.g_kind, tau=p.tau, nsteps=nsteps, checkpoint=checkpoint,
              diff_components=(1,))   # d_v only, as the workload asks
    with torch.no_grad():
        target = sad.integrate(u0, torch.tensor([0.55, 2.1, 0.0], dtype=torch.float64),
                               torch.tensor([1.0, dv], dtype=torch.float64), **kw).clone()
    times = []
    for rep in range(2):                      # the first run includes the set-up of both banks
        params = torch.tensor(list(p.params[:3]), dtype=torch.float64, requires_grad=True)
        diff = torch.tensor([1.0, dv], dtype=torch.float64, requires_grad=True)
        ui = u0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uT = sad.integrate(ui, params, diff, **kw)
        loss = 0.5 * ((uT - target) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        times.append((t1 - t0, time.perf_counter() - t1))
    fwd, bwd = times[-1]
    log("adjoint: forward %.3f s, backward %.3f s" % (fwd, bwd))
    return dict(workload="fhn3d_128", steps=nsteps, checkpoint=checkpoint, loss=loss.item(),
                forward_s=round(fwd, 4), backward_s=round(bwd, 4), backward_over_forward=round(bwd / fwd, 3),
                grad_eps=params.grad[0].item(), grad_a1=params.grad[1].item(), grad_dv=diff.grad[1].item())


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fhn3d_256")
    ap.add_argument("--cpu-sample-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="MB",
                    help="only run a plain device copy of this size (HBM counter calibration) and exit")
    ap.add_argument("--forms", default="f64,i8x4,f32,bf16x3,bf16x2,batch,methods,adjoint",
                    help="forms to time besides the FP64 metric: i8x4, f32, bf16x3, bf16x2 (compared against f64), "
                         "batch (64 uneven 2D Schnakenberg instances, 100 steps), methods (exprk3ds_cplx and "
                         "etd2rkds on the same workload) and adjoint (gradient of the 3D FHN 128^3, 200-step loss)")
    ap.add_argument("--library-gemm", action="store_true",
                    help="only time the vendor library's FP64 GEMM at the 256^3 mode-product shapes and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the split-ETD3 path here runs on a single MI355X "
              "(no multi-GPU path is built); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    if args.library_gemm:
        library_gemm()
        return

    import torch
    import paper_2310_07551_amd as setd
    import workloads as wl

    prob = wl.make(args.workload)
    log("workload %s dims %s tau %g" % (prob.name, prob.dims, prob.tau))
    dev = torch.device("cuda:0")
    A = [[torch.from_numpy(M.ravel(order="F").copy()).to(dev) for M in Ac] for Ac in prob.A]
    u0 = torch.from_numpy(prob.u0_flat()).to(dev)

    def run_form(prec, steps, warmup):
        """phi bank, W warm-up steps, K timed steps (graph replay, no events),
        then K more steps with per-launch events.  Returns the open context,
        phi seconds, timed seconds, profiled seconds, per-class profile and
        the state after the timed steps."""
        u = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = setd.Context(prob.dims, A, prob.tau, prec=prec)
        torch.cuda.synchronize()
        phi = time.perf_counter() - t0
        ctx.step(u, warmup, prob.g_kind, prob.params)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(u, steps, prob.g_kind, prob.params)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        u_timed = u.clone()
        setd.profile_enable(True)
        setd.profile_read(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(u, steps, prob.g_kind, prob.params)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0
        prof = setd.profile_read(reset=True)
        setd.profile_enable(False)
        return ctx, phi, dt, dtp, prof, u_timed

    # stored oracle values of this workload (3D FitzHugh-Nagumo grids)
    goldens = {}
    if prob.name == "fhn3d" and len(set(prob.dims)) == 1:
        for k in range(1, prob.nsteps + 1):
            g = read_golden(prob.dims[0], k)
            if g is not None:
                goldens[k] = g

    def accuracy(ctx, ref_states=None):
        """A clean trajectory from u0 to each stored step count: errors against
        the oracle's stored values and, when given, the FP64 states."""
        u = u0.clone()
        done, res, states = 0, {}, {}
        for k in sorted(goldens):
            ctx.step(u, k - done, prob.g_kind, prob.params)
            torch.cuda.synchronize()
            done = k
            res[k] = golden_errors(u, prob.N, goldens[k])
            states[k] = u.clone()
            if ref_states is not None:
                for c, name in enumerate(("u", "v")):
                    e = setd.field_norms(u[c * prob.N:(c + 1) * prob.N], ref_states[k][c * prob.N:(c + 1) * prob.N])
                    res[k][name]["rel_l2_vs_f64"] = e[2] / e[0]
        return res, states

    def form_roofline(prof_l, name):
        """Dominant reduced-precision mode class against the peak of its own
        arithmetic (matrix-core flops = algorithmic flops x products per
        product) or HBM, whichever bounds it."""
        cls = max(("mode1_lp", "modeB_lp"), key=lambda k: prof_l[k]["ms"])
        v = prof_l[cls]
        if v["ms"] <= 0:
            return None
        sec = v["ms"] * 1e-3
        mfma = v["flops"] * MFMA_PER_PRODUCT[name]
        t_compute = mfma / (PEAK_TFLOPS[name] * 1e12)
        t_memory = v["bytes"] / (PEAK_HBM_GBS * 1e9)
        if t_compute >= t_memory:
            ach = mfma / sec / 1e12
            r = dict(bound="mfma", achieved=round(ach, 3), peak=PEAK_TFLOPS[name], unit="TFLOP/s",
                     frac=round(ach / PEAK_TFLOPS[name], 4))
        else:
            ach = v["bytes"] / sec / 1e9
            r = dict(bound="hbm", achieved=round(ach, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                     frac=round(ach / PEAK_HBM_GBS, 4))
        r.update(kernel=cls, launches=v["launches"], avg_launch_ms=round(v["ms"] / max(1, v["launches"]), 4),
                 algorithmic_tflops=round(v["flops"] / sec / 1e12, 3), algorithmic_gbs=round(v["bytes"] / sec / 1e9, 1),
                 traffic=None)
        return r

    ctx, phi_s, dt, dtp, prof, u = run_form(setd.PREC_F64, args.steps, args.warmup)
    log("phi bank %.3f s, %d steps in %.3f s (graph replay), %.3f s with per-launch events" %
        (phi_s, args.steps, dt, dtp))
    norms = setd.field_norms(u[:prob.N])
    if not all(map(lambda x: x == x and abs(x) != float("inf"), norms)):
        log("non-finite state after the timed steps")
        sys.exit(1)
    acc64, states64 = accuracy(ctx) if goldens else ({}, {})
    ctx.close()
    for k, e in acc64.items():
        log("f64 vs stored oracle at step %d: %s" % (k, {f: "%.2e" % v["samples_rel_l2"] for f, v in e.items()}))

    forms = {}
    for name in [f for f in args.forms.split(",") if f in ("i8x4", "f32", "bf16x3", "bf16x2")]:
        prec = {"f32": setd.PREC_F32, "bf16x3": setd.PREC_BF16X3, "bf16x2": setd.PREC_BF16X2,
                "i8x4": setd.PREC_I8X4}[name]
        ctx_l, phi_l, dt_l, dtp_l, prof_l, u_l = run_form(prec, args.steps, args.warmup)
        acc_l, _ = accuracy(ctx_l, states64) if goldens else ({}, {})
        ctx_l.close()
        ms = sum(prof_l[k]["ms"] for k in ("mode1_lp", "modeB_lp"))
        fl = sum(prof_l[k]["flops"] for k in ("mode1_lp", "modeB_lp"))
        last = max(acc_l) if acc_l else None
        worst = max(v["rel_l2_vs_f64"] for v in acc_l[last].values()) if last else None
        forms[name] = dict(steps_per_s=round(args.steps / dt_l, 4), ms_per_step=round(dt_l / args.steps * 1e3, 4),
                           speedup_vs_f64=round(dt / dt_l, 3),
                           accuracy=acc_l, accuracy_step=last, worst_rel_l2_vs_f64=worst,
                           meets_1e_5=(worst is not None and worst <= 1e-5),
                           tucker_tflops=round(fl / (ms * 1e-3) / 1e12, 3) if ms > 0 else None,
                           roofline=form_roofline(prof_l, name), phi_setup_s=round(phi_l, 3))
        log("%s: %.2f steps/s, worst rel_l2 vs f64 at step %s: %s" % (name, args.steps / dt_l, last, worst))

    batch = run_batch(torch, setd, wl) if "batch" in args.forms.split(",") else None
    methods = run_methods(torch, setd, prob, A, u0, dt / args.steps) if "methods" in args.forms.split(",") else None
    adjoint = run_adjoint(torch, setd, wl) if "adjoint" in args.forms.split(",") else None

    steps_per_s = args.steps / dt
    nterms = 2 if prob.d == 2 else 3
    flops_step = mode_flops_per_step(prob.dims, nterms)
    mode_ms = sum(prof[k]["ms"] for k in F64_MODE_CLASSES)
    mode_flops = sum(prof[k]["flops"] for k in F64_MODE_CLASSES)
    tucker_tflops = mode_flops / (mode_ms * 1e-3) / 1e12 if mode_ms > 0 else 0.0
    dom = max(prof, key=lambda k: prof[k]["ms"])
    dp = prof[dom]
    if dp["flops"] > 0:
        achieved = dp["flops"] / (dp["ms"] * 1e-3) / 1e12
        roof = dict(bound="mfma", achieved=round(achieved, 3), peak=PEAK_TFLOPS["f64"], unit="TFLOP/s",
                    frac=round(achieved / PEAK_TFLOPS["f64"], 4), traffic=None)
    else:
        achieved = dp["bytes"] / (dp["ms"] * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(achieved / PEAK_HBM_GBS, 4), traffic=None)
    tb = counted_traffic(dom, args.workload)
    roof["traffic"] = None if tb is None else round(tb, 0)
    roof["kernel"] = dom
    roof["launches"] = dp["launches"]
    roof["avg_launch_ms"] = round(dp["ms"] / max(1, dp["launches"]), 4)

    kernels = {k: dict(launches=v["launches"], ms_per_step=round(v["ms"] / args.steps, 4),
                       tflops=round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 3) if v["ms"] > 0 and v["flops"] else None,
                       gbs=round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None)
               for k, v in prof.items() if v["launches"]}

    out = {
        "metric": METRIC,
        "value": round(steps_per_s, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": list(prob.dims), "tau": prob.tau, "components": 2,
                   "kinetics": prob.name, "phi_setup_s": round(phi_s, 3)},
        "timing": "graph replay, no per-launch events; kernels and roofline from a second pass of the same "
                  "steps with per-launch events",
        "profiled_ms_per_step": round(dtp / args.steps * 1e3, 4),
        "f64_vs_oracle": acc64,
        "tucker_tflops": round(tucker_tflops, 3),
        "tucker_frac_peak": round(tucker_tflops / PEAK_TFLOPS["f64"], 4),
        "tucker_flops_per_step": flops_step,
        "kernels": kernels,
        "precision_forms": forms,
        "batch_form": batch,
        "method_forms": methods,
        "adjoint_form": adjoint,
        "roofline": roof,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle (%d step(s))" % args.cpu_sample_steps)
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_sample_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
