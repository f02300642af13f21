"""Benchmark: throughput of the matrix-free operator J v on one MI355X.

Workload (default): the 3D mixing layer on a 256 x 128 x 128 grid (x and z
periodic, walls in y), 5 variables, tanh(y) base flow with seeded 1e-3 N(0,1)
spanwise velocity, M = 0.5, Re = 1000, FP64.  One step is one application of
y = (J - sigma I) x over the whole grid (sa_op_apply, sigma = 0.2), inputs
resident in HBM.  value = grid-point updates per second (all five outputs of
one point = one update).

Also reported: the roofline record of the operator kernel (algorithmic bytes
= read x + read q0 + write y = 3 nv 8 B per point, against 8 TB/s), the same
operator in FP32, the time to the 6 leading eigenpairs of the same workload
in the FP64 and the mixed form (Cayley-IRAM with mean-flow-preconditioned
inner solves; --no-eigs skips it), optional extras (--extras: GMRES(40) at 2D 512 x 512, the
block-Jacobi preconditioner of the 3D grid with 8 shifts, 8-shift batched
GMRES cycles, time to eigenpairs FP64 vs mixed on a small case, a reduced
sweep of uneven base flows run in turn and concurrently), and the oracle
timed on the host cores on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--extras]
       [--no-cpu] [--calib-copy]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpt-updates/s of matrix-free Jv; time to 6 eigenpairs, mixed vs FP64 GPU"
HBM_PEAK_GBS = 8000.0


# committed rocprofv3 FETCH_SIZE / WRITE_SIZE summaries: (file, kernel sources
# hashed at measurement, the key of that hash in the file)
COUNTERS = {
    "iso": (os.path.join(ROOT, "profiles", "jv_iso_fp64_256x128x128_hbm_counters.md"),
            ["paper_1502_03701_amd/csrc/jv_iso.hip", "paper_1502_03701_amd/csrc/jv_common.h",
             "paper_1502_03701_amd/csrc/sa_internal.h"],
            "kernel_source_sha256 (jv_iso.hip, jv_common.h, sa_internal.h at measurement)"),
    "general": (os.path.join(ROOT, "profiles", "jv_prefetch_fp64_256x128x128_hbm_counters.md"),
                ["paper_1502_03701_amd/csrc/jv_prefetch.hip", "paper_1502_03701_amd/csrc/jv_stage.hip",
                 "paper_1502_03701_amd/csrc/jv_common.h", "paper_1502_03701_amd/csrc/jv.hip"],
                "kernel_source_sha256 (jv_prefetch.hip, jv_stage.hip, jv_common.h, jv.hip at measurement)"),
}


def measured_traffic(variant):
    """HBM bytes per launch of the FP64 operator kernel variant the autotuner
    kept, from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary
    (calibrated against a copy of known size), or None if that variant was
    not measured or the kernel source changed since."""
    import hashlib
    path, sources, key = COUNTERS["iso" if variant.startswith("iso") else "general"]
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    name = "traffic_bytes_per_launch[%s]" % variant
    if fields.get(key) != h.hexdigest() or name not in fields:
        return None
    return int(fields[name])


def kernel_name(variant, real="double"):
    """The HIP kernel behind an operator variant name (e.g. 'iso_z32')."""
    kind = variant.split("_z")[0]
    return {"prefetch": "jv_prefetch_kernel", "stage": "jv_stage_kernel",
            "iso": "jv_iso_kernel"}.get(kind, "jv_prefetch_kernel") + "<%s,3>" % real


def hbm_probe(torch, dev):
    """Achievable HBM bandwidth of plain torch kernels on 4 GiB FP64 tensors
    (context for the Krylov kernels' GB/s): a read-only sum, a two-read
    one-write add, a copy."""
    n = 512 * 1024 * 1024
    a = torch.randn(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    c = torch.empty(n // 4, dtype=torch.float64, device=dev)
    out = {}
    for name, fn, nbytes in (("sum_read", lambda: torch.sum(a), 8 * n),
                             ("add_2r1w", lambda: torch.add(a[: n // 4], a[n // 4: n // 2], out=c), 3 * 8 * (n // 4)),
                             ("copy_1r1w", lambda: b.copy_(a), 2 * 8 * n)):
        sec = timed(fn, 10, 2, torch) / 10
        out[name] = {"ms": sec * 1e3, "TBs": nbytes / sec / 1e12}
    del a, b, c
    return out


def calib_copy(torch, dev):
    """A device copy of known size, 16x the 256 MB last-level cache: reads and
    writes 4 GiB each (the reference for the rocprofv3 byte counters)."""
    ca = torch.ones(512 * 1024 * 1024, dtype=torch.float64, device=dev)
    cb = torch.empty_like(ca)
    timed(lambda: cb.copy_(ca), 2, 0, torch)
    del ca, cb


def timed(fn, steps, warmup, torch):
    """Seconds for `steps` calls, HIP events on the current stream (the
    stream the library launches on)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3


def cpu_baseline(prob, q0, v):
    """Oracle complex-step Jv on a bounded window of the workload (a 16-wide
    slab in x and z over the full y range), repeated for about 10 s, scaled
    to Gpt/s."""
    import synth
    from oracle import operator as op
    W = 16
    nx, ny, nz = prob.n
    sub = synth.mixing_layer_3d(W, ny, W, prob.mach, prob.re, lx=W * prob.length[0] / nx,
                                ly=prob.length[1], lz=W * prob.length[2] / nz)
    import numpy as np
    qs = np.ascontiguousarray(q0[:, :W, :, :W])
    vs = np.ascontiguousarray(v[:, :W, :, :W])
    op.jv_cstep(sub, qs, vs)            # warm-up
    reps = 0
    t0 = time.perf_counter()
    while True:
        op.jv_cstep(sub, qs, vs)
        reps += 1
        el = time.perf_counter() - t0
        if el > 10.0 or reps >= 2000:
            break
    rate = reps * sub.npts / el / 1e9
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"value": rate, "unit": "Gpt/s", "cores": 1, "kind": "oracle",
            "sample": "complex-step Jv (NumPy, elementwise work on one thread) on a %dx%dx%d "
                      "window of the workload, %d repetitions in %.1f s; the host has %d cores"
                      % (W, ny, W, reps, el, cores)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-eigs", action="store_true", help="skip the eigen-time record")
    ap.add_argument("--eigs-only", action="store_true", help="only the eigen-time record (3D workload)")
    ap.add_argument("--sweep", action="store_true", help="only the 48-flow sweep (128^2 - 768^2)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a device copy of known size (counter calibration)")
    ap.add_argument("--bjac-only", action="store_true",
                    help="only the block-Jacobi setup and apply of the 3D grid (for profiling)")
    ap.add_argument("--c0-eigs", action="store_true",
                    help="only the time to the four separated eigenpairs of the 48x48 case: FP64 / mixed, "
                         "GMRES / LGMRES inner solves")
    ap.add_argument("--iram-only", action="store_true",
                    help="only the 3D 32^3 eigen solve (2 eigenpairs, LGMRES(37, 3) inner solves, FP64 and "
                         "mixed; for profiling the Arnoldi, Cayley and Ritz kernels)")
    ap.add_argument("--eigs-64", action="store_true",
                    help="only the 3D 64^3 eigen solve (2 eigenpairs, LGMRES(37, 3) inner solves, FP64 and mixed)")
    ap.add_argument("--sweep-modes", default="sequential,concurrent",
                    help="modes of --sweep, comma-separated: sequential (in turn), concurrent (16 at a time)")
    ap.add_argument("--sweep-mid", action="store_true",
                    help="only the sweep of 8 uneven flows on sides 64-128 (LGMRES(37, 3), concurrent)")
    ap.add_argument("--c2-solve", action="store_true",
                    help="only one Cayley system of the 3D grid to 1e-10: FP64 against the mixed form, "
                         "GMRES(30) and LGMRES(30, 3)")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="only the achievable HBM bandwidth of plain torch sum / add / copy on 4 GiB")
    ap.add_argument("--c2-cap", type=int, default=30000,
                    help="product budget of each --c2-solve solve (a small cap for profiling)")
    ap.add_argument("--discretisations", action="store_true",
                    help="only the operator on 256x128x128 with explicit / compact first derivatives on "
                         "uniform / stretched rows, FP64 and FP32")
    ap.add_argument("--bjac-gmres", action="store_true",
                    help="FP32 GMRES(30) of the 8 shifts on the 3D grid, 300 products, with and without block-Jacobi")
    ap.add_argument("--gmres-only", action="store_true",
                    help="only capped GMRES runs: 512x512 FP64 (1 and 8 shifts), one FP32 cycle of "
                         "8 shifts on the 3D grid (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is documented, not built).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1502_03701_amd import Context

    dev = torch.device("cuda:0")
    if args.discretisations:
        print(json.dumps(discretisations(torch, dev, args.steps, args.warmup)))
        return
    if args.hbm_probe:
        print(json.dumps(hbm_probe(torch, dev)))
        return
    if args.c0_eigs:
        print(json.dumps(eigs_c0(torch, dev, log=lambda m: print(m, file=sys.stderr, flush=True))))
        return
    if args.sweep_mid:
        print(json.dumps(sweep(torch, dev, augment=3, modes=("concurrent",), sides=(64, 96, 128), tag="mid",
                               max_matvec=30000, log=lambda m: print(m, file=sys.stderr, flush=True))))
        return
    if args.sweep:
        modes = tuple(m for m in args.sweep_modes.split(",") if m)
        if not modes or any(m not in ("sequential", "concurrent") for m in modes):
            sys.exit("--sweep-modes: sequential and/or concurrent")
        print(json.dumps(sweep_c4(torch, dev, modes=modes, log=lambda m: print(m, file=sys.stderr, flush=True))))
        return
    if args.eigs_only:
        print(json.dumps(eigs_c2(torch, dev, log=lambda m: print(m, file=sys.stderr, flush=True))))
        return
    if args.eigs_64:
        print(json.dumps(eigs_3d(torch, dev, side=64, max_restarts=20, augment=3,
                                 log=lambda m: print(m, file=sys.stderr, flush=True))))
        return
    if args.iram_only:
        print(json.dumps(eigs_3d(torch, dev, augment=3, log=lambda m: print(m, file=sys.stderr, flush=True))))
        return
    prob = synth.config2()
    q0 = synth.base_flow(prob, seed=2, w_noise=1e-3)
    v = synth.random_vector(prob, 2)
    ctx = Context()
    ctx.base_set(prob, torch.from_numpy(q0.ravel()).to(dev))
    if args.gmres_only:
        print(json.dumps(gmres_runs(torch, dev, ctx, prob)))
        return
    if args.c2_solve:
        log = lambda m: print(m, file=sys.stderr, flush=True)   # noqa: E731
        out = c2_solve(torch, dev, ctx, prob, max_matvec=args.c2_cap, log=log)
        out.update(c2_solve(torch, dev, ctx, prob, augment=3, max_matvec=args.c2_cap, log=log))
        print(json.dumps(out))
        return
    if args.bjac_gmres:
        out = bjac(torch, dev, ctx, prob)
        out.update(bjac_gmres(torch, dev, ctx, prob))
        print(json.dumps(out))
        return
    if args.bjac_only:
        out = bjac(torch, dev, ctx, prob)
        if args.calib_copy:
            calib_copy(torch, dev)
        print(json.dumps(out))
        return
    x = torch.from_numpy(v.ravel()).to(dev)
    y = torch.empty_like(x)
    npts = prob.npts
    nv = prob.nv

    sec = timed(lambda: ctx.op_apply(x, y, shift=0.2), args.steps, args.warmup, torch)
    per = sec / args.steps
    value = npts / per / 1e9
    alg_bytes = 3 * nv * 8 * npts
    achieved = alg_bytes / per / 1e9

    from paper_1502_03701_amd import SA_F32, SA_F64
    from paper_1502_03701_amd._native import JV_VARIANTS
    tuned = {}
    for name, prec in (("f64", SA_F64), ("f32", SA_F32)):
        var, times = ctx.jv_variant(prec)
        tuned[name] = {"variant": JV_VARIANTS[var] if var >= 0 else "default", "tune_us": times}

    traffic = measured_traffic(tuned["f64"]["variant"])

    x32 = x.float()
    y32 = torch.empty_like(x32)
    sec32 = timed(lambda: ctx.op_apply(x32, y32, shift=0.2), args.steps, args.warmup, torch)
    per32 = sec32 / args.steps

    if args.calib_copy:
        calib_copy(torch, dev)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Gpt/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D mixing layer 256x128x128 (x,z periodic, y walls), 5 vars, "
                               "tanh + 1e-3 N(0,1) spanwise base, M=0.5 Re=1000; "
                               "one FP64 sa_op_apply per step",
                   "grid": [256, 128, 128], "nv": nv, "shift": 0.2},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": kernel_name(tuned["f64"]["variant"]), "alg_bytes_per_point": 3 * nv * 8,
                     "frac_basis": "achieved and frac: algorithmic bytes (x, q0 in; y out) per launch over the "
                                   "HIP-event time; traffic_GBs and traffic_frac: the measured HBM bytes "
                                   "(rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated) over the same time",
                     "traffic_GBs": traffic / per / 1e9 if traffic else None,
                     "traffic_frac": traffic / per / 1e9 / HBM_PEAK_GBS if traffic else None},
        "fp32_jv": {"gpts": npts / per32 / 1e9, "ms": per32 * 1e3,
                    "achieved_GBs": 3 * nv * 4 * npts / per32 / 1e9},
        "autotuned_jv": tuned,
    }
    if not args.no_eigs:
        out["eigs"] = eigs_c2(torch, dev, log=lambda m: print(m, file=sys.stderr, flush=True))
    if args.extras:
        out["extras"] = extras(torch, dev, ctx, prob)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, q0, v)
    print(json.dumps(out))


def bjac(torch, dev, ctx3, prob3):
    """Block-Jacobi of the 3D grid: 4x4x1-cell blocks x 5 vars = 80x80,
    262144 blocks, 8 shifts 0.05..0.40, FP32 factors; setup wall time and
    apply time per shift (HIP events)."""
    import synth
    shifts = synth.config3_shifts()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx3.precond_setup(shifts, 4, 4, 1, diag_add=0.1, noise_std=0.01, seed=3)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    r32 = torch.from_numpy(synth.random_vector(prob3, 3).ravel()).to(dev).float()
    z32 = torch.empty_like(r32)
    t_apply = timed(lambda: ctx3.precond_apply(0, r32, z32), 10, 2, torch) / 10
    nblocks = prob3.npts // 16
    return {"bjac_256x128x128_8shifts": {
        "setup_s": t_setup, "nblocks": nblocks, "nb": 80, "apply_ms_per_shift": t_apply * 1e3,
        "apply_factor_GBs": nblocks * 80 * 80 * 4 / t_apply / 1e9}}


def gmres_runs(torch, dev, ctx3, prob3, max_mv_512=2000):
    """GMRES step costs: one FP32 GMRES(30) cycle of the 8 shifts in lockstep on
    the 3D grid (with the block-Jacobi factors if they are set up), GMRES(40)
    at 512 x 512 FP64 for one shift and for 8 shifts in lockstep (capped)."""
    import synth
    from paper_1502_03701_amd import SA_F32, Context
    res = {}
    shifts = synth.config3_shifts()

    def wall(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    B = torch.from_numpy(synth.random_vector(prob3, 4, nrhs=8).ravel()).to(dev).float()
    for use_pc in ((False, True) if ctx3.has_precond() else (False,)):
        X = torch.zeros_like(B)
        (rc, info), el = wall(lambda: ctx3.gmres_solve(shifts, B, X, restart=30, tol=1e-6, max_matvec=31,
                                                      use_precond=use_pc, prec=SA_F32))
        res["gmres30_fp32_8shifts_" + ("bjac" if use_pc else "plain")] = {
            "seconds_one_cycle": el, "relres": [i["relres"] for i in info], "iters": [i["iters"] for i in info]}
    del B, X
    p1 = synth.config1()
    c1 = Context()
    c1.base_set(p1, torch.from_numpy(synth.base_flow(p1).ravel()).to(dev))
    b = torch.from_numpy(synth.random_vector(p1, 1).ravel()).to(dev)
    x = torch.zeros_like(b)
    (rc, info), el = wall(lambda: c1.gmres_solve([0.2], b, x, restart=40, tol=1e-10, max_matvec=max_mv_512))
    res["gmres40_512x512"] = {"iters": info[0]["iters"], "relres": info[0]["relres"],
                              "ms_per_iter": el / max(1, info[0]["iters"]) * 1e3}
    B8 = torch.from_numpy(synth.random_vector(p1, 5, nrhs=8).ravel()).to(dev)
    X8 = torch.zeros_like(B8)
    (rc, info), el = wall(lambda: c1.gmres_solve(shifts, B8, X8, restart=40, tol=1e-10, max_matvec=401))
    res["gmres40_512x512_8shifts"] = {"ms_per_iter_all_shifts": el / max(1, info[0]["iters"]) * 1e3,
                                      "iters": info[0]["iters"]}
    c1.close()
    return res


def bjac_gmres(torch, dev, ctx3, prob3, max_matvec=300):
    """What the block-Jacobi preconditioner (set up on ctx3: 4x4x1-cell
    blocks, +0.1 I, 1e-2 noise, FP32 factors) does for the solves it is built
    for: FP32 GMRES(30) of the 8 shifts in lockstep on the 3D grid, seeded
    N(0,1) right-hand sides, the same product budget with and without it;
    the relative residual each shift reaches and the wall time."""
    import synth
    from paper_1502_03701_amd import SA_F32
    shifts = synth.config3_shifts()
    B = torch.from_numpy(synth.random_vector(prob3, 4, nrhs=8).ravel()).to(dev).float()
    res = {}
    for use_pc in (False, True):
        X = torch.zeros_like(B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, info = ctx3.gmres_solve(shifts, B, X, restart=30, tol=1e-6, max_matvec=max_matvec,
                                    use_precond=use_pc, prec=SA_F32)
        torch.cuda.synchronize()
        res["bjac_gmres30_fp32_8shifts_%d_%s" % (max_matvec, "bjac" if use_pc else "plain")] = {
            "seconds": time.perf_counter() - t0, "shifts": list(shifts),
            "relres": [i["relres"] for i in info], "matvecs": [i["matvecs"] for i in info]}
    return res


def c2_solve(torch, dev, ctx3, prob3, sigma=0.2, restart=30, augment=0, max_matvec=30000, log=None):
    """One Cayley system (J - sigma I) x = b of the full 3D grid, b seeded
    N(0,1), to 1e-10 relative residual: all-FP64 GMRES(restart) against
    FP32 GMRES(restart) inner solves (relative tolerance 1e-4) inside FP64
    refinement, both capped at max_matvec products; augment = k > 0 makes
    both LGMRES(restart, k).  The true FP64 residual of each
    solution is recomputed with one FP64 operator product."""
    import synth
    from paper_1502_03701_amd import SA_F64, SA_MIXED
    res = {}
    key = "c2_solve_%s%d%s_" % ("lgmres" if augment else "gmres", restart, "_%d" % augment if augment else "")
    b = torch.from_numpy(synth.random_vector(prob3, 6, stream=1).ravel()).to(dev)
    bn = float(torch.linalg.vector_norm(b))
    y = torch.empty_like(b)
    for name, prec in (("fp64", SA_F64), ("mixed", SA_MIXED)):
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, info = ctx3.gmres_solve([sigma], b, x, restart=restart, tol=1e-10, max_matvec=max_matvec, prec=prec,
                                    inner_tol=1e-4, max_outer=20, augment=augment)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx3.op_apply(x, y, shift=sigma)
        true_rel = float(torch.linalg.vector_norm(b - y)) / bn
        i = info[0]
        res[key + name] = {"seconds": el, "matvecs": i["matvecs"], "iters": i["iters"], "outer": i["outer"], "relres": i["relres"], "true_relres": true_rel,
                           "status": i["status"], "ms_per_matvec": el / max(1, i["matvecs"]) * 1e3}
        if log:
            log(key + "%s: %.2f s, %d products, relres %.2e (true %.2e)"
                % (name, el, i["matvecs"], i["relres"], true_rel))
    f, m = res[key + "fp64"], res[key + "mixed"]
    res[key + "mixed_vs_fp64"] = {"speedup": f["seconds"] / m["seconds"],
                                  "per_matvec_speedup": f["ms_per_matvec"] / m["ms_per_matvec"]}
    return res


def extras(torch, dev, ctx3, prob3):
    """Secondary measurements (not the headline value)."""
    import synth
    from paper_1502_03701_amd import SA_F32, SA_MIXED, Context, arnoldi_eigs
    res = {}

    def wall(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    res.update(bjac(torch, dev, ctx3, prob3))
    res.update(gmres_runs(torch, dev, ctx3, prob3))
    res.update(c2_solve(torch, dev, ctx3, prob3, log=lambda m: print(m, file=sys.stderr, flush=True)))
    # time to eigenpairs, FP64 vs mixed, small case (KH pair)
    pe = synth.mixing_layer_2d(32, 32, 0.5, 1000.0)
    ce = Context()
    ce.base_set(pe, torch.from_numpy(synth.base_flow(pe).ravel()).to(dev))
    v0 = torch.from_numpy(synth.random_vector(pe, 0).ravel()).to(dev)
    for name, prec in (("fp64", 0), ("mixed", SA_MIXED)):
        (rc, r), el = wall(lambda: arnoldi_eigs([ce], [v0], nev=2, ncv=16, tol=1e-10, restart=40, lin_tol=1e-12,
                                                prec=prec, inner_tol=1e-4, max_outer=20))
        res["eigs_kh_32x32_" + name] = {"seconds": el, "nconv": r[0]["nconv"],
                                        "lam": [[l.real, l.imag] for l in r[0]["lam"]],
                                        "n_matvec": r[0]["n_matvec"]}
    log = lambda m: print(m, file=sys.stderr, flush=True)   # noqa: E731
    res.update(sweep(torch, dev, log=log))
    res.update(sweep(torch, dev, augment=3, modes=("concurrent",), log=log))
    res.update(sweep(torch, dev, augment=3, modes=("concurrent",), sides=(64, 96, 128), tag="mid",
                     max_matvec=30000, log=log))
    res.update(eigs_3d(torch, dev, log=log))
    res.update(eigs_3d(torch, dev, augment=3, log=log))
    res.update(eigs_3d(torch, dev, nev=4, ncv=20, max_restarts=40, augment=3, log=log))
    res.update(eigs_3d(torch, dev, side=64, max_restarts=20, augment=3, log=log))
    return res


def discretisations(torch, dev, steps, warmup):
    """The operator y = (J - 0.2 I) x on the 256 x 128 x 128 workload grid
    (tanh + 1e-3 spanwise noise, M 0.5, Re 1000) with explicit or compact
    first derivatives, on uniform rows or rows stretched with beta = 3:
    ms per product and Gpt/s in FP64 and FP32 (HIP events, steps products
    after warmup)."""
    import synth
    from paper_1502_03701_amd import SA_F32, SA_F64, Context
    out = {}
    for scheme, sname in ((synth.SCHEME_EXPLICIT, "explicit"), (synth.SCHEME_COMPACT, "compact")):
        for beta in (0.0, 3.0):
            p = synth.mixing_layer_3d(256, 128, 128, 0.5, 1000.0, scheme=scheme, stretch=beta)
            ctx = Context()
            ctx.base_set(p, torch.from_numpy(synth.base_flow(p, seed=2, w_noise=1e-3).ravel()).to(dev))
            x = torch.from_numpy(synth.random_vector(p, 2).ravel()).to(dev)
            rec = {"variant_f64": ctx.jv_variant(SA_F64)[0], "variant_f32": ctx.jv_variant(SA_F32)[0]}
            for dt, tag in ((torch.float64, "f64"), (torch.float32, "f32")):
                xx = x.to(dt)
                y = torch.empty_like(xx)
                sec = timed(lambda: ctx.op_apply(xx, y, shift=0.2), steps, warmup, torch) / steps
                rec[tag] = {"ms": sec * 1e3, "gpts": p.npts / sec / 1e9}
            ctx.close()
            out["%s_%s" % (sname, "stretched" if beta > 0 else "uniform")] = rec
    return {"discretisations_256x128x128": out}


def eigs_c2(torch, dev, log=None, max_restarts=60, restart=(4, 4)):
    """The metric's second half, time to 6 eigenpairs, mixed against FP64 on
    the GPU, at the full 3D workload (256 x 128 x 128, 5 vars, tanh + 1e-3
    spanwise noise, M = 0.5, Re = 1000; sigma = 0.2, mu = -0.2, Arnoldi
    dimension 30, 6 eigenpairs, tol 1e-10).  Inner Cayley solves: GMRES(4)
    (restart = (FP64, mixed) lengths) right-preconditioned with the mean-flow
    operator M(sigma) (the operator of the base averaged over x and z,
    factored per Fourier mode): with it a solve needs a few Krylov steps, and
    the steps of a captured cycle past convergence are launches that return
    at once, so a short cycle is the faster one for both forms (FP64 12.31 s
    and mixed 9.32 s at GMRES(4), 12.43 s and 9.68 s at GMRES(10), measured
    before the refinement loop ran its inner cycles on its own buffers and
    solves from x0 = 0 skipped their first product).  FP64 form:
    FP64 GMRES, operator and factors, solves to 1e-12.  Mixed form: FP32
    GMRES, operator and factors for solves to 1e-4, inside FP64 refinement to
    1e-12.  The timed region covers the preconditioner setup, the IRAM solve,
    the Ritz vectors and their FP64 true residuals."""
    import synth
    from paper_1502_03701_amd import SA_F32, SA_F64, SA_MIXED, SA_PC_MEAN_FLOW, Context, arnoldi_eigs
    p = synth.config2()
    ctx = Context()
    ctx.base_set(p, torch.from_numpy(synth.base_flow(p, seed=2, w_noise=1e-3).ravel()).to(dev))
    v0 = torch.from_numpy(synth.random_vector(p, 0).ravel()).to(dev)
    nev = 6
    evr = torch.empty(nev * p.ndof, dtype=torch.float64, device=dev)
    evi = torch.empty_like(evr)
    out, lam = {}, {}
    for (name, prec, fprec), m in zip((("fp64", SA_F64, SA_F64), ("mixed", SA_MIXED, SA_F32)), restart):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.precond_setup([0.2], factor_prec=fprec, kind=SA_PC_MEAN_FLOW)
        rc, r = arnoldi_eigs([ctx], [v0], nev=nev, ncv=30, sigma=0.2, mu=-0.2, tol=1e-10,
                             max_restarts=max_restarts, restart=m, lin_tol=1e-12, use_precond=True, prec=prec,
                             inner_tol=1e-4, max_outer=30, evecs=[(evr, evi)])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        r = r[0]
        lam[name] = r["lam"]
        out[name] = {"seconds": el, "rc": rc, "nconv": r["nconv"], "restarts": r["restarts"],
                     "n_cayley": r["n_cayley"], "n_matvec": r["n_matvec"], "n_precond": r["n_precond"],
                     "lam": [[l.real, l.imag] for l in r["lam"]], "resid": r["resid"]}
        if log:
            log("eigs c2 %s: %.2f s, nconv %d, %d Cayley solves, %d products" % (name, el, r["nconv"],
                                                                              r["n_cayley"], r["n_matvec"]))
    key = lambda z: (-z.real, z.imag)   # noqa: E731
    rel = [abs(a - b) / abs(a) for a, b in zip(sorted(lam["fp64"], key=key), sorted(lam["mixed"], key=key))]
    ctx.close()
    return {"workload": "3D mixing layer 256x128x128 (x, z periodic, y walls), 5 vars, tanh + 1e-3 N(0,1) "
                        "spanwise base, M=0.5 Re=1000; sigma=0.2, mu=-0.2, Arnoldi dimension 30, 6 eigenpairs, "
                        "tol 1e-10; GMRES(4) inner solves right-preconditioned with the mean-flow operator",
            "fp64_seconds": out["fp64"]["seconds"], "mixed_seconds": out["mixed"]["seconds"],
            "speedup_mixed_vs_fp64": out["fp64"]["seconds"] / out["mixed"]["seconds"],
            "fp64": out["fp64"], "mixed": out["mixed"], "rel_diff_mixed_vs_fp64": rel}


def eigs_c0(torch, dev, log=None):
    """Time to the four separated leading eigenpairs of the 48 x 48 mixing
    layer (M = 0.3, Re = 500; the KH pair and its harmonic), FP64 and mixed
    inner solves, GMRES(40) and LGMRES(37, 3)."""
    import synth
    from paper_1502_03701_amd import SA_F64, SA_MIXED, Context, arnoldi_eigs
    p = synth.config0()
    ctx = Context()
    ctx.base_set(p, torch.from_numpy(synth.base_flow(p).ravel()).to(dev))
    v0 = torch.from_numpy(synth.random_vector(p, 0).ravel()).to(dev)
    out = {}
    for solver, aug in (("gmres", 0), ("lgmres", 3)):
        for name, prec in (("fp64", SA_F64), ("mixed", SA_MIXED)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, r = arnoldi_eigs([ctx], [v0], nev=4, ncv=20, sigma=0.2, mu=-0.2, tol=1e-10, max_restarts=50,
                                 restart=40 - aug, augment=aug, lin_tol=1e-12, prec=prec, inner_tol=1e-4,
                                 max_outer=30)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            out["eigs_c0_nev4_%s_%s" % (solver, name)] = {
                "seconds": el, "rc": rc, "nconv": r[0]["nconv"], "n_matvec": r[0]["n_matvec"],
                "n_cayley": r[0]["n_cayley"], "lam": [[l.real, l.imag] for l in r[0]["lam"]]}
            if log:
                log("eigs c0 %s %s: %.1f s, %d matvecs" % (solver, name, el, r[0]["n_matvec"]))
    ctx.close()
    return out


def eigs_3d(torch, dev, side=32, nev=2, ncv=16, max_restarts=60, augment=0, log=None):
    """Time to the leading eigenpairs of a 3D mixing layer (side^3, M = 0.5,
    Re = 1000, 1e-3 spanwise noise), FP64 against the mixed form, and the
    mixed eigenvalues' relative deviation from the FP64 ones."""
    import synth
    from paper_1502_03701_amd import SA_F64, SA_MIXED, Context, arnoldi_eigs
    p = synth.mixing_layer_3d(side, side, side, 0.5, 1000.0)
    ctx = Context()
    ctx.base_set(p, torch.from_numpy(synth.base_flow(p, seed=1, w_noise=1e-3).ravel()).to(dev))
    v0 = torch.from_numpy(synth.random_vector(p, 0).ravel()).to(dev)
    # Ritz vectors and their true residuals are part of the timed solve
    evr = torch.empty(nev * p.ndof, dtype=torch.float64, device=dev)
    evi = torch.empty_like(evr)
    out, lam = {}, {}
    for name, prec in (("fp64", SA_F64), ("mixed", SA_MIXED)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, r = arnoldi_eigs([ctx], [v0], nev=nev, ncv=ncv, sigma=0.2, mu=-0.2, tol=1e-10, max_restarts=max_restarts,
                             restart=40 - augment, augment=augment, lin_tol=1e-12, prec=prec, inner_tol=1e-4,
                             max_outer=30, evecs=[(evr, evi)])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        lam[name] = r[0]["lam"]
        out["eigs_3d_%d_nev%d_%s%s" % (side, nev, "lgmres_" if augment else "", name)] = {"seconds": el, "rc": rc, "nconv": r[0]["nconv"],
                                                "n_matvec": r[0]["n_matvec"], "n_cayley": r[0]["n_cayley"],
                                                "lam": [[l.real, l.imag] for l in r[0]["lam"]],
                                                "resid": r[0]["resid"]}
        if log:
            log("eigs 3d %d %s%s: %.1f s, %d matvecs" % (side, "lgmres " if augment else "", name, el,
                                                       r[0]["n_matvec"]))
    dev_rel = [abs(a - b) / abs(a) for a, b in zip(sorted(lam["fp64"], key=abs), sorted(lam["mixed"], key=abs))]
    key = "eigs_3d_%d_nev%d_%s" % (side, nev, "lgmres_" if augment else "")
    out[key + "mixed_vs_fp64"] = {"speedup": out[key + "fp64"]["seconds"] / out[key + "mixed"]["seconds"],
                                  "max_rel_dev": max(dev_rel)}
    ctx.close()
    return out


def sweep(torch, dev, nev=2, augment=0, modes=("sequential", "concurrent"), log=None, sides=(16, 24, 32),
          tag="reduced", max_matvec=10 ** 7):
    """Sweep of uneven base flows (the sweep's Mach/Re recipe on the given
    sides, 8 problems), each its own mixed-precision Cayley-IRAM: the
    problems one after another on one stream, then all at once on one stream
    each (run concurrently by the library).  max_matvec caps each inner
    solve."""
    import numpy as np
    import synth
    from paper_1502_03701_amd import SA_MIXED, Context, arnoldi_eigs
    items = synth.config4_reduced(sides=sides)
    kw = dict(nev=nev, ncv=16, sigma=0.2, mu=-0.2, tol=1e-8, max_restarts=100, restart=40 - augment,
              augment=augment, lin_tol=1e-10, prec=SA_MIXED, inner_tol=1e-4, max_outer=20, max_matvec=max_matvec)
    out = {}
    for mode in modes:
        if mode == "sequential":
            streams = [torch.cuda.current_stream()] * len(items)
        else:
            streams = [torch.cuda.Stream() for _ in items]
        ctxs, v0s = [], []
        for it, st in zip(items, streams):
            c = Context(stream=st)
            c.base_set(it.problem, torch.from_numpy(synth.base_flow(it.problem).ravel()).to(dev))
            ctxs.append(c)
            v0s.append(torch.from_numpy(synth.random_vector(it.problem, it.seed).ravel()).to(dev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode == "sequential":
            r = []
            for i, (c, v) in enumerate(zip(ctxs, v0s)):
                r += arnoldi_eigs([c], [v], **kw)[1]
                if log:
                    log("sweep problem %d (%dx%d): %.2f s" % (i, items[i].problem.n[0], items[i].problem.n[1],
                                                             r[-1]["seconds"]))
        else:
            r = arnoldi_eigs(ctxs, v0s, **kw)[1]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        secs = np.array([x["seconds"] for x in r])
        pairs = int(sum(min(x["nconv"], nev) for x in r))
        out["sweep_" + tag + "_" + ("lgmres_" if augment else "") + mode] = {
            "problems": len(items), "sides": [it.problem.n[0] for it in items], "eigenpairs": pairs,
            "seconds": el, "eigenpairs_per_s": pairs / el, "p50_s": float(np.percentile(secs, 50)),
            "p99_s": float(np.percentile(secs, 99)), "n_matvec": int(sum(x["n_matvec"] for x in r))}
        if log:
            log("sweep %s %s%s: %.2f s" % (tag, "lgmres " if augment else "", mode, el))
        for c in ctxs:
            c.close()
    return out


def sweep_c4(torch, dev, log=None, nev=2, modes=("sequential", "concurrent"), restart=4):
    """The 48-flow sweep as configured (sides 128^2 - 768^2, M ~ U[0.1, 0.8],
    Re ~ U[300, 2000], seed 4), each flow its own Cayley-IRAM problem (nev
    leading eigenpairs, Arnoldi dimension 16, tol 1e-10) in the mixed form,
    inner solves right-preconditioned with the mean-flow operator (for
    these parallel bases, J - sigma I itself, factored per x-Fourier mode).
    With that preconditioner each inner solve converges in one or two Krylov
    steps, and the rest of a captured GMRES(m) cycle is launches that return
    at once; these small problems are launch-bound, so the inner solver is
    GMRES(4) (the same products and eigenvalues as GMRES(30), 1.6x faster).
    Run twice: in turn on one stream, and concurrently: every problem on a
    stream of its own (created here: torch's pool hands out at most 32
    distinct streams per device), handed to the library largest first, whose
    16 host threads take the next problem as they finish one.  The timed
    region covers each problem's preconditioner setup and its eigen solve;
    p50/p99 are over the library's per-problem wall times."""
    import numpy as np
    import synth
    from paper_1502_03701_amd import SA_F32, SA_MIXED, SA_PC_MEAN_FLOW, Context, arnoldi_eigs
    items = synth.config4_sweep()
    kw = dict(nev=nev, ncv=16, sigma=0.2, mu=-0.2, tol=1e-10, max_restarts=60, restart=restart, lin_tol=1e-12,
              prec=SA_MIXED, inner_tol=1e-4, use_precond=True)
    out = {}
    for mode in modes:
        own = []
        if mode == "sequential":
            streams = [torch.cuda.current_stream()] * len(items)
        else:
            own = [_hip_stream() for _ in items]
            streams = [torch.cuda.ExternalStream(h, device=dev) for h in own]
        ctxs, v0s = [], []
        for it, st in zip(items, streams):
            c = Context(stream=st)
            c.base_set(it.problem, torch.from_numpy(synth.base_flow(it.problem).ravel()).to(dev))
            ctxs.append(c)
            v0s.append(torch.from_numpy(synth.random_vector(it.problem, it.seed).ravel()).to(dev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode == "sequential":
            r = []
            for c, v in zip(ctxs, v0s):
                c.precond_setup([0.2], factor_prec=SA_F32, kind=SA_PC_MEAN_FLOW)
                r += arnoldi_eigs([c], [v], **kw)[1]
        else:
            order = sorted(range(len(items)), key=lambda i: -items[i].problem.ndof)
            for c in ctxs:
                c.precond_setup([0.2], factor_prec=SA_F32, kind=SA_PC_MEAN_FLOW)
            ro = arnoldi_eigs([ctxs[i] for i in order], [v0s[i] for i in order], **kw)[1]
            r = [None] * len(items)
            for i, x in zip(order, ro):
                r[i] = x
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        secs = np.array([x["seconds"] for x in r])
        pairs = int(sum(min(x["nconv"], nev) for x in r))
        out[mode] = {"problems": len(items), "eigenpairs": pairs, "seconds": el, "eigenpairs_per_s": pairs / el,
                     "p50_s": float(np.percentile(secs, 50)), "p99_s": float(np.percentile(secs, 99)),
                     "n_cayley": int(sum(x["n_cayley"] for x in r)),
                     "n_matvec": int(sum(x["n_matvec"] for x in r))}
        if mode == "sequential":
            out["leading"] = [[it.problem.n[0], it.problem.mach, it.problem.re, max(x["lam"], key=lambda z: z.real).real]
                              for it, x in zip(items, r)]
        if log:
            log("sweep c4 %s: %.2f s, %d eigenpairs" % (mode, el, pairs))
        for c in ctxs:
            c.close()
        for h in own:
            _hip_stream_destroy(h)
    return out


def _hip():
    """The HIP runtime this process already runs on (torch and libsa share
    it); opening the library by name could map a second copy."""
    import ctypes
    paths = sorted({ln.split()[-1] for ln in open("/proc/self/maps") if "libamdhip64.so" in ln})
    if len(paths) != 1:
        raise RuntimeError("expected one mapped HIP runtime, found %s" % paths)
    lib = ctypes.CDLL(paths[0])
    lib.hipStreamCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
    lib.hipStreamDestroy.argtypes = [ctypes.c_void_p]
    return lib


def _hip_stream():
    """A new non-blocking HIP stream of the default priority (its handle)."""
    import ctypes
    h = ctypes.c_void_p()
    rc = _hip().hipStreamCreateWithFlags(ctypes.byref(h), 1)
    if rc != 0:
        raise RuntimeError("hipStreamCreateWithFlags failed: %d" % rc)
    return h.value


def _hip_stream_destroy(h):
    import ctypes
    _hip().hipStreamDestroy(ctypes.c_void_p(h))


if __name__ == "__main__":
    main()
