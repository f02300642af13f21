"""Benchmark: throughput of the matrix-free operator J v on one MI355X.

Workload (default): the 3D mixing layer on a 256 x 128 x 128 grid (x and z
periodic, walls in y), 5 variables, tanh(y) base flow with seeded 1e-3 N(0,1)
spanwise velocity, M = 0.5, Re = 1000, FP64.  One step is one application of
y = (J - sigma I) x over the whole grid (sa_op_apply, sigma = 0.2), inputs
resident in HBM.  value = grid-point updates per second (all five outputs of
one point = one update).

Also reported: the roofline record of the operator kernel (algorithmic bytes
= read x + read q0 + write y = 3 nv 8 B per point, against 8 TB/s), the same
operator in FP32, optional extras (--extras: GMRES iteration time at the 2D
512 x 512 case, block-Jacobi apply, time to eigenpairs FP64 vs mixed on a
small case), and the oracle timed on the host cores on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--extras]
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


def timed_launches(fn, steps, warmup, torch):
    """HIP events on the current stream (the stream the library launches on)."""
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
    return start.elapsed_time(stop) / 1e3   # seconds


def cpu_baseline(prob, q0, v):
    """Oracle complex-step Jv on a bounded window of the workload (a 16-wide
    slab in x and z over the full y range, about 10 s of CPU work), scaled
    to Gpt/s."""
    import numpy as np
    import synth
    from oracle import operator as op
    W = 16
    nx, ny, nz = prob.n
    sub = synth.mixing_layer_3d(W, ny, W, prob.mach, prob.re, lx=W * prob.length[0] / nx,
                                ly=prob.length[1], lz=W * prob.length[2] / nz)
    qs = np.ascontiguousarray(q0[:, :W, :, :W])
    vs = np.ascontiguousarray(v[:, :W, :, :W])
    op.jv_cstep(sub, qs, vs)            # warm-up
    reps = 0
    t0 = time.perf_counter()
    while True:
        op.jv_cstep(sub, qs, vs)
        reps += 1
        el = time.perf_counter() - t0
        if el > 10.0 or reps >= 50:
            break
    rate = reps * sub.npts / el / 1e9
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"value": rate, "unit": "Gpt/s", "cores": 1, "kind": "oracle",
            "sample": "complex-step Jv (NumPy, one thread for elementwise work) on a "
                      "%dx%dx%d window of the workload, %d repetitions in %.1f s; host has %d cores"
                      % (W, ny, W, reps, el, cores)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is documented, not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1502_03701_amd import Context

    dev = torch.device("cuda:0")
    prob = synth.config2()
    q0 = synth.base_flow(prob, seed=2, w_noise=1e-3)
    v = synth.random_vector(prob, 2)
    ctx = Context()
    ctx.base_set(prob, torch.from_numpy(q0.ravel()).to(dev))
    x = torch.from_numpy(v.ravel()).to(dev)
    y = torch.empty_like(x)
    npts = prob.npts
    nv = prob.nv

    sec = timed_launches(lambda: ctx.op_apply(x, y, shift=0.2), args.steps, args.warmup, torch)
    per = sec / args.steps
    value = npts / per / 1e9
    alg_bytes = 3 * nv * 8 * npts
    achieved = alg_bytes / per / 1e9

    x32 = x.float()
    y32 = torch.empty_like(x32)
    sec32 = timed_launches(lambda: ctx.op_apply(x32, y32, shift=0.2), args.steps, args.warmup, torch)
    per32 = sec32 / args.steps

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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "jv (FP64, 3D)", "alg_bytes_per_point": 3 * nv * 8},
        "fp32_jv": {"gpts": npts / per32 / 1e9, "ms": per32 * 1e3,
                    "achieved_GBs": 3 * nv * 4 * npts / per32 / 1e9},
    }
    if args.extras:
        out["extras"] = extras(torch, dev)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, q0, v)
    print(json.dumps(out))


def extras(torch, dev):
    """Secondary measurements (not the headline value)."""
    import synth
    from paper_1502_03701_amd import SA_MIXED, Context, arnoldi_eigs
    res = {}
    # GMRES(40) iteration cost at 512 x 512 (2D, FP64), capped solve
    p1 = synth.config1()
    c1 = Context()
    c1.base_set(p1, torch.from_numpy(synth.base_flow(p1).ravel()).to(dev))
    b = torch.from_numpy(synth.random_vector(p1, 1).ravel()).to(dev)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, info = c1.gmres_solve([0.2], b, x, restart=40, tol=1e-10, max_matvec=2000)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res["gmres40_512x512"] = {"iters": info[0]["iters"], "relres": info[0]["relres"],
                              "ms_per_iter": el / max(1, info[0]["iters"]) * 1e3}
    # time to eigenpairs, FP64 vs mixed, small case (KH pair)
    pe = synth.mixing_layer_2d(32, 32, 0.5, 1000.0)
    ce = Context()
    ce.base_set(pe, torch.from_numpy(synth.base_flow(pe).ravel()).to(dev))
    v0 = torch.from_numpy(synth.random_vector(pe, 0).ravel()).to(dev)
    for name, prec in (("fp64", 0), ("mixed", SA_MIXED)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, r = arnoldi_eigs([ce], [v0], nev=2, ncv=16, tol=1e-10, restart=40, lin_tol=1e-12,
                             prec=prec, inner_tol=1e-4, max_outer=20)
        el = time.perf_counter() - t0
        res["eigs_kh_32x32_" + name] = {"seconds": el, "nconv": r[0]["nconv"],
                                        "lam": [[l.real, l.imag] for l in r[0]["lam"]],
                                        "n_matvec": r[0]["n_matvec"]}
    return res


if __name__ == "__main__":
    main()
