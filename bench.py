#!/usr/bin/env python
"""Benchmark: Chebyshev-filtered subspace iteration on one MI355X.

One step = one complete solve (Algorithm 1: reduction, Lanczos, filter, QR,
Rayleigh-Ritz, locking, back-transform) of one generalized eigenproblem of a
correlated sequence, warm-started from the previous solve's vectors, with the
matrices already resident in device memory.

Default workload: a sequence of correlated complex Hermitian DGEVPs with
n = 4000, nev = 400, nex = 40, Chebyshev degree 20, tol 1e-10, FP64
throughout (synthetic FLAPW-shaped inputs; the paper's FLEUR matrices are not
available).  Prints one JSON line.

The filter kernel is timed live with HIP events around every launch on the
solver's stream (profile mode of the library); its algorithmic work is
8 n^2 k_active flops per degree step.
"""
import argparse
import json
import math
import os
import sys
import time

METRIC = "Chebyshev-filter TFLOP/s + eigensolves/s (FP64 vs mixed) at residual ≤1e-10"
PEAK_FP64_MFMA = 78.6  # TFLOP/s, MI355X dense FP64 matrix peak

WORKLOADS = {
    # correlated sequence (the plain method at scale)
    "seq4000": dict(n=4000, nev=400, nex=40, degree=20, seed=1, sequence=True,
                    desc="sequence of correlated complex Hermitian DGEVPs, FLAPW-shaped synthetic spectrum"),
    # single problem of the small configuration
    "single512": dict(n=512, nev=51, nex=13, degree=10, seed=0, sequence=False,
                      desc="single complex Hermitian DGEVP, FLAPW-shaped synthetic spectrum"),
    # single large problem (FP64 path of the precision study)
    "single10000": dict(n=10000, nev=600, nex=60, degree=20, seed=2, sequence=False,
                        desc="single complex Hermitian DGEVP, FLAPW-shaped synthetic spectrum"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_problems(cfg, count, device):
    import torch
    import workloads
    if cfg["sequence"]:
        gen = workloads.make_sequence_torch(cfg["n"], count, cfg["seed"], device=device)
        probs = []
        for i, p in enumerate(gen):
            probs.append(p)
            log(f"[bench] generated problem {i + 1}/{count}")
        return probs
    p = workloads.make_problem_torch(cfg["n"], cfg["seed"], device=device)
    return [p] * count


def residual_check(p, evals, X):
    """max_j ||H x_j - lam_j S x_j|| / ||H||_2 estimate, on the device (a
    check of the result, not part of the timed path)."""
    import torch
    H, S = p["H"], p["S"]
    lam = torch.as_tensor(evals, dtype=torch.complex128, device=X.device)
    R = H @ X - (S @ X) * lam[None, :]
    v = torch.ones(H.shape[0], dtype=torch.complex128, device=X.device)
    for _ in range(30):
        v = H @ v
        v = v / torch.linalg.vector_norm(v)
    hn = float(torch.linalg.vector_norm(H @ v))
    return float(torch.linalg.vector_norm(R, dim=0).max()) / hn


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "chebyshev_step_f64_seq4000_traffic.md")
KERNEL_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1305_5120_amd", "csrc", "zgemm.hip")


def measured_traffic(workload):
    """HBM bytes per filter launch from the committed counter summary, or
    None when the summary is absent, for another workload, or was taken on a
    different version of the kernel source."""
    import hashlib
    if workload != "seq4000" or not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if vals.get("kernel_source_sha256") != sha:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


CAL_N = 6000


def calibrate_copy():
    """Plain device copies of known size for scaling the memory counters of a
    profiled run: the library's k_copy2d kernel moving contiguous
    6000 x 6000 complex128 matrices (576,000,000 bytes read and written per
    launch; the reduction copies S once and chfsi_copy_factors copies A, L
    and L^{-1})."""
    import torch
    from paper_1305_5120_amd import chfsi
    n = CAL_N
    eye = torch.eye(n, dtype=torch.complex128, device="cuda").mT.contiguous().mT
    ctx = chfsi.create(n)
    chfsi.reduce(ctx, eye, eye)
    chfsi.copy_factors(ctx)
    torch.cuda.synchronize()
    ctx.release()
    log(f"[bench] copy calibration: k_copy2d launches with grid {n * n} moving {16 * n * n} bytes each way")


def cpu_baseline(cfg, gpu_filter_flops_per_solve, target_seconds=12.0):
    """Time the CPU oracle's filter on a bounded sample of the same problem
    and scale it to solves/s of the filter work of one GPU solve."""
    import numpy as np
    import oracle
    import workloads
    n = cfg["n"]
    rng = np.random.default_rng(99)
    # standard-form matrix with the workload's spectrum law (host copy)
    lam = workloads.spectrum(n, rng)
    G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2)
    Q, _ = np.linalg.qr(G)
    A = np.asfortranarray((Q * lam) @ Q.conj().T)
    A = (A + A.conj().T) / 2
    del G, Q
    lo, hi = float(np.sort(lam)[cfg["nev"] + cfg["nex"]]), float(lam.max() * 1.1)
    m = 2
    k = 8
    Y = oracle.gauss_block(1, 3, n, k)
    t0 = time.perf_counter()
    oracle.chebyshev_filter(A, Y, m, lo, hi, float(lam.min()))
    dt = time.perf_counter() - t0
    rate = 8.0 * n * n * k * m / dt
    # scale the sample (columns first, then degree) to about target_seconds
    k2 = int(max(8, min(cfg["nev"] + cfg["nex"], rate * target_seconds / (8.0 * n * n * m))))
    m2 = int(max(2, min(cfg["degree"], round(rate * target_seconds / (8.0 * n * n * k2)))))
    if k2 > k or m2 > m:
        Y = oracle.gauss_block(1, 3, n, k2)
        t0 = time.perf_counter()
        oracle.chebyshev_filter(A, Y, m2, lo, hi, float(lam.min()))
        dt = time.perf_counter() - t0
        rate = 8.0 * n * n * k2 * m2 / dt
        k, m = k2, m2
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    solve_s = gpu_filter_flops_per_solve / rate
    return {
        "value": 1.0 / solve_s,
        "unit": "solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"oracle Chebyshev filter, n={n}, {k} columns, degree {m} ({dt:.1f} s, "
                   f"{rate / 1e9:.2f} GFLOP/s); solve rate = that rate applied to the filter work of one GPU "
                   f"solve ({gpu_filter_flops_per_solve / 1e12:.2f} TFLOP), the rest of the solve not counted"),
        "filter_gflops": rate / 1e9,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="seq4000", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="do not time filter launches with events")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, run a device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs one problem sequence on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        sys.exit("need --steps >= 1 and --warmup >= 0")

    import torch
    from paper_1305_5120_amd import chfsi
    chfsi.load()
    dev = torch.device("cuda:0")
    cfg = WORKLOADS[args.workload]
    total = args.warmup + args.steps
    probs = make_problems(cfg, total, dev)
    torch.cuda.synchronize()

    n, nev, nex = cfg["n"], cfg["nev"], cfg["nex"]
    ctx = chfsi.create(n, degree=cfg["degree"], seed=0, profile=0 if args.no_profile else 1)
    S0 = probs[0]["S"]
    infos = []

    def one(i):
        p = probs[i]
        S = S0 if i == 0 else (None if cfg["sequence"] else p["S"])
        if not cfg["sequence"]:
            ctx.reset()
        ev, X, info, st = chfsi.solve(ctx, p["H"], S, nev, nex, tol=1e-10)
        return ev, X, info

    for i in range(args.warmup):
        ev, X, info = one(i)
        log(f"[bench] warmup solve {i}: {info['iterations']} iterations, {info['t_total']:.3f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, total):
        ev, X, info = one(i)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i, info in enumerate(infos):
        log(f"[bench] timed solve {i}: {info['iterations']} iterations, warm={info['warm_start']}, "
            f"{info['t_total']:.3f} s, filter {info['t_filter']:.3f} s")
    elapsed = t1 - t0
    rel_res = residual_check(probs[total - 1], ev, X)

    flops = sum(i["filter_flops"] for i in infos)
    fsec = sum(i["filter_kernel_seconds"] for i in infos)
    launches = sum(i["filter_launches"] for i in infos)
    achieved = flops / fsec / 1e12 if fsec > 0 else None
    phase = {k: sum(i[k] for i in infos) for k in ("t_reduce", "t_lanczos", "t_filter", "t_qr", "t_rr", "t_resid")}
    # algorithmic bytes per launch: A once, Y_i and Y_{i-1} read, Y_{i+1}
    # written; 8 n^2 k_a flops per launch give the mean k_a
    mean_ka = (flops / launches) / (8.0 * n * n) if launches else 0.0
    alg_bytes = 16.0 * n * n + 48.0 * n * mean_ka
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex128 (f64)",
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "n": n, "nev": nev, "nex": nex, "degree": cfg["degree"], "tol": 1e-10,
                   "precision": "fp64", "warm_start": cfg["sequence"], "parallelism": "none (1 GPU)"},
        "filter_tflops": achieved,
        "filter_avg_launch_ms": 1e3 * fsec / launches if launches else None,
        "filter_launches": launches,
        "max_rel_residual": rel_res,
        "iterations": [i["iterations"] for i in infos],
        "phase_seconds": phase,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s",
                     "frac": (achieved / PEAK_FP64_MFMA) if achieved else None,
                     "traffic": measured_traffic(args.workload),
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "algorithmic_flops_per_launch": flops / launches if launches else None},
    }
    if args.calibrate_copy:
        calibrate_copy()
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(cfg, flops / len(infos))
    print(json.dumps(out), flush=True)
    ctx.release()


if __name__ == "__main__":
    main()
