#!/usr/bin/env python
"""Benchmark: Chebyshev-filtered subspace iteration on one MI355X.

One step = one complete solve (Algorithm 1: reduction, Lanczos, filter, QR,
Rayleigh-Ritz, locking, back-transform) of one generalized eigenproblem with
the matrices already resident in device memory.

Default workload: a single complex Hermitian DGEVP with n = 10000,
nev = 600, nex = 60, Chebyshev degree 20, tol 1e-10, solved cold (random
start block) at every step, FP64 throughout (`value`); the same problem is
then solved with the two mixed-precision filters (complex FP32 degree steps,
FP64 everything else and FP64 final sweeps; every degree step in complex
FP32 on the Ritz residual, no FP64 sweeps; the same with FP16 operands),
reported beside it with the error
of every eigenpair against the constructed spectrum and the FP64 path.  The
inputs are synthetic FLAPW-shaped problems (the paper's FLEUR matrices are
not available).  Prints one JSON line.  `--workload seq4000` runs the
correlated n = 4000 sequence (warm starts) instead.

The filter kernel is timed live with HIP events on the solver's stream
(profile mode of the library): one event pair around each filter call's
consecutive degree steps, so the average per launch includes the short gaps
between back-to-back launches; its algorithmic work is 8 n^2 k_active flops
per degree step.
"""
import argparse
import json
import math
import os
import sys
import time

METRIC = "Chebyshev-filter TFLOP/s + eigensolves/s (FP64 vs mixed) at residual ≤1e-10"
PEAK_FP64_MFMA = 78.6  # TFLOP/s, MI355X dense FP64 matrix peak
# Filter flops are the method's complex work, 8 real flops per complex
# multiply-add; the filter kernels form complex products with three real
# matrix products (Gauss's 3M form), so the matrix cores execute 6 of the 8.
FLOP_COUNT_NOTE = "8 real flops per complex multiply-add; the 3M products execute 6 of them on the matrix cores"
GAUSS3_SHARE = 6.0 / 8.0

WORKLOADS = {
    # correlated sequence (the plain method at scale)
    "seq4000": dict(n=4000, nev=400, nex=40, degree=20, seed=1, sequence=True,
                    desc="sequence of correlated complex Hermitian DGEVPs, FLAPW-shaped synthetic spectrum"),
    # single problem of the small configuration
    "single512": dict(n=512, nev=51, nex=13, degree=10, seed=0, sequence=False,
                      desc="single complex Hermitian DGEVP, FLAPW-shaped synthetic spectrum"),
    # single large problem, cold solves: FP64 (the value) and mixed precision
    "single10000": dict(n=10000, nev=600, nex=60, degree=20, seed=2, sequence=False,
                        desc="single complex Hermitian DGEVP, FLAPW-shaped synthetic spectrum, cold start"),
}
DEFAULT_WORKLOAD = "single10000"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class _Marker:
    """A named host range for profilers that record ROCTX markers
    (rocprofv3 --marker-trace): the timed region is marked so a profile can
    be restricted to it.  A no-op where the marker library is absent."""

    def __init__(self):
        import ctypes
        try:
            self.lib = ctypes.CDLL("librocprofiler-sdk-roctx.so.1")
            self.lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
        except OSError:
            self.lib = None

    def push(self, name):
        if self.lib:
            self.lib.roctxRangePushA(name.encode())

    def pop(self):
        if self.lib:
            self.lib.roctxRangePop()


MARKER = _Marker()


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


def residual_norm_scale(H):
    """||H||_2 from 40 Lanczos steps with full re-orthogonalization on the
    device: an estimate from below that is accurate to many digits (a check of
    results, not part of any timed path)."""
    import numpy as np
    import torch
    n = H.shape[0]
    g = torch.Generator(device="cpu").manual_seed(7)
    v = torch.complex(torch.randn(n, generator=g, dtype=torch.float64),
                      torch.randn(n, generator=g, dtype=torch.float64)).to(H.device)
    V = [v / torch.linalg.vector_norm(v)]
    alpha, beta = [], []
    for j in range(min(40, n)):
        w = H @ V[-1]
        alpha.append(float(torch.vdot(V[-1], w).real))
        for u in V:
            w = w - torch.vdot(u, w) * u
        b = float(torch.linalg.vector_norm(w))
        if b == 0.0:
            break
        beta.append(b)
        V.append(w / b)
    T = np.diag(alpha) + np.diag(beta[:len(alpha) - 1], 1) + np.diag(beta[:len(alpha) - 1], -1)
    return float(np.abs(np.linalg.eigvalsh(T)).max())


def residual_check(p, evals, X, hnorm=None):
    """max_j ||H x_j - lam_j S x_j|| / ||H||_2 on the device (a check of the
    result, not part of the timed path)."""
    import torch
    H, S = p["H"], p["S"]
    lam = torch.as_tensor(evals, dtype=torch.complex128, device=X.device)
    R = H @ X - (S @ X) * lam[None, :]
    hn = hnorm if hnorm is not None else residual_norm_scale(H)
    return float(torch.linalg.vector_norm(R, dim=0).max()) / hn


PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
KERNEL_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1305_5120_amd", "csrc", "zgemm.hip")


def _summary_fields(path):
    """`- key: value` lines of a committed profile summary."""
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    return vals


def _current_summary(name):
    """Fields of profiles/<name> when it exists and was taken on the current
    kernel source (its kernel_source_sha256 matches), else None."""
    import hashlib
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    vals = _summary_fields(path)
    sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    return vals if vals.get("kernel_source_sha256") == sha else None


def measured_traffic(workload):
    """HBM bytes per filter launch from the committed counter summary of this
    workload, or None when the summary is absent or was taken on a different
    version of the kernel source."""
    vals = _current_summary(f"chebyshev_step_f64_{workload}_traffic.md")
    try:
        return float(vals["hbm_bytes_per_launch"]) if vals else None
    except (KeyError, ValueError):
        return None


def measured_mfma(workload):
    """Matrix-core use of the filter kernel from the committed counter
    summary of this workload: (busy fraction of the matrix pipes over the
    CUs' busy cycles, executed matrix flops over the FP64 matrix peak), or
    (None, None) when the summary is absent or was taken on a different
    version of the kernel source."""
    vals = _current_summary(f"chebyshev_step_f64_{workload}_mfma.md")
    try:
        return (float(vals["mfma_busy_fraction"]), float(vals["matrix_core_flop_fraction"])) if vals else (None, None)
    except (KeyError, ValueError):
        return None, None


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_c0_solves(threads, runs, warmup, budget_s):
    """Full oracle solves of the small configuration (n = 512, nev = 51,
    nex = 13, degree 10, tol 1e-10, cold start) on `threads` threads: median
    of up to `runs` timed solves after `warmup` untimed ones, stopping early
    once `budget_s` seconds have been spent."""
    import numpy as np
    import oracle
    import workloads
    p = workloads.make_problem(512, 0)
    prev = oracle.set_threads(threads)
    try:
        t_all = time.perf_counter()
        for _ in range(warmup):
            oracle.solve(p.H, p.S, 51, 13, tol=1e-10, degree=10, seed=0)
        times = []
        for _ in range(runs):
            t0 = time.perf_counter()
            r = oracle.solve(p.H, p.S, 51, 13, tol=1e-10, degree=10, seed=0)
            times.append(time.perf_counter() - t0)
            if time.perf_counter() - t_all > budget_s:
                break
        assert r["info"]["status"] == 0
        return {"threads": oracle.set_threads(prev), "median_s": float(np.median(times)), "runs": len(times),
                "warmup": warmup, "iterations": r["info"]["iterations"]}
    finally:
        oracle.set_threads(prev)


def cpu_baseline(cfg, gpu_filter_flops_per_solve, target_seconds=8.0):
    """The CPU oracle timed on this host.

    * value: the oracle's Chebyshev filter timed on a bounded sample of the
      benchmarked problem's size (n, a few columns and degree steps, about
      target_seconds), its rate applied to the filter work of one GPU solve
      -- an upper bound on the oracle's solve rate, since the rest of its
      solve (reduction, QR, Rayleigh-Ritz, residuals) is not counted;
    * c0_full_solve: complete oracle solves of the small configuration
      (n = 512) on all threads (warm-up, median of 5) and on one thread."""
    import numpy as np
    import oracle
    import workloads
    threads = oracle.set_threads(0)
    full = _oracle_c0_solves(threads, 5, 1, 25.0)
    one = _oracle_c0_solves(1, 3, 0, 20.0)
    log(f"[bench] oracle n=512 solve: {full['median_s']:.2f} s on {full['threads']} threads, "
        f"{one['median_s']:.2f} s on 1 thread")
    n = cfg["n"]
    rng = np.random.default_rng(99)
    lam = workloads.spectrum(n, rng)
    # the oracle's filter runs the full dense n x n product for every column
    # whatever the values, so a diagonal matrix with the workload's spectrum
    # costs what a dense one does (and needs no n x n QR on the host); its
    # loops are parallel over columns, so the sample takes a multiple of the
    # thread count
    A = np.asfortranarray(np.diag(lam).astype(np.complex128))
    lo, hi = float(np.sort(lam)[cfg["nev"] + cfg["nex"]]), float(lam.max() * 1.1)
    k, m = threads, 1
    rate, dt = 0.0, 0.0
    for _ in range(3):
        Y = oracle.gauss_block(1, 3, n, k)
        t0 = time.perf_counter()
        oracle.chebyshev_filter(A, Y, m, lo, hi, float(lam.min()))
        dt = time.perf_counter() - t0
        rate = 8.0 * n * n * k * m / dt
        if dt >= 0.4 * target_seconds:
            break
        grow = target_seconds / dt
        m2 = int(min(cfg["degree"], max(1, round(m * grow))))
        k2 = k if m2 * dt / m >= 0.4 * target_seconds else \
            int(min(cfg["nev"] + cfg["nex"], threads * max(1, round(k * grow * m / m2 / threads))))
        if (m2, k2) == (m, k):
            break
        m, k = m2, k2
    solve_s = gpu_filter_flops_per_solve / rate
    return {
        "value": 1.0 / solve_s,
        "unit": "solves/s",
        "cores": threads,
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": (f"oracle Chebyshev filter at n={n}: {k} columns, degree {m} ({dt:.1f} s, "
                   f"{rate / 1e9:.2f} GFLOP/s on {threads} threads); value = that rate applied to the filter work "
                   f"of one GPU solve ({gpu_filter_flops_per_solve / 1e12:.2f} TFLOP), the rest of the solve not "
                   f"counted (an upper bound on the oracle's solve rate)"),
        "filter_gflops": rate / 1e9,
        "c0_full_solve": {"workload": "n=512, nev=51, nex=13, degree 10, tol 1e-10, cold start",
                          "all_threads": full, "one_thread": one,
                          "solves_per_s_all_threads": 1.0 / full["median_s"],
                          "solves_per_s_one_thread": 1.0 / one["median_s"]},
    }


# --------------------------------------------------------------------------
# Further forms of the method, each printing its own JSON line: the
# precision form (FP64 vs mixed on one large problem), the batching form
# (many k-point sequences in lockstep), the serving form (Poisson arrivals),
# and the warm-versus-cold study along a sequence.
# --------------------------------------------------------------------------

def _base(metric, value, unit, steps, warmup, ms, dtype, config, higher=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def _exact_errors(p, evals):
    """max |lambda_i - lambda_i(exact)| / ||A||_2 over the returned pairs,
    against the spectrum the problem was built with."""
    import numpy as np
    lam = np.sort(p["lam"])[:len(evals)]
    return float(np.abs(np.asarray(evals) - lam).max() / np.abs(p["lam"]).max())


def run_precision(args):
    """One n = 10000 problem solved cold in FP64 and with the three mixed
    filters (precision 1: FP64 final sweeps; 2: FP32 on the Ritz residual;
    3: FP16 operands on the Ritz residual)."""
    import torch
    from paper_1305_5120_amd import chfsi
    import workloads
    n, nev, nex, m = 10000, 600, 60, 20
    p = workloads.make_problem_torch(n, 2, device="cuda")
    torch.cuda.synchronize()
    res = {}
    for prec in (0, 1, 2, 3):
        ctx = chfsi.create(n, degree=m, seed=0, precision=prec, profile=1)
        times = []
        for i in range(args.warmup + args.steps):
            ctx.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev, X, info, st = chfsi.solve(ctx, p["H"], p["S"], nev, nex, tol=1e-10)
            torch.cuda.synchronize()
            if i >= args.warmup:
                times.append(time.perf_counter() - t0)
        res[prec] = dict(t=sum(times) / len(times), info=info, err=_exact_errors(p, ev),
                         res=residual_check(p, ev, X),
                         phases={k: info[k] for k in ("t_reduce", "t_lanczos", "t_filter", "t_qr", "t_rr", "t_resid")})
        log(f"[bench] precision {prec}: {res[prec]['t']:.3f} s/solve, {info['iterations']} iterations "
            f"({info['iterations_fp32']} FP32), max eigenvalue error {res[prec]['err']:.2e}, "
            f"residual {res[prec]['res']:.2e}; phases " +
            ", ".join(f"{k[2:]} {info[k]:.2f}" for k in ("t_reduce", "t_lanczos", "t_filter", "t_qr", "t_rr", "t_resid")) +
            f"; filter kernels FP64 {info['filter_kernel_seconds'] - info['filter_kernel_seconds_fp32']:.2f} s, "
            f"FP32 {info['filter_kernel_seconds_fp32']:.2f} s")
        ctx.release()
    i64, i32, ir, ih = res[0]["info"], res[1]["info"], res[2]["info"], res[3]["info"]
    f32 = i32["filter_flops_fp32"] / i32["filter_kernel_seconds_fp32"] / 1e12 if i32["filter_kernel_seconds_fp32"] else None
    fr = ir["filter_flops_fp32"] / ir["filter_kernel_seconds_fp32"] / 1e12 if ir["filter_kernel_seconds_fp32"] else None
    fh = ih["filter_flops_fp32"] / ih["filter_kernel_seconds_fp32"] / 1e12 if ih["filter_kernel_seconds_fp32"] else None
    f64 = i64["filter_flops"] / i64["filter_kernel_seconds"] / 1e12 if i64["filter_kernel_seconds"] else None
    out = _base("eigensolves/s, mixed-precision filter (FP32 MFMA) with FP64 final sweeps, residual <=1e-10",
                1.0 / res[1]["t"], "solves/s", args.steps, args.warmup, 1e3 * res[1]["t"], "complex64 filter + f64",
                {"workload": "single complex Hermitian DGEVP, FLAPW-shaped synthetic spectrum", "n": n, "nev": nev,
                 "nex": nex, "degree": m, "tol": 1e-10, "precision": "mixed", "warm_start": False})
    out.update({"fp64_solves_per_s": 1.0 / res[0]["t"], "speedup_vs_fp64": res[0]["t"] / res[1]["t"],
                "fp64": {"iterations": i64["iterations"], "max_eig_error_rel": res[0]["err"],
                         "max_rel_residual": res[0]["res"], "filter_tflops": f64, "phase_seconds": res[0]["phases"]},
                "mixed": {"iterations": i32["iterations"], "iterations_fp32": i32["iterations_fp32"],
                          "max_eig_error_rel": res[1]["err"], "max_rel_residual": res[1]["res"],
                          "filter_tflops_fp32": f32, "phase_seconds": res[1]["phases"],
                          "filter_flops_fp32_share": i32["filter_flops_fp32"] / i32["filter_flops"]},
                "ritz32": {"solves_per_s": 1.0 / res[2]["t"], "speedup_vs_fp64": res[0]["t"] / res[2]["t"],
                           "iterations": ir["iterations"], "iterations_fp32": ir["iterations_fp32"],
                           "max_eig_error_rel": res[2]["err"], "max_rel_residual": res[2]["res"],
                           "filter_tflops_fp32": fr, "phase_seconds": res[2]["phases"],
                           "filter_flops_fp32_share": ir["filter_flops_fp32"] / ir["filter_flops"]},
                "ritz16": {"solves_per_s": 1.0 / res[3]["t"], "speedup_vs_fp64": res[0]["t"] / res[3]["t"],
                           "iterations": ih["iterations"], "iterations_low_precision": ih["iterations_fp32"],
                           "max_eig_error_rel": res[3]["err"], "max_rel_residual": res[3]["res"],
                           "filter_tflops_fp16_operands": fh, "phase_seconds": res[3]["phases"]},
                "roofline": {"bound": "mfma", "achieved": f32, "peak": 157.3, "unit": "TFLOP/s",
                             "frac": f32 / 157.3 if f32 else None, "flop_count": FLOP_COUNT_NOTE,
                             "matrix_core_frac": GAUSS3_SHARE * f32 / 157.3 if f32 else None, "traffic": None}})
    print(json.dumps(out), flush=True)


def _batch_sizes(count, seed):
    import numpy as np
    rng = np.random.default_rng(seed)
    return [int(v) for v in rng.integers(2000, 6001, count)]


def run_batch(args):
    """k-point sequences in lockstep (grouped filter launches, captured
    graphs, online tile choice, a mixed-precision filter) against the same problems
    solved one after another with one context per sequence.  The sequences
    advance together: only the current step's matrices are resident (the
    one-after-another pass draws the same sequences again)."""
    import torch
    from paper_1305_5120_amd import chfsi
    import workloads
    G, steps = args.members, args.seq_steps
    sizes = _batch_sizes(G, 3)
    nevs = [n // 10 for n in sizes]
    nexs = [max(1, v // 10) for v in nevs]
    prec = args.batch_precision
    sample = list(range(0, G, max(1, G // 4)))

    def sequences():
        return [workloads.make_sequence_torch(n, steps, 3 + i, device="cuda", rng_kind=args.gen_rng)
                for i, n in enumerate(sizes)]

    def first_step(gens):
        ps = []
        for i, g in enumerate(gens):
            ps.append(next(g))
            log(f"[bench] generated sequence {i + 1}/{G} (n={sizes[i]})")
        return [p["H"] for p in ps], [p["S"] for p in ps]

    # batched: step 0 cold (and the online tile choice), steps 1.. timed
    gens = sequences()
    H, S0 = first_step(gens)
    torch.cuda.synchronize()
    b = chfsi.Batch(sizes, use_graph=True, degree=20, seed=0, precision=prec)
    _, _, _, st, rep0 = b.solve(H, S0, nevs, nexs, tol=1e-10)
    log(f"[bench] batch cold step: {rep0['seconds']:.2f} s, tile {rep0['tile_config']}/{rep0['tile_config_fp32']}")
    reps = []
    tb = 0.0
    worst = 0.0
    none = [None] * G
    for ell in range(1, steps):
        H = [next(g)["H"] for g in gens]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, X, infos, st, rep = b.solve(H, none, nevs, nexs, tol=1e-10)
        torch.cuda.synchronize()
        tb += time.perf_counter() - t0
        reps.append(rep)
        log(f"[bench] batch step {ell}: {rep['seconds']:.2f} s, {rep['outer_iterations']} outer iterations, "
            f"grouped filter {rep['filter_seconds']:.2f} s ({rep['filter_flops'] / max(rep['filter_seconds'], 1e-9) / 1e12:.1f} TFLOP/s)")
        if ell == steps - 1:
            worst = max(residual_check({"H": H[i], "S": S0[i]}, ev[i], X[i]) for i in sample)
        del ev, X
    b.close()
    del gens, H
    # one after another (the same sequences drawn again)
    gens = sequences()
    H, S0 = first_step(gens)
    ctxs = [chfsi.create(n, degree=20, seed=0, precision=prec) for n in sizes]
    for i in range(G):
        chfsi.solve(ctxs[i], H[i], S0[i], nevs[i], nexs[i], tol=1e-10, want_vectors=False)
    ts = 0.0
    seq_filter = 0.0
    for ell in range(1, steps):
        H = [next(g)["H"] for g in gens]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(G):
            _, _, inf, _ = chfsi.solve(ctxs[i], H[i], None, nevs[i], nexs[i], tol=1e-10)
            seq_filter += inf["t_filter"]
        torch.cuda.synchronize()
        ts += time.perf_counter() - t0
        log(f"[bench] one after another, step {ell}: {ts:.2f} s so far")
    log(f"[bench] one after another: {ts:.2f} s for {G * (steps - 1)} solves, filter phases {seq_filter:.2f} s")
    for c in ctxs:
        c.release()
    del gens, H
    solves = G * (steps - 1)
    ff = sum(r["filter_flops"] for r in reps)
    fs = sum(r["filter_seconds"] for r in reps)
    out = _base("batched eigensolves/s over k-point sequences (grouped filter launches), residual <=1e-10",
                solves / tb, "solves/s", steps - 1, 1, 1e3 * tb / (steps - 1), "complex64 filter + f64",
                {"workload": "independent k-point sequences of correlated complex Hermitian DGEVPs",
                 "sequences": G, "n": f"uniform integers in [2000, 6000] (seed 3): {sizes}",
                 "nev": "n/10", "nex": "nev/10", "degree": 20, "tol": 1e-10,
                 "precision": {1: "mixed", 2: "FP32 filter on the Ritz residual"}[prec], "warm_start": True, "sequence_steps_timed": steps - 1, "generator_draws": args.gen_rng})
    out.update({"sequential_solves_per_s": solves / ts, "speedup_vs_sequential": ts / tb,
                "grouped_filter_tflops": ff / fs / 1e12 if fs else None,
                "tile_config": rep0["tile_config"], "tile_config_fp32": rep0["tile_config_fp32"],
                "tile_rate_tflops": rep0["tile_rate"], "graph": reps[-1]["graph"] if reps else None,
                "max_rel_residual_sampled": worst})
    print(json.dumps(out), flush=True)


def serving_law(nseq, seed, n_lo, n_hi):
    """Sizes of the serving form's sequences: n log-uniform in [n_lo, n_hi],
    nev uniform in 3-20 % of n (at least 4), nex = nev/10 (at least 1)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sizes = [int(round(math.exp(v))) for v in rng.uniform(math.log(n_lo), math.log(n_hi), nseq)]
    nevs = [max(4, int(n * f)) for n, f in zip(sizes, rng.uniform(0.03, 0.20, nseq))]
    nexs = [max(1, v // 10) for v in nevs]
    return sizes, nevs, nexs, rng


def serving_trace(nseq, requests, seed):
    """The first `requests` arrivals of the serving configuration's trace:
    each arrival is the next problem of a sequence drawn uniformly from the
    nseq sequences.  Returns [(sequence, step)]."""
    import numpy as np
    rng = np.random.default_rng(seed)
    count = [0] * nseq
    out = []
    for s in rng.integers(0, nseq, requests):
        out.append((int(s), count[s]))
        count[s] += 1
    return out


def run_serve(args):
    """Poisson arrivals of problems from many k-point sequences, served twice
    on the same arrival trace: by the plain FP64 path (one worker, one
    request at a time, warm starts) and by the full server (several workers
    on their own streams admitted by device memory, mixed-precision filter,
    warm starts).  Both must reach the same residual bound.  Later problems
    of a sequence pass no overlap matrix (S fixed along a sequence), so a
    worker holding the sequence's factor reuses it.

    --law small: sequences of the scaled-down law (n log-uniform in
    [1000, 6000], every sequence's steps in order); --law full: the serving
    configuration's law (128 sequences, n log-uniform in [2000, 20000]),
    bounded to the first --requests arrivals of its trace (each arrival the
    next problem of a uniformly drawn sequence); --serve-paths runs one of
    the two paths (the same trace and seeds either way)."""
    import numpy as np
    import torch
    from paper_1305_5120_amd import chfsi
    import workloads
    full = args.law == "full"
    if full:
        nseq = 128
        sizes, nevs, nexs, rng = serving_law(nseq, 4, 2000, 20000)
        order = serving_trace(nseq, args.requests, 41)
        rate = args.rate if args.rate_set else 0.05
    else:
        nseq, steps = args.members, args.seq_steps
        sizes, nevs, nexs, rng = serving_law(nseq, 4, 1000, 6000)
        order = [(s, ell) for ell in range(steps) for s in range(nseq)]
        rate = args.rate
    need = {}
    for s, ell in order:
        need[s] = max(need.get(s, 0), ell + 1)
    seqs = {}
    for i, s in enumerate(sorted(need)):
        # only H and S stay resident (the generator's A, Q, L are freed)
        seqs[s] = [{"H": p["H"], "S": p["S"]} for p in
                   workloads.make_sequence_torch(sizes[s], need[s], 400 + s, device="cuda",
                                                 rng_kind="device" if full else "host")]
        log(f"[bench] generated sequence {s} ({i + 1}/{len(need)}: n={sizes[s]}, nev={nevs[s]}, steps {need[s]})")
    torch.cuda.synchronize()
    gaps = rng.exponential(1.0 / rate, len(order))

    def serve(workers, precision, label):
        srv = chfsi.Server(workers=workers, hbm_budget_bytes=int(args.budget_gb * (1 << 30)), degree=20, seed=0,
                           precision=precision)
        t0 = time.perf_counter()
        tickets = []
        t_next = t0
        for (s, ell), g in zip(order, gaps):
            t_next += g
            d = t_next - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tickets.append(srv.submit(s, seqs[s][ell]["H"], seqs[s][0]["S"] if ell == 0 else None, nevs[s],
                                      nexs[s], tol=1e-10, want_vectors=False))
            log(f"[bench] {label}: submitted sequence {s} step {ell} (n={sizes[s]}, nev={nevs[s]})")
        worst = 0.0
        for t in tickets:
            _, _, info, lat, _ = srv.wait(t)
            worst = max(worst, info["max_rel_residual"])
            log(f"[bench] {label}: request done in {lat:.2f} s, {info['iterations']} iterations")
        elapsed = time.perf_counter() - t0
        stats = srv.stats()
        srv.close()
        log(f"[bench] {label}: {stats['completed']} requests in {elapsed:.1f} s, {stats['solves_per_second']:.3f} "
            f"solves/s, p50 {stats['p50_latency']:.3f} s, p99 {stats['p99_latency']:.3f} s, worst residual {worst:.2e}")
        return stats, elapsed, worst

    def path_report(st, res):
        return {"solves_per_s": st["solves_per_second"], "p50_latency_s": st["p50_latency"],
                "p99_latency_s": st["p99_latency"], "mean_latency_s": st["mean_latency"],
                "completed": st["completed"], "failed": st["failed"], "peak_bytes": st["peak_bytes"],
                "max_rel_residual": res}

    config = {"workload": "Poisson arrivals of DGEVP requests from k-point sequences", "sequences": nseq,
              "law": args.law,
              "n": (f"log-uniform in [2000, 20000] (seed 4)" if full else f"log-uniform in [1000, 6000] (seed 4)"),
              "requests": [{"sequence": s, "step": ell, "n": sizes[s], "nev": nevs[s], "nex": nexs[s]}
                           for s, ell in order],
              "nev": "uniform 3-20% of n", "nex": "nev/10", "arrival_rate_per_s": rate,
              "workers": args.workers, "hbm_budget_gb": args.budget_gb, "degree": 20, "tol": 1e-10}
    sp = args.serve_precision
    pname = {1: "mixed precision", 2: "FP32 filter on the Ritz residual", 3: "FP16-operand filter on the Ritz residual"}[sp]
    if args.serve_paths != "both":
        plain_only = args.serve_paths == "plain"
        st, elapsed, res = (serve(1, 0, "plain FP64, one worker") if plain_only else
                            serve(args.workers, sp, f"server, {args.workers} workers, {pname}"))
        out = _base("eigensolves/s and p50/p99 latency under Poisson arrivals, residual <=1e-10",
                    st["solves_per_second"], "solves/s", len(order), 0, 1e3 * elapsed / len(order),
                    "complex128 (f64)" if plain_only else "complex64 filter + f64",
                    dict(config, path="plain FP64, one worker" if plain_only else f"server, {pname}"))
        out.update(path_report(st, res))
        print(json.dumps(out), flush=True)
        return
    plain, _, plain_res = serve(1, 0, "plain FP64, one worker")
    stats, elapsed, res = serve(args.workers, sp, f"server, {args.workers} workers, {pname}")
    out = _base("eigensolves/s and p50/p99 latency under Poisson arrivals, residual <=1e-10",
                stats["solves_per_second"], "solves/s", len(order), 0, 1e3 * elapsed / len(order),
                "complex64 filter + f64", dict(config, precision=pname))
    out.update({"p50_latency_s": stats["p50_latency"], "p99_latency_s": stats["p99_latency"],
                "mean_latency_s": stats["mean_latency"], "completed": stats["completed"], "failed": stats["failed"],
                "peak_bytes": stats["peak_bytes"], "max_rel_residual": res,
                "plain_fp64_one_worker": path_report(plain, plain_res),
                "gain_vs_plain": {"solves_per_s": stats["solves_per_second"] / plain["solves_per_second"],
                                  "p50": plain["p50_latency"] / stats["p50_latency"],
                                  "p99": plain["p99_latency"] / stats["p99_latency"]}})
    print(json.dumps(out), flush=True)


def theta_angles(prevX, X, S):
    """Angles theta_i between consecutive eigenvectors x_i^(l-1), x_i^(l) in
    the S inner product (Sec. 2's correlation measure, read for S-normalized
    vectors as theta_i = arccos |<x_i^(l-1), x_i^(l)>_S|).  sin(theta) is taken
    from the S-norm of the part of x^(l) orthogonal to x^(l-1) and theta =
    atan2(sin, cos), which resolves small angles that arccos of a cosine near
    1 would round away.  Tensors of any device; returns a numpy array."""
    import torch
    c = torch.sum(prevX.conj() * (S @ X), dim=0)           # <x_(l-1), x_l>_S
    R = X - prevX * c[None, :]                             # part orthogonal to x_(l-1)
    sin = torch.sqrt(torch.clamp(torch.real(torch.sum(R.conj() * (S @ R), dim=0)), min=0.0))
    return torch.atan2(sin, torch.abs(c)).cpu().numpy()


def _standard_eigvals(H, S, count):
    """The `count` smallest eigenvalues of the pencil (H, S) from dense
    library eigensolvers on the device: S = V diag(s) V^H, then the
    eigenvalues of S^{-1/2} H S^{-1/2} (a pencil similar to (H, S); S is
    well conditioned here).  The reference of the warm/cold study's checks
    (the library's triangular solve runs out of workspace at these sizes)."""
    import torch
    s, V = torch.linalg.eigh(S)
    Sih = (V * s.rsqrt().to(V.dtype)[None, :]) @ V.conj().T
    A = Sih @ H @ Sih
    A = (A + A.conj().T) / 2
    return torch.linalg.eigvalsh(A)[:count].cpu().numpy()


def run_warmcold(args):
    """Warm versus cold starts along correlated sequences: a fixed
    perturbation with fixed S, the same with S varying (through the
    generalized-space map of the block), and a converging cycle (fixed S,
    perturbation 1e-2 shrinking tenfold per step).  Per step: iterations and
    times of both starts and the angle theta between consecutive eigenvectors
    in the S inner product (median over the wanted ones; sin(theta) from the
    S-norm of the part of x_l orthogonal to x_(l-1), accurate for small
    angles)."""
    import numpy as np
    import torch
    from paper_1305_5120_amd import chfsi
    import workloads
    n, nev, nex, steps = args.wc_n, args.wc_n // 10, max(1, args.wc_n // 100), args.seq_steps
    seq = list(workloads.make_sequence_torch(n, steps, 5, device="cuda"))
    seq_c = list(workloads.make_sequence_torch(n, steps, 5, eps=1e-2, eps_decay=0.1, device="cuda"))
    S0 = seq[0]["S"]
    # varying-S variant: S_l = L_l L_l^H with L_l = L_0 + 1e-4 (strict lower Gaussian)/sqrt(n) per step
    gen = torch.Generator(device="cpu").manual_seed(55)
    Ls = [seq[0]["L"]]
    for _ in range(1, steps):
        E = torch.complex(torch.randn(n, n, generator=gen, dtype=torch.float64),
                          torch.randn(n, n, generator=gen, dtype=torch.float64)).to("cuda") / math.sqrt(2)
        Ls.append(Ls[-1] + 1e-4 * torch.tril(E, -1) / math.sqrt(n))
    A_of = [p["A"] for p in seq]
    Hs_v = [(L @ A @ L.conj().T) for L, A in zip(Ls, A_of)]
    Hs_v = [((h + h.conj().T) / 2).mT.contiguous().mT for h in Hs_v]
    Ss_v = [((L @ L.conj().T + (L @ L.conj().T).conj().T) / 2).mT.contiguous().mT for L in Ls]
    torch.cuda.synchronize()

    def theta_median(prevX, X, S):
        return float(np.median(theta_angles(prevX, X, S)))

    rows = {}
    for variant in ("fixed_S", "varying_S", "converging"):
        warm = chfsi.create(n, degree=20, seed=0)
        cold = chfsi.create(n, degree=20, seed=0)
        prevX = None
        recs = []
        for ell in range(steps):
            if variant == "fixed_S":
                H, S_w, S_c, Sm = seq[ell]["H"], (S0 if ell == 0 else None), S0, S0
            elif variant == "varying_S":
                H, S_w, S_c, Sm = Hs_v[ell], Ss_v[ell], Ss_v[ell], Ss_v[ell]
            else:
                H, S_w, S_c, Sm = seq_c[ell]["H"], (S0 if ell == 0 else None), S0, S0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev, X, iw, _ = chfsi.solve(warm, H, S_w, nev, nex, tol=1e-10)
            torch.cuda.synchronize()
            tw = time.perf_counter() - t0
            cold.reset()
            t0 = time.perf_counter()
            evc, Xc, ic, _ = chfsi.solve(cold, H, S_c, nev, nex, tol=1e-10)
            torch.cuda.synchronize()
            tc = time.perf_counter() - t0
            theta = theta_median(prevX, X, Sm) if prevX is not None else None
            # verification (outside the timed solves): residuals of both
            # starts' pairs and their eigenvalues against a dense solver
            Sfull = Sm
            ref = _standard_eigvals(H, Sfull, nev)
            hn = residual_norm_scale(H)
            err_w = float(np.abs(np.asarray(ev) - ref).max() / hn)
            err_c = float(np.abs(np.asarray(evc) - ref).max() / hn)
            res_w = residual_check({"H": H, "S": Sfull}, ev, X, hnorm=hn)
            res_c = residual_check({"H": H, "S": Sfull}, evc, Xc, hnorm=hn)
            prevX = X
            recs.append({"step": ell, "warm_iterations": iw["iterations"], "cold_iterations": ic["iterations"],
                         "warm_s": tw, "cold_s": tc, "warm_start": iw["warm_start"], "median_theta": theta,
                         "warm_max_rel_residual": res_w, "cold_max_rel_residual": res_c,
                         "warm_max_eig_error": err_w, "cold_max_eig_error": err_c})
            log(f"[bench] {variant} step {ell}: warm {iw['iterations']} it {tw:.3f} s, cold {ic['iterations']} it "
                f"{tc:.3f} s, median theta {theta}; residual warm {res_w:.1e} cold {res_c:.1e}, "
                f"eigenvalue error warm {err_w:.1e} cold {err_c:.1e} (x ||H||)")
        warm.release()
        cold.release()
        rows[variant] = recs
    r = rows["fixed_S"][1:]
    speed = sum(x["cold_s"] for x in r) / sum(x["warm_s"] for x in r)
    out = _base("speed-up of warm over cold starts along a correlated sequence (eigensolves)", speed, "x",
                steps - 1, 1, 1e3 * sum(x["warm_s"] for x in r) / len(r), "complex128 (f64)",
                {"workload": "sequence of correlated complex Hermitian DGEVPs, FLAPW-shaped synthetic spectrum",
                 "n": n, "nev": nev, "nex": nex, "degree": 20, "tol": 1e-10, "steps": steps,
                 "perturbation": 1e-4, "converging_perturbation": "1e-2 * 0.1**(step - 1)"})
    out["per_step"] = rows
    out["speedup_varying_S"] = (sum(x["cold_s"] for x in rows["varying_S"][1:]) /
                                sum(x["warm_s"] for x in rows["varying_S"][1:]))
    out["speedup_converging"] = (sum(x["cold_s"] for x in rows["converging"][1:]) /
                                 sum(x["warm_s"] for x in rows["converging"][1:]))
    print(json.dumps(out), flush=True)


def run_mixed_same_workload(args, cfg, probs, fp64_rate, precision=1):
    """After the FP64 timed region: the same problems, in the same order and
    with the same warm starts, solved with a mixed-precision filter, timed
    the same way.  precision 1: complex FP32 degree steps for columns whose
    residual is above the switch, FP64 final sweeps to the same tolerance;
    precision 2: every degree step in complex FP32 on the Ritz residual (the
    recurrence split by linearity), no FP64 sweeps, the same tolerance;
    precision 3: as 2 with FP16 operands (FP32 accumulation)."""
    import torch
    from paper_1305_5120_amd import chfsi
    n, nev, nex = cfg["n"], cfg["nev"], cfg["nex"]
    ctx = chfsi.create(n, degree=cfg["degree"], seed=0, precision=precision, profile=0 if args.no_profile else 1)
    S0 = probs[0]["S"]
    # a bounded pass: the timed FP64 region above is the benchmark's value
    warmup = min(args.warmup, 1)
    steps = min(args.steps, 5)
    total = warmup + steps

    def one(i):
        p = probs[i]
        S = S0 if i == 0 else (None if cfg["sequence"] else p["S"])
        if not cfg["sequence"]:
            ctx.reset()
        return chfsi.solve(ctx, p["H"], S, nev, nex, tol=1e-10)

    for i in range(warmup):
        one(i)
    torch.cuda.synchronize()
    infos = []
    MARKER.push(f"bench.mixed_region_p{precision}")
    t0 = time.perf_counter()
    for i in range(warmup, total):
        ev, X, info, st = one(i)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    MARKER.pop()
    rel_res = residual_check(probs[total - 1], ev, X)
    del X
    ctx.release()
    f32s = sum(i["filter_kernel_seconds_fp32"] for i in infos)
    f32f = sum(i["filter_flops_fp32"] for i in infos)
    rate = steps / elapsed
    log(f"[bench] precision {precision}, same problems: {rate:.3f} solves/s ({rate / fp64_rate:.2f}x FP64), "
        f"iterations {[i['iterations'] for i in infos]}, residual {rel_res:.2e}")
    f64s = sum(i["filter_kernel_seconds"] for i in infos) - f32s
    f64f = sum(i["filter_flops"] for i in infos) - f32f
    phase = {k: sum(i[k] for i in infos) / len(infos)
             for k in ("t_reduce", "t_lanczos", "t_filter", "t_qr", "t_rr", "t_resid", "t_total")}
    return {"evals": ev, "solves_per_s": rate, "speedup_vs_fp64": rate / fp64_rate, "ms_per_step": 1e3 * elapsed / steps,
            "steps": steps, "warmup": warmup,
            "iterations": [i["iterations"] for i in infos], "iterations_fp32": [i["iterations_fp32"] for i in infos],
            "max_rel_residual": rel_res, "filter_tflops_fp32": f32f / f32s / 1e12 if f32s else None,
            "filter_flops_fp32": f32f, "filter_event_seconds_fp32": f32s,
            "filter_launches_fp32": sum(i["filter_launches_fp32"] for i in infos),
            "filter_tflops_fp64_part": f64f / f64s / 1e12 if f64s > 0 else None,
            "filter_flops_fp32_share": f32f / max(1.0, sum(i["filter_flops"] for i in infos)),
            "low_precision_roofline": low_precision_roofline(precision, f32f, f32s),
            "phase_seconds_per_solve": phase}


def low_precision_roofline(precision, flops, seconds):
    """Roofline of a mixed form's lower-precision filter steps against the
    matrix peak of their operand type: FP32 (157.3 TFLOP/s dense) for
    precision 1 and 2, FP16 (2500 TFLOP/s dense) for precision 3."""
    peak, operands = (2500.0, "fp16") if precision == 3 else (157.3, "fp32")
    achieved = flops / seconds / 1e12 if seconds else None
    note = ("8 real flops per complex multiply-add; the FP16 steps execute all 8 (four real products)"
            if precision == 3 else FLOP_COUNT_NOTE)
    return {"bound": "mfma", "operands": operands, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak if achieved else None, "flop_count": note}


def _eig_report(lam_exact, ev64, others, anorm):
    """Per-eigenpair errors (3 significant digits) relative to ||A||_2: FP64
    and each mixed form (others: name -> eigenvalues) against the constructed
    spectrum, each mixed form against FP64."""
    import numpy as np
    ex = np.sort(np.asarray(lam_exact))[:len(ev64)]

    def vec(d):
        return [float(f"{x:.3g}") for x in np.asarray(d)]

    d64 = np.abs(np.asarray(ev64) - ex) / anorm
    out = {"norm": "|dlambda_i| / ||A||_2, i = 1..nev ascending", "max": {"fp64_vs_exact": float(d64.max())},
           "fp64_vs_exact": vec(d64)}
    for name, ev in others.items():
        dx = np.abs(np.asarray(ev) - ex) / anorm
        df = np.abs(np.asarray(ev) - np.asarray(ev64)) / anorm
        out["max"][f"{name}_vs_exact"] = float(dx.max())
        out["max"][f"{name}_vs_fp64"] = float(df.max())
        out[f"{name}_vs_exact"] = vec(dx)
        out[f"{name}_vs_fp64"] = vec(df)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD,
                    choices=sorted(WORKLOADS) + ["precision", "batch", "serve", "warmcold"])
    ap.add_argument("--members", type=int, default=16, help="sequences (batch / serve forms)")
    ap.add_argument("--seq-steps", type=int, default=3, help="problems per sequence (batch / serve / warmcold)")
    ap.add_argument("--rate", type=float, default=None,
                    help="Poisson arrival rate per second (serve form; default 3 for the small law, 0.05 for the full)")
    ap.add_argument("--law", choices=["small", "full"], default="small",
                    help="serve form: the scaled-down law or the serving configuration's law (bounded trace)")
    ap.add_argument("--requests", type=int, default=16, help="serve form, full law: arrivals of the trace served")
    ap.add_argument("--serve-paths", choices=["both", "plain", "server"], default="both",
                    help="serve form: run both paths or one of them on the trace")
    ap.add_argument("--workers", type=int, default=4, help="serving workers")
    ap.add_argument("--batch-precision", type=int, choices=[1, 2], default=2,
                    help="batch form: the filter of both passes (1: FP32 with FP64 final sweeps, 2: FP32 on the Ritz residual)")
    ap.add_argument("--serve-precision", type=int, choices=[1, 2, 3], default=3,
                    help="serve form: the server's filter (1: FP32 with FP64 final sweeps, 2: FP32 on the Ritz residual, "
                         "3: FP16 operands on the Ritz residual)")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serving device-memory budget")
    ap.add_argument("--wc-n", type=int, default=4000, help="problem size of the warm/cold study")
    ap.add_argument("--gen-rng", choices=["host", "device"], default="host",
                    help="where the batch form's sequences draw their Gaussian matrices (device: faster at scale)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="do not time filter launches with events")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision pass over the same problems (after the timed region)")
    ap.add_argument("--save-inputs", default=None,
                    help="write the generated problems (H, S, spectrum) to this file and exit")
    ap.add_argument("--load-inputs", default=None, help="read the problems from a --save-inputs file")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, run a device copy of known size (counter calibration)")
    args = ap.parse_args()
    args.rate_set = args.rate is not None
    if args.rate is None:
        args.rate = 3.0
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU (no multi-GPU path); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        sys.exit("need --steps >= 1 and --warmup >= 0")

    import torch
    from paper_1305_5120_amd import chfsi
    chfsi.load()
    forms = {"precision": run_precision, "batch": run_batch, "serve": run_serve, "warmcold": run_warmcold}
    if args.workload in forms:
        forms[args.workload](args)
        return
    dev = torch.device("cuda:0")
    cfg = WORKLOADS[args.workload]
    total = args.warmup + args.steps
    if args.load_inputs:
        # inputs written by an earlier --save-inputs run of this workload
        # (profilers that intercept every launch need not see the generator)
        saved = torch.load(args.load_inputs, map_location=dev, weights_only=True)
        if saved["workload"] != args.workload or (cfg["sequence"] and len(saved["problems"]) < total):
            sys.exit(f"{args.load_inputs} holds other inputs than this run needs")
        probs = [{k: (v.cpu().numpy() if k == "lam" else v.mT.contiguous().mT) for k, v in p.items()}
                 for p in saved["problems"][:total]]
        if not cfg["sequence"]:
            probs = probs[:1] * total  # one problem, solved cold at every step
        log(f"[bench] workload {args.workload}: inputs loaded from {args.load_inputs}")
    else:
        log(f"[bench] workload {args.workload}: generating inputs")
        probs = make_problems(cfg, total, dev)
    torch.cuda.synchronize()
    if args.save_inputs:
        keep = ("H", "S", "lam")
        torch.save({"workload": args.workload,
                    "problems": [{k: (v.cpu() if torch.is_tensor(v) else torch.as_tensor(v)) for k, v in p.items()
                                  if k in keep} for p in (probs if cfg["sequence"] else probs[:1])]},
                   args.save_inputs)
        log(f"[bench] inputs saved to {args.save_inputs}")
        return

    n, nev, nex = cfg["n"], cfg["nev"], cfg["nex"]
    ctx = chfsi.create(n, degree=cfg["degree"], seed=0, profile=0 if args.no_profile else 1)
    S0 = probs[0]["S"]
    infos = []

    def one(i):
        p = probs[i]
        S = S0 if i == 0 else (None if cfg["sequence"] else p["S"])
        if not cfg["sequence"]:
            ctx.reset()  # cold start: the timed work is the whole solve from a random block
        ev, X, info, st = chfsi.solve(ctx, p["H"], S, nev, nex, tol=1e-10)
        return ev, X, info

    for i in range(args.warmup):
        ev, X, info = one(i)
        log(f"[bench] warmup solve {i}: {info['iterations']} iterations, {info['t_total']:.3f} s")
    torch.cuda.synchronize()
    MARKER.push("bench.timed_region")
    t0 = time.perf_counter()
    for i in range(args.warmup, total):
        ev, X, info = one(i)
        infos.append(info)
        log(f"[bench] timed solve {i - args.warmup}: {info['iterations']} iterations, warm={info['warm_start']}, "
            f"{info['t_total']:.3f} s, filter {info['t_filter']:.3f} s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    MARKER.pop()
    elapsed = t1 - t0
    rel_res = residual_check(probs[total - 1], ev, X)
    ev64 = ev
    del X

    flops = sum(i["filter_flops"] for i in infos)
    fsec = sum(i["filter_kernel_seconds"] for i in infos)
    launches = sum(i["filter_launches"] for i in infos)
    achieved = flops / fsec / 1e12 if fsec > 0 else None
    phase = {k: sum(i[k] for i in infos) / len(infos)
             for k in ("t_reduce", "t_lanczos", "t_filter", "t_qr", "t_rr", "t_resid", "t_total")}
    # algorithmic bytes per launch: A once, Y_i and Y_{i-1} read, Y_{i+1}
    # written; 8 n^2 k_a flops per launch give the mean k_a
    mean_ka = (flops / launches) / (8.0 * n * n) if launches else 0.0
    alg_bytes = 16.0 * n * n + 48.0 * n * mean_ka
    busy, core_frac = measured_mfma(args.workload)
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
        "phase_seconds_per_solve": phase,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s",
                     "frac": (achieved / PEAK_FP64_MFMA) if achieved else None,
                     "flop_count": FLOP_COUNT_NOTE,
                     "matrix_core_frac_from_flops": (GAUSS3_SHARE * achieved / PEAK_FP64_MFMA) if achieved else None,
                     "matrix_core_busy_counter": busy,
                     "matrix_core_flop_frac_counter": core_frac,
                     "traffic": measured_traffic(args.workload),
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "algorithmic_flops_per_launch": flops / launches if launches else None},
    }
    if not args.no_mixed:
        mixed = run_mixed_same_workload(args, cfg, probs, out["value"], precision=1)
        ev_mixed = mixed.pop("evals")
        out["mixed_precision"] = mixed
        ritz = run_mixed_same_workload(args, cfg, probs, out["value"], precision=2)
        ev_ritz = ritz.pop("evals")
        out["mixed_precision_ritz"] = ritz
        ritz16 = run_mixed_same_workload(args, cfg, probs, out["value"], precision=3)
        ev_ritz16 = ritz16.pop("evals")
        out["mixed_precision_ritz_fp16"] = ritz16
        if not cfg["sequence"]:
            anorm = float(abs(probs[0]["lam"]).max())
            out["eigenpair_errors"] = _eig_report(probs[0]["lam"], ev64, {"mixed": ev_mixed, "ritz32": ev_ritz,
                                                                          "ritz16": ev_ritz16}, anorm)
    if args.calibrate_copy:
        calibrate_copy()
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(cfg, flops / len(infos))
    print(json.dumps(out), flush=True)
    ctx.release()


if __name__ == "__main__":
    main()
