#!/usr/bin/env python3
"""Throughput of the fast-FCM mobility on one MI355X.

A step is one fcm_mobility call (sort, spread, FFT Stokes solve, interpolation,
FP64 pair correction) on the dense suspension: N = 100,000 spheres (a = 1) at
volume fraction 10 %, 256^3 grid, Sigma = dx, M_G = 10, R_c = 5.5 Sigma, with
inputs resident in device memory.  The value is particle-mobility evaluations
per second (N / seconds per step) of the FP32-bulk path; the FP64 path, call
latency percentiles, per-stage times, the roofline of the dominant kernel and
the oracle timed on host cores are reported beside it on the same JSON line,
together with the serving leg: a 512-request mixed-size stream replayed with
Poisson arrivals through the one-request-at-a-time FP64 path and through the
continuous-batching FP32-bulk server (p50/p99 latency, throughput).

    python bench.py [--steps K] [--warmup W] [--workload dense|dilute|rods|small|serving]
                    [--no-cpu] [--no-fp64] [--no-serving] [--requests R]
    python bench.py --compare-standard [--compare-al A,..] [--compare-phi P,..]

The second form prints the fast-against-standard FCM comparison of Sec. 5.3 instead
(evaluations/s ratio over volume fraction and a/L, and the crossover fraction).
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {"small": 0, "dilute": 1, "dense": 2, "rods": 3, "serving": None}
HBM_PEAK_GBS = 8000.0
METRIC = "mobility evals/s (N=1e5, ≤1e-4 rel err) FP32 vs FP64; p50/p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="dense", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 path")
    ap.add_argument("--cpu-sample", type=int, default=1000)
    ap.add_argument("--requests", type=int, default=512, help="serving stream length")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-stream leg")
    ap.add_argument("--compare-standard", action="store_true",
                    help="instead of the headline run: particle-mobility evaluations/s of fast FCM "
                         "against standard FCM over volume fraction and a/L (force-only, "
                         "eps = 1e-4 parameters), the crossover fraction phi_c and its fit")
    ap.add_argument("--compare-al", default="0.002,0.004,0.008,0.012")
    ap.add_argument("--compare-phi", default="0.005,0.01,0.02,0.04,0.08,0.12,0.16,0.20,0.25,0.30")
    ap.add_argument("--compare-steps", type=int, default=10)
    ap.add_argument("--calibrate", action="store_true",
                    help="instead of the headline run: the library's error calibration "
                         "(Tables 1-2 of Sec. 5.1) on the FP64 path at N = 64457, phi = 8 %%, a/L = 1/150")
    ap.add_argument("--tune-sigma", action="store_true",
                    help="instead of the headline run: evaluations/s against Sigma/sigma at "
                         "a/L = 1/400 for the volume fractions of Table 3 (its optimum on this GPU)")
    ap.add_argument("--paper-grids", action="store_true",
                    help="call times on the grids of the paper's Sec. 6.3 runs (512x512x8, 256x256x16)")
    ap.add_argument("--serving-grids", action="store_true",
                    help="call and stage times (FP32 bulk) of the serving stream's largest "
                         "request on each grid of 216^3 and above")
    ap.add_argument("--brownian", action="store_true",
                    help="instead of the headline run: time fcm_brownian on the workload (FP32 bulk "
                         "and FP64, Lanczos tolerance 1e-6)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="before timing, copy a field-sized device buffer 3 times (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# FP32 grids whose x and y passes run as one kernel per (component, z) plane:
# the x stage times the fused pass and the y stage is empty
FUSED_XY_GRIDS = (64, 96, 128, 192, 256)


def algorithmic_bytes(w, stage):
    """Bytes one launch of `stage` must move (FP32 bulk): a field is 3 M^3 floats."""
    M, N = w["grid"], w["N"]
    field = 12 * M ** 3
    rec = 48 * N                   # s[3], f[3], F[3], T[3] at 4 bytes
    y = None if M in FUSED_XY_GRIDS else 2 * field
    return {"spread": field + rec, "fft_x_fwd": 2 * field, "fft_y_fwd": y,
            "fft_z_solve": 2 * field, "fft_y_inv": y, "fft_x_inv": 2 * field,
            "interp": field + rec + 48 * N}.get(stage)


KERNEL_OF_STAGE = {"spread": "k_spread", "fft_x_fwd": "k_fft_x_r2c_reg", "fft_y_fwd": "k_fft_y_reg",
                   "fft_z_solve": "k_fft_z_solve_reg", "fft_y_inv": "k_fft_y_reg",
                   "fft_x_inv": "k_fft_x_c2r_reg", "interp": "k_interp8", "pair": "k_pair_eval",
                   "sort": "k_hash"}


def kernel_of_stage(stage, w):
    if w["grid"] in FUSED_XY_GRIDS and stage in ("fft_x_fwd", "fft_x_inv"):
        return "k_fft_xy_r2c" if stage == "fft_x_fwd" else "k_fft_xy_c2r"
    return KERNEL_OF_STAGE[stage]
SOURCE_OF_STAGE = {"spread": "fcm_grid.hip", "interp": "fcm_grid.hip", "pair": "fcm_pair.hip",
                   "sort": "fcm_sort.hip"}


def traffic_for(stage, workload):
    """HBM bytes per launch from the committed counter summary of this kernel and
    workload, or None when absent or taken on a different kernel source."""
    src = SOURCE_OF_STAGE.get(stage, "fcm_fft.hip")
    path = os.path.join(ROOT, "profiles", f"traffic_{stage}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    h = hashlib.sha256(open(os.path.join(ROOT, "paper_2310_12651_amd", "csrc", src), "rb").read()).hexdigest()
    if vals.get("kernel_source_sha256") != h:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def valu_for(stage, workload):
    """VALU wave instructions per launch from the committed counter summary of
    this kernel and workload, or None when absent or taken on another source."""
    path = os.path.join(ROOT, "profiles", f"valu_{stage}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = SOURCE_OF_STAGE.get(stage, "fcm_fft.hip")
    h = hashlib.sha256(open(os.path.join(ROOT, "paper_2310_12651_amd", "csrc", src), "rb").read()).hexdigest()
    if vals.get("kernel_source_sha256") != h:
        return None
    try:
        return float(vals["sq_insts_valu_per_dispatch"])
    except (KeyError, ValueError):
        return None


def time_path(plan, args, Y, F, T, V, W, torch, candidates):
    """Warm up; a short pass with every stage timed gives the stage breakdown
    and the dominant stage among `candidates`; then exactly args.steps calls are
    timed with events around that stage only (two per call instead of twelve,
    which would add their gaps to the call) and one per-call event for latency."""
    st = torch.cuda.current_stream()
    for _ in range(args.warmup):
        plan.mobility(Y, F, T, V, W)
    torch.cuda.synchronize()
    plan.set_timing(True)
    for _ in range(max(3, min(args.steps, 10))):
        plan.mobility(Y, F, T, V, W)
    stages, ncalls = plan.stage_times()
    stages = {k: v / max(ncalls, 1) for k, v in stages.items()}
    dom = max(candidates, key=stages.get)
    plan.set_timing(True, stage=dom)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(st)
    for k in range(args.steps):
        plan.mobility(Y, F, T, V, W)
        evs[k + 1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = sorted(evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps))
    total_ms = evs[0].elapsed_time(evs[-1])
    timed, ncalls = plan.stage_times()
    plan.set_timing(False)
    q = lambda p: lat[min(len(lat) - 1, int(math.ceil(p * len(lat))) - 1)]
    return dict(ms_per_step=total_ms / args.steps, wall_s=wall, p50_ms=q(0.50), p99_ms=q(0.99),
                stages_ms=stages, dom_stage=dom, dom_ms=timed[dom] / max(ncalls, 1))


def cpu_baseline(w, n_sample, V_gpu, W_gpu):
    """The oracle (plain FP64 numpy) on a bounded sample of the same workload:
    spreading of all N particles and the full FFT solve are timed as they are;
    interpolation and pair correction are timed on a seeded subsample and scaled
    to N.  Also returns the GPU error against the oracle on the subsample."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import fastfcm as ff
    threadpool_limits(1)
    p = ff.Params(L=w["L"], M=w["grid"], a=w["a"], Sigma=w["Sigma"], M_G=w["M_G"], R_c=w["R_c"])
    N = w["N"]
    rng = np.random.default_rng(12345)
    sub = np.sort(rng.choice(N, size=min(n_sample, N), replace=False))
    t0 = time.perf_counter()
    f = ff.spread(p, w["Y"], w["F"], w["T"])
    t1 = time.perf_counter()
    u = ff.stokes_solve(p, f)
    t2 = time.perf_counter()
    V, W = ff.interp(p, w["Y"][sub], u)
    t3 = time.perf_counter()
    dV, dW = ff.pair_correction(p, w["Y"], w["F"], w["T"], targets=sub)
    t4 = time.perf_counter()
    scale = N / len(sub)
    est = (t1 - t0) + (t2 - t1) + scale * ((t3 - t2) + (t4 - t3))
    Vo, Wo = V + dV, W + dW
    err = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    epsm = lambda a, b: float(np.mean(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))
    acc = dict(relV=err(V_gpu[sub], Vo), relW=err(W_gpu[sub], Wo), epsV=epsm(V_gpu[sub], Vo),
               epsW=epsm(W_gpu[sub], Wo), n=len(sub))
    base = dict(value=N / est, unit="evals/s", cores=1, kind="oracle",
                sample=(f"numpy FP64 oracle, single thread: spread of all {N} particles "
                        f"({t1 - t0:.1f} s) and the {w['grid']}^3 FFT solve ({t2 - t1:.1f} s) timed in "
                        f"full; interpolation ({t3 - t2:.2f} s) and pair correction ({t4 - t3:.2f} s) "
                        f"timed on {len(sub)} seeded particles and scaled by {scale:.0f}"))
    return base, acc


def serving_leg(args, torch):
    """The mixed-size request stream: the one-request-at-a-time FP64 path
    (closed loop, then Poisson arrivals at 0.8x and at 1.5x its throughput)
    against the continuous-batching FP32-bulk server (8 slots) on the same
    arrivals."""
    import numpy as np

    import workloads
    from paper_2310_12651_amd import FCM_FP32_BULK, FCM_FP64
    from paper_2310_12651_amd.serving import Server, replay, run_sequential
    reqs = workloads.serving_stream(args.requests)
    t = time.perf_counter()
    dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    tensors = []
    for r in reqs:
        Y, F, T = workloads.request_inputs(r)
        V = torch.empty((r["N"], 3), dtype=torch.float64, device="cuda")
        tensors.append((dev(Y), dev(F), dev(T), V, torch.empty_like(V)))
    torch.cuda.synchronize()
    total = sum(r["N"] for r in reqs)
    log(f"[bench] serving stream: {len(reqs)} requests, {total} particles, inputs in {time.perf_counter() - t:.1f} s")
    budget = int(0.35 * torch.cuda.mem_get_info()[0])
    pct = lambda lat, p: float(np.percentile(np.asarray(lat), p))

    def warm(server):
        # one request per grid, the largest, so that the cached plans hold every
        # request of the stream (plans are built once and stay resident)
        big = {}
        for i, r in enumerate(reqs):
            if r["grid"] not in big or r["N"] > reqs[big[r["grid"]]]["N"]:
                big[r["grid"]] = i
        for i in big.values():
            run_sequential(server, [reqs[i]], [tensors[i]])

    s64 = Server(slots=1, precision=FCM_FP64, max_bytes=budget)
    warm(s64)
    _, T_seq = run_sequential(s64, reqs, tensors)
    rate = 0.8 * len(reqs) / T_seq
    rng = np.random.default_rng(workloads.SEED_BASE + 5)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(reqs)))
    lat64, mk64 = replay(s64, reqs, tensors, arrivals)
    # and at 1.5x the FP64 path's closed-loop rate, beyond what it can serve
    rate_hi = 1.5 * len(reqs) / T_seq
    arrivals_hi = np.cumsum(np.random.default_rng(workloads.SEED_BASE + 6).exponential(1.0 / rate_hi,
                                                                                       size=len(reqs)))
    lat64h, mk64h = replay(s64, reqs, tensors, arrivals_hi)
    st64 = s64.stats()
    s64.close()
    log(f"[bench] fp64 one-at-a-time: closed loop {T_seq:.2f} s; Poisson at {rate:.1f}/s: p50 "
        f"{pct(lat64, 50):.2f} ms p99 {pct(lat64, 99):.2f} ms makespan {mk64:.2f} s")
    # the grid work in flight stays within 1.2 of the stream's largest grid, so
    # that the largest requests run with little company
    max_points = int(1.2 * max(r["grid"] ** 3 for r in reqs))
    s32 = Server(slots=8, precision=FCM_FP32_BULK, max_bytes=budget, max_points=max_points)
    warm(s32)
    lat32, mk32 = replay(s32, reqs, tensors, arrivals)
    lat32h, mk32h = replay(s32, reqs, tensors, arrivals_hi)
    _, T32 = replay(s32, reqs, tensors, None)
    st32 = s32.stats()
    s32.close()
    log(f"[bench] fp32 server: p50 {pct(lat32, 50):.2f} ms p99 {pct(lat32, 99):.2f} ms makespan "
        f"{mk32:.2f} s; closed loop {T32:.2f} s")
    log(f"[bench] at {rate_hi:.1f}/s: fp64 p50 {pct(lat64h, 50):.2f} p99 {pct(lat64h, 99):.2f} ms makespan "
        f"{mk64h:.2f} s; fp32 server p50 {pct(lat32h, 50):.2f} p99 {pct(lat32h, 99):.2f} ms makespan {mk32h:.2f} s")
    return {
        "requests": len(reqs), "particles": total, "arrival_rate_per_s": rate,
        "fp64_one_at_a_time": {"p50_ms": pct(lat64, 50), "p99_ms": pct(lat64, 99),
                               "throughput_evals_per_s": total / mk64,
                               "closed_loop_evals_per_s": total / T_seq,
                               "plans_built": st64["plans_built"], "plans_rebound": st64["plans_rebound"]},
        "fp32_server_8_slots": {"max_points": max_points, "p50_ms": pct(lat32, 50), "p99_ms": pct(lat32, 99),
                                "throughput_evals_per_s": total / mk32,
                                "closed_loop_evals_per_s": total / T32,
                                "inflight_peak": st32["inflight_peak"], "plans_built": st32["plans_built"],
                                "plans_rebound": st32["plans_rebound"],
                                "plans_evicted": st32["plans_evicted"]},
        "above_fp64_saturation": {
            "arrival_rate_per_s": rate_hi,
            "fp64_one_at_a_time": {"p50_ms": pct(lat64h, 50), "p99_ms": pct(lat64h, 99),
                                   "throughput_evals_per_s": total / mk64h},
            "fp32_server_8_slots": {"p50_ms": pct(lat32h, 50), "p99_ms": pct(lat32h, 99),
                                    "throughput_evals_per_s": total / mk32h}},
    }


# Optimal Sigma/sigma of the paper's Table 3 (eps = 1e-4, a/L = 1/400, RTX 2080 Ti):
# the centre of the Sigma sweep of the comparison, which then picks the fastest
# Sigma on this GPU (the paper tunes Sigma per device the same way, Sec. 5.2).
T3_PHI = (0.0005, 0.002, 0.008, 0.032, 0.128)
T3_RATIO = (5.9, 5.1, 3.4, 1.8, 1.4)
SWEEP = (0.7, 0.85, 1.0, 1.2, 1.45)


def compare_standard(args, torch):
    """Fast FCM against standard FCM (Sec. 5.3): for each a/L and volume
    fraction phi, the evaluations/s (PTPS) of fast FCM at the fastest Sigma of a
    sweep around the Table-3 optimum (Sigma/dx = 1, M_G = 10, R_c = 5.5 Sigma,
    the eps = 1e-4 parameters of Tables 1-2) and of standard FCM (Sigma = sigma,
    Sigma_D = sigma_D, no pair correction, grid the smallest even 2^p 3^q with
    dx <= sigma, M_G = 10), both FP32 bulk, force only (the setting of the
    paper's error measure).  Positions: the jittered lattice of the request
    stream; F ~ N(0, 1).  phi_c is where the PTPS ratio crosses 1 (linear
    interpolation in phi), fitted linearly in a/L as in Fig. 3."""
    import numpy as np

    import workloads
    from paper_2310_12651_amd import FCM_FP32_BULK, Plan
    a, sigma = 1.0, 1.0 / math.sqrt(math.pi)
    sigma_D = a / (6.0 * math.sqrt(math.pi)) ** (1.0 / 3.0)
    als = [float(x) for x in args.compare_al.split(",") if x]
    phis = [float(x) for x in args.compare_phi.split(",") if x]

    def ptps(plan, Y, F, V):
        for _ in range(2):
            plan.mobility(Y, F, None, V, None, want_omega=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.compare_steps):
            plan.mobility(Y, F, None, V, None, want_omega=False)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.compare_steps

    rows, crossings = [], {}
    for al in als:
        L = a / al
        ratios = []
        for phi in phis:
            N = int(round(phi * L ** 3 / (4.0 * math.pi * a ** 3 / 3.0)))
            rng = np.random.default_rng(workloads.SEED_BASE + 2000 + int(1e4 * al) + int(1e3 * phi))
            Yh, kind = suspension_positions(N, L, a, phi, rng)
            Fh = rng.normal(size=(N, 3))
            Y = torch.as_tensor(Yh, device="cuda")
            F = torch.as_tensor(Fh, device="cuda")
            V = torch.empty((N, 3), dtype=torch.float64, device="cuda")
            Ms = workloads.smooth_grid(int(math.ceil(L / sigma)))
            std = Plan(N, L, a, sigma, Ms, 0.0, support=10, sigma_D_grid=sigma_D,
                       precision=FCM_FP32_BULK)
            t_std = ptps(std, Y, F, V)
            V_std = V.clone()
            std.close()
            centre = float(np.interp(math.log(phi), np.log(T3_PHI), T3_RATIO))
            best = None
            for fac in SWEEP:
                Sig = max(1.0, centre * fac) * sigma
                M = workloads.smooth_grid(int(math.ceil(L / Sig)))
                Sig = L / M                      # Sigma / dx = 1 on the chosen grid
                if Sig < sigma or 5.5 * Sig >= L / 2:
                    continue
                fp = Plan(N, L, a, Sig, M, 5.5 * Sig, support=10, precision=FCM_FP32_BULK)
                t = ptps(fp, Y, F, V)
                fp.close()
                if best is None or t < best[0]:
                    best = (t, Sig, M, V.clone())
            t_fast, Sig, M, V_fast = best
            dv = torch.linalg.vector_norm(V_fast - V_std, dim=1) / torch.linalg.vector_norm(V_std, dim=1)
            row = dict(a_over_L=al, phi=phi, N=N, L=L, positions=kind,
                       standard=dict(grid=Ms, ms=t_std, ptps=N / (t_std * 1e-3)),
                       fast=dict(grid=M, Sigma_over_sigma=Sig / sigma, R_c=5.5 * Sig, ms=t_fast,
                                 ptps=N / (t_fast * 1e-3)),
                       ratio=t_std / t_fast, eps_fast_vs_standard=float(dv.mean()))
            rows.append(row)
            ratios.append(row["ratio"])
            log(f"[compare] a/L={al} phi={phi} N={N} ({kind}): standard {Ms}^3 {t_std:.3f} ms, fast "
                f"{M}^3 Sigma/sigma={Sig / sigma:.2f} {t_fast:.3f} ms, ratio {row['ratio']:.2f}, "
                f"eps {row['eps_fast_vs_standard']:.2e}")
            del Y, F, V, V_std, V_fast
            torch.cuda.empty_cache()
        pc = None
        for k in range(1, len(phis)):
            if ratios[k - 1] >= 1.0 > ratios[k]:
                f0, f1 = ratios[k - 1], ratios[k]
                pc = phis[k - 1] + (f0 - 1.0) / (f0 - f1) * (phis[k] - phis[k - 1])
                break
        crossings[al] = pc
    fit = None
    pts = [(al, pc) for al, pc in crossings.items() if pc is not None]
    if len(pts) >= 2:
        sl, ic = np.polyfit([p[0] for p in pts], [p[1] for p in pts], 1)
        fit = dict(slope=float(sl), intercept=float(ic))
    return dict(metric="PTPS fast FCM / standard FCM vs volume fraction (eps 1e-4, FP32 bulk)",
                rows=rows, phi_c={str(k): v for k, v in crossings.items()}, phi_c_fit=fit,
                paper_context="RTX 2080 Ti: phi_c ~18% at a/L=0.004, ~10% at 0.012, "
                              "phi_c ~ -9.24 a/L + 0.22")


# random sequential addition, the paper's random suspensions (Sec. 5), is used
# where it converges within seconds on the host: up to 16 % volume fraction and
# 2e5 spheres; denser or larger suspensions use the jittered lattice
RSA_MAX_PHI, RSA_MAX_N = 0.16, 200_000


def suspension_positions(N, L, a, phi, rng):
    """(positions, 'rsa' | 'lattice') of N spheres in the cube of side L."""
    import workloads
    if phi <= RSA_MAX_PHI + 1e-12 and N <= RSA_MAX_N:
        return workloads.rsa_positions(N, L, a, rng), "rsa"
    return workloads.lattice_positions(N, L, a, rng), "lattice"


def calibrate(args, torch):
    """The error calibration of Sec. 5.1 redone for this library (FP64 path,
    force only, eps = mean_n |V_n - U_n| / |U_n|), in the paper's setting: a
    suspension at phi = 8 % in a box with a/L = 1/150 (N = 64457).  U is fast
    FCM with every error far below 1e-8 (Sigma/dx = 1.6, M_G = 24, R_c = 12
    Sigma).  Table 1: eps over Sigma/dx and M_G with all pairs within 12 Sigma
    corrected (Sigma ~ 2 sigma); per tolerance, the smallest Sigma/dx whose
    best error over M_G reaches it, and there the smallest M_G that does.
    Table 2: eps over Sigma/sigma and R_c = lambda Sigma with the grid resolved
    (Sigma/dx = 1.6, M_G = 24) at phi = 4, 8, 16, 32 %; per tolerance the
    smallest lambda (interpolated in log eps) that reaches it, per Sigma and
    the largest over Sigma.  Positions: random sequential addition (the
    paper's random suspensions) up to phi = 16 %, the jittered lattice at 32 %;
    F ~ N(0, 1)."""
    import numpy as np

    import workloads
    from paper_2310_12651_amd import FCM_FP64, Plan
    a, sigma, L = 1.0, 1.0 / math.sqrt(math.pi), 150.0
    tols = (1e-2, 1e-3, 1e-4, 1e-6, 1e-8)
    kinds = {}

    def grid_for(ratio, Sigma0):
        M = workloads.smooth_grid(int(math.ceil(L * ratio / Sigma0 - 1e-9)))
        return M, ratio * L / M

    def velocities(Y, F, N, Sigma, M, MG, R_c):
        plan = Plan(N, L, a, Sigma, M, R_c, support=MG, precision=FCM_FP64)
        V, _ = plan.mobility(Y, F, None, want_omega=False)
        torch.cuda.synchronize()
        plan.close()
        return V.cpu().numpy()

    def eps(V, U):
        return float(np.mean(np.linalg.norm(V - U, axis=1) / np.linalg.norm(U, axis=1)))

    def suspension(phi, seed):
        N = int(round(phi * L ** 3 / (4.0 * math.pi * a ** 3 / 3.0)))
        rng = np.random.default_rng(workloads.SEED_BASE + seed)
        Yh, kind = suspension_positions(N, L, a, phi, rng)
        kinds[phi] = kind
        return N, torch.as_tensor(Yh, device="cuda"), torch.as_tensor(rng.normal(size=(N, 3)), device="cuda")

    def first_below(xs, es, tol):
        """Smallest x reaching tol, interpolated in log eps between neighbours."""
        for k, (x, e) in enumerate(zip(xs, es)):
            if e <= tol:
                if k == 0:
                    return x
                x0, e0 = xs[k - 1], es[k - 1]
                t = (math.log(e0) - math.log(tol)) / (math.log(e0) - math.log(e))
                return x0 + t * (x - x0)
        return None

    # Table 1
    N, Y, F = suspension(0.08, 3000)
    M, S = grid_for(1.6, 2.0 * sigma)
    U = velocities(Y, F, N, S, M, 24, 12.0 * S)
    ratios = [round(0.6 + 0.05 * k, 2) for k in range(21)]
    mgs = list(range(6, 21))
    t1 = {}
    for r in ratios:
        M, S = grid_for(r, 2.0 * sigma)
        for MG in mgs:
            if MG <= M:
                t1[(r, MG)] = eps(velocities(Y, F, N, S, M, MG, 12.0 * S), U)
        log(f"[calibrate] table 1: Sigma/dx={r} grid {M}: " +
            " ".join(f"{MG}:{t1[(r, MG)]:.1e}" for MG in mgs if (r, MG) in t1))
    table1 = []
    for tol in tols:
        floor = [min(t1[(r, MG)] for MG in mgs if (r, MG) in t1) for r in ratios]
        r = next((r for r, f in zip(ratios, floor) if f <= tol), None)
        mg = None if r is None else next(MG for MG in mgs if (r, MG) in t1 and t1[(r, MG)] <= tol)
        table1.append(dict(eps=tol, Sigma_over_dx=r, M_G=mg,
                           Sigma_over_dx_interpolated=first_below(ratios, floor, tol)))
    # Table 2
    lams = [2.0 + 0.5 * k for k in range(17)]
    sfacs = (1.5, 2.0, 3.0, 4.0, 5.0, 6.0)
    table2 = {}
    for phi in (0.04, 0.08, 0.16, 0.32):
        N, Y, F = suspension(phi, 3100 + int(100 * phi))
        M, S = grid_for(1.6, 1.5 * sigma)
        U = velocities(Y, F, N, S, M, 24, 12.0 * S)
        per = {}
        for sf in sfacs:
            M, S = grid_for(1.6, sf * sigma)
            es = [eps(velocities(Y, F, N, S, M, 24, lam * S), U) for lam in lams]
            per[sf] = es
            log(f"[calibrate] table 2: phi={phi} Sigma/sigma={S / sigma:.2f} grid {M}: " +
                " ".join(f"{lam:g}:{e:.1e}" for lam, e in zip(lams, es)))
        rows = []
        for tol in tols:
            each = {str(sf): first_below(lams, per[sf], tol) for sf in sfacs}
            vals = [v for v in each.values() if v is not None]
            rows.append(dict(eps=tol, lambda_max=max(vals) if len(vals) == len(sfacs) else None,
                             per_Sigma=each))
        table2[str(phi)] = dict(N=N, positions=kinds[phi], rows=rows)
    return dict(metric="error calibration of the FP64 path (Tables 1-2 of Sec. 5.1)",
                table1_positions=kinds.get(0.08), table1=table1, table1_eps={f"{r},{mg}": e for (r, mg), e in t1.items()},
                table2=table2,
                paper_context=dict(table1=[[1e-2, 0.71, 8], [1e-3, 0.87, 9], [1e-4, 0.99, 10],
                                           [1e-6, 1.20, 12], [1e-8, 1.39, 14]],
                                   table2_phi8=[[1e-2, 2.47], [1e-3, 3.66], [1e-4, 5.08],
                                                [1e-6, 7.18], [1e-8, 8.57]]))


def tune_sigma(args, torch):
    """Fig. 2 / Table 3 of Sec. 5.2 on this GPU: for a/L = 1/400 and the volume
    fractions of Table 3, the evaluations/s (PTPS) of fast FCM (FP32 bulk,
    force only) at eps = 1e-4 parameters (Sigma/dx = 1, M_G = 10, R_c = 5.5
    Sigma) over Sigma/sigma, and the Sigma/sigma of the peak.  Grid: the
    smallest even 2^p 3^q with dx <= Sigma (Sigma is then L / grid).
    Positions: the jittered lattice; F ~ N(0, 1); 10 timed calls after 2."""
    import numpy as np

    import workloads
    from paper_2310_12651_amd import FCM_FP32_BULK, Plan
    a, sigma, L = 1.0, 1.0 / math.sqrt(math.pi), 400.0
    facs = (1.0, 1.2, 1.4, 1.6, 1.8, 2.0, 2.3, 2.6, 3.0, 3.5, 4.0, 4.5, 5.0, 6.0, 7.0, 8.0)
    out = []
    for phi in (0.0005, 0.002, 0.008, 0.032, 0.128):
        N = int(round(phi * L ** 3 / (4.0 * math.pi * a ** 3 / 3.0)))
        rng = np.random.default_rng(workloads.SEED_BASE + 4000 + int(1e4 * phi))
        Y = torch.as_tensor(workloads.lattice_positions(N, L, a, rng), device="cuda")
        F = torch.as_tensor(rng.normal(size=(N, 3)), device="cuda")
        V = torch.empty((N, 3), dtype=torch.float64, device="cuda")
        pts, seen = [], set()
        for fac in facs:
            M = workloads.smooth_grid(int(math.ceil(L / (fac * sigma) - 1e-9)))
            if M in seen or M > 1024:
                continue
            seen.add(M)
            Sig = L / M
            if Sig < sigma:
                continue
            plan = Plan(N, L, a, Sig, M, 5.5 * Sig, support=10, precision=FCM_FP32_BULK)
            for _ in range(2):
                plan.mobility(Y, F, None, V, None, want_omega=False)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.compare_steps):
                plan.mobility(Y, F, None, V, None, want_omega=False)
            e1.record()
            torch.cuda.synchronize()
            plan.close()
            ms = e0.elapsed_time(e1) / args.compare_steps
            pts.append(dict(Sigma_over_sigma=Sig / sigma, grid=M, ms=ms, ptps=N / (ms * 1e-3)))
            log(f"[tune] phi={phi} N={N} Sigma/sigma={Sig / sigma:.2f} grid {M}: {ms:.3f} ms, "
                f"{N / (ms * 1e-3):.3g} evals/s")
        best = max(pts, key=lambda q: q["ptps"])
        out.append(dict(phi=phi, N=N, points=pts, optimum_Sigma_over_sigma=best["Sigma_over_sigma"],
                        optimum_R_c_over_sigma=5.5 * best["Sigma_over_sigma"], peak_ptps=best["ptps"]))
        del Y, F, V
        torch.cuda.empty_cache()
    return dict(metric="PTPS against Sigma/sigma at a/L = 1/400 (Fig. 2, Table 3), FP32 bulk",
                rows=out, paper_context="RTX 2080 Ti: optimum Sigma/sigma 5.9, 5.1, 3.4, 1.8, 1.4 "
                                        "for phi 0.05, 0.2, 0.8, 3.2, 12.8 %; peak ~7e6 PTPS")


def paper_grids(args, torch):
    """Call times of the mobility on the grids of the paper's Sec. 6.3
    scaling runs (Fig. 8), as the number of bodies grows at a fixed domain:
    planar rod suspensions in a 3840a x 3840a x 60a box on 512 x 512 x 8
    points (dx = 7.5a, Sigma = dx, M_G = 10, so the support wraps once around
    z), and tethered filaments in 5760a x 5760a x 360a on 256 x 256 x 16
    points (dx = 22.5a, Sigma = dx, M_G = 10).  R_c = 6 Sigma as in the paper
    for the filaments; for the rods it is held below half the 60a height
    (29.9a = 3.99 Sigma), since the pair correction takes one image per pair.
    Rods: 22 spheres each (touching spheres of spacing 2a stand in for the
    paper's doublets); filaments: 20 segments of spacing 2.2a.  F, T ~ N(0, 1)."""
    import numpy as np

    import workloads
    from paper_2310_12651_amd import FCM_FP32_BULK, FCM_FP64, Plan
    rng = np.random.default_rng(workloads.SEED_BASE + 7)
    dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    out = {"rods_512x512x8": [], "filaments_256x256x16": []}
    cases = [("rods_512x512x8", n, (3840.0, 3840.0, 60.0), (512, 512, 8), 29.9) for n in (576, 2304, 7744)]
    cases += [("filaments_256x256x16", n, (5760.0, 5760.0, 360.0), (256, 256, 16), 6 * 22.5)
              for n in (100, 400, 1600, 6400)]
    for key, nb, L, grid, rc in cases:
        if key.startswith("rods"):
            Y = workloads.rod_monolayer(nb, 22, L[0], 0.5 * L[2], 1.0, rng)
        else:
            Y = workloads.filament_array(nb, 20, L[0], 2.2, 1.0, rng)
        N = len(Y)
        F, T = rng.normal(size=(N, 3)), rng.normal(size=(N, 3))
        Yd, Fd, Td = dev(Y), dev(F), dev(T)
        V = torch.empty((N, 3), dtype=torch.float64, device="cuda")
        W = torch.empty_like(V)
        row = {"bodies": nb, "N": N}
        for name, prec in (("fp32", FCM_FP32_BULK), ("fp64", FCM_FP64)):
            plan = Plan(N, L, 1.0, L[0] / grid[0], grid, rc, support=10, precision=prec)
            for _ in range(3):
                plan.mobility(Yd, Fd, Td, V, W)
            plan.set_timing(True)
            for _ in range(5):
                plan.mobility(Yd, Fd, Td, V, W)
            stages, nc = plan.stage_times()
            plan.set_timing(False)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                plan.mobility(Yd, Fd, Td, V, W)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            row[name] = {"ms_per_call": round(ms, 4), "evals_per_s": N / (ms * 1e-3),
                         "stages_ms": {k: round(v / max(nc, 1), 4) for k, v in stages.items()}}
            plan.close()
        log(f"[bench] {key} bodies={nb} N={N}: fp32 {row['fp32']['ms_per_call']:.3f} ms, "
            f"fp64 {row['fp64']['ms_per_call']:.3f} ms")
        out[key].append(row)
    return out


def serving_grids(args, torch):
    """Call and per-stage times (FP32 bulk, one plan, warm) of the largest
    request of the 512-request serving stream on each grid of 216^3 and above
    (M_G = 16, Sigma from Table 3, R_c = 5.5 Sigma): the requests that set the
    stream's p99."""
    import workloads
    from paper_2310_12651_amd import FCM_FP32_BULK, Plan
    reqs = workloads.serving_stream(512)
    big = {}
    for r in reqs:
        if r["grid"] >= 216 and (r["grid"] not in big or r["N"] > big[r["grid"]]["N"]):
            big[r["grid"]] = r
    dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    out = []
    for g in sorted(big):
        r = big[g]
        Y, F, T = (dev(x) for x in workloads.request_inputs(r))
        V = torch.empty((r["N"], 3), dtype=torch.float64, device="cuda")
        W = torch.empty_like(V)
        plan = Plan(r["N"], r["L"], r["a"], r["Sigma"], g, r["R_c"], support=r["M_G"], precision=FCM_FP32_BULK)
        for _ in range(3):
            plan.mobility(Y, F, T, V, W)
        plan.set_timing(True)
        for _ in range(5):
            plan.mobility(Y, F, T, V, W)
        stages, nc = plan.stage_times()
        plan.set_timing(False)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            plan.mobility(Y, F, T, V, W)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        out.append({"grid": g, "request": r["id"], "N": r["N"], "phi": round(r["phi"], 4),
                    "ms_per_call": round(ms, 4),
                    "stages_ms": {k: round(v / max(nc, 1), 4) for k, v in stages.items()}})
        log(f"[bench] serving grid {g}^3 request {r['id']} N={r['N']}: {ms:.3f} ms")
        plan.close()
    return {"serving_grids": out}


def brownian_leg(args, torch):
    """Brownian velocities (fcm_brownian) on the workload: ms per call for FP32
    bulk and FP64 with seeded noise (grid noise in the grid precision), the
    Lanczos steps to a relative change of 1e-6, and the deterministic part's
    ms per call beside it for scale."""
    import numpy as np

    import workloads
    from paper_2310_12651_amd import FCM_FP32_BULK, FCM_FP64, Plan
    w = workloads.workload(WORKLOADS[args.workload])
    N, M = w["N"], w["grid"]
    Y = torch.as_tensor(w["Y"], device="cuda")
    rng = np.random.default_rng(workloads.SEED_BASE + 7)
    xp = torch.as_tensor(rng.normal(size=(N, 3)), device="cuda")
    out = {}
    for name, prec in (("fp32", FCM_FP32_BULK), ("fp64", FCM_FP64)):
        plan = Plan(N, w["L"], w["a"], w["Sigma"], M, w["R_c"], support=w["M_G"], precision=prec)
        xg = torch.randn((3, M, M, M), dtype=plan.grid_dtype, device="cuda",
                         generator=torch.Generator(device="cuda").manual_seed(11))
        V = torch.empty((N, 3), dtype=torch.float64, device="cuda")
        for _ in range(2):
            _, it = plan.brownian(Y, xg, xp, 1.0, tol=1e-6, V=V)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, it = plan.brownian(Y, xg, xp, 1.0, tol=1e-6, V=V)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        F = torch.as_tensor(w["F"], device="cuda")
        plan.mobility(Y, F, None, V, None, want_omega=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.mobility(Y, F, None, V, None, want_omega=False)
        torch.cuda.synchronize()
        ms_det = (time.perf_counter() - t0) * 1e3 / args.steps
        plan.close()
        out[name] = dict(ms_per_call=ms, lanczos_steps=it, evals_per_s=N / (ms * 1e-3),
                         deterministic_force_only_ms=ms_det)
        log(f"[brownian] {name}: {ms:.3f} ms per call, {it} Lanczos steps; force-only mobility {ms_det:.3f} ms")
    return dict(metric="Brownian velocities per call (fcm_brownian), wall clock", workload=w["name"],
                steps=args.steps, **out)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the fast-FCM path here runs on a single device "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads
    from paper_2310_12651_amd import FCM_FP32_BULK, FCM_FP64, STAGES, Plan

    if args.brownian:
        print(json.dumps(brownian_leg(args, torch)), flush=True)
        return
    if args.paper_grids:
        print(json.dumps(paper_grids(args, torch)), flush=True)
        return
    if args.serving_grids:
        print(json.dumps(serving_grids(args, torch)), flush=True)
        return
    if args.tune_sigma:
        print(json.dumps(tune_sigma(args, torch)), flush=True)
        return
    if args.calibrate:
        print(json.dumps(calibrate(args, torch)), flush=True)
        return
    if args.compare_standard:
        print(json.dumps(compare_standard(args, torch)), flush=True)
        return
    if args.workload == "serving":
        print(json.dumps({"metric": "serving stream p50/p99 latency and throughput", "serving":
                          serving_leg(args, torch)}), flush=True)
        return
    wid = WORKLOADS[args.workload]
    t = time.perf_counter()
    w = workloads.workload(wid)
    log(f"[bench] workload {w['name']} drawn in {time.perf_counter() - t:.1f} s")
    dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    Y, F, T = dev(w["Y"]), dev(w["F"]), dev(w["T"])
    N = w["N"]
    V = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    W = torch.empty_like(V)
    mk = lambda prec, kahan=0: Plan(N, w["L"], w["a"], w["Sigma"], w["grid"], w["R_c"], support=w["M_G"],
                                    precision=prec, kahan=kahan)
    if args.copy_calib:
        src = torch.ones(3 * w["grid"] ** 3, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 copies of {src.numel() * 4} bytes")
        del src, dst
    plan32 = mk(FCM_FP32_BULK)
    grid_stages = [s for s in STAGES if algorithmic_bytes(w, s)]
    r32 = time_path(plan32, args, Y, F, T, V, W, torch, grid_stages)
    # the same positions again with the last call's sort, records and pair
    # lists (fcm_mobility_repeat), as in repeated solves at one configuration
    plan32.mobility(Y, F, T, V, W)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan32.mobility_repeat(F, T, V, W)
    e1.record()
    torch.cuda.synchronize()
    repeat_ms = e0.elapsed_time(e1) / args.steps
    log(f"[bench] fp32 repeat at the same positions {repeat_ms:.3f} ms/step")
    log(f"[bench] fp32 {r32['ms_per_step']:.3f} ms/step  stages {r32['stages_ms']}")
    V32, W32 = V.cpu().numpy(), W.cpu().numpy()
    plan32.close()
    # the same FP32 path with Kahan-compensated sums in the spreading tiles
    plan_k = mk(FCM_FP32_BULK, kahan=1)
    rk = time_path(plan_k, args, Y, F, T, V, W, torch, grid_stages)
    plan_k.close()
    Vk, Wk = V.cpu().numpy(), W.cpu().numpy()
    log(f"[bench] fp32 kahan {rk['ms_per_step']:.3f} ms/step  spread {rk['stages_ms']['spread']:.4f} ms")
    r64 = None
    acc64 = None
    if not args.no_fp64:
        plan64 = mk(FCM_FP64)
        r64 = time_path(plan64, args, Y, F, T, V, W, torch, grid_stages)
        log(f"[bench] fp64 {r64['ms_per_step']:.3f} ms/step  stages {r64['stages_ms']}")
        V64, W64 = V.cpu().numpy(), W.cpu().numpy()
        acc64 = dict(relV_fp32_vs_fp64=float(np.linalg.norm(V32 - V64) / np.linalg.norm(V64)),
                     relW_fp32_vs_fp64=float(np.linalg.norm(W32 - W64) / np.linalg.norm(W64)),
                     relV_fp32_kahan_vs_fp64=float(np.linalg.norm(Vk - V64) / np.linalg.norm(V64)),
                     relW_fp32_kahan_vs_fp64=float(np.linalg.norm(Wk - W64) / np.linalg.norm(W64)))
        plan64.close()
    stages = {k: v for k, v in r32["stages_ms"].items()}
    roof = None
    if grid_stages:
        # the dominant grid kernel's duration, timed live in the timed region
        dom_grid, dom_ms = r32["dom_stage"], r32["dom_ms"]
        ab = algorithmic_bytes(w, dom_grid)
        ach = ab / (dom_ms * 1e-3) / 1e9
        tr = traffic_for(dom_grid, args.workload)
        roof = dict(kernel=kernel_of_stage(dom_grid, w), bound="hbm", achieved=round(ach, 1),
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4),
                    traffic=tr, algorithmic_bytes=ab, launch_ms=round(dom_ms, 5))
        # what actually bounds spread and interpolation: VALU issue (a wave64
        # instruction holds a 16-lane SIMD 4 cycles; 1024 SIMDs at 2.4 GHz),
        # counted once by rocprofv3 and divided by this run's launch time
        nv = valu_for(dom_grid, args.workload)
        if nv is not None:
            roof["valu_issue"] = dict(wave_instructions=nv, simds=1024, clock_ghz=2.4,
                                      frac=round(nv * 4 / (1024 * 2.4e9 * dom_ms * 1e-3), 3))
    per_stage_gbs = {s: round(algorithmic_bytes(w, s) / (stages[s] * 1e-3) / 1e9, 1)
                     for s in grid_stages}
    serving = None
    if not args.no_serving:
        serving = serving_leg(args, torch)
    base, acc = None, None
    if not args.no_cpu:
        log("[bench] timing the oracle on the host (bounded sample)")
        base, acc = cpu_baseline(w, args.cpu_sample, V32, W32)
        log(f"[bench] oracle {base['value']:.3g} evals/s; accuracy {acc}")
    out = {
        "metric": METRIC,
        "value": N / (r32["ms_per_step"] * 1e-3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 grid + f64 pair",
        "data": "synthetic",
        "config": {"workload": w["name"], "N": N, "grid": w["grid"], "Sigma": w["Sigma"],
                   "M_G": w["M_G"], "R_c": w["R_c"], "L": w["L"], "parallelism": "single GPU"},
        "latency_ms": {"p50": r32["p50_ms"], "p99": r32["p99_ms"]},
        "repeat_same_positions": {"ms_per_step": repeat_ms, "value": N / (repeat_ms * 1e-3)},
        "fp32_kahan_spread": {"value": N / (rk["ms_per_step"] * 1e-3), "ms_per_step": rk["ms_per_step"],
                              "spread_ms": round(rk["stages_ms"]["spread"], 5),
                              "spread_ms_plain": round(stages["spread"], 5)},
        "stages_ms": {k: round(v, 5) for k, v in stages.items()},
        "stage_gbs": per_stage_gbs,
        "fp64": None if r64 is None else {"value": N / (r64["ms_per_step"] * 1e-3),
                                           "ms_per_step": r64["ms_per_step"],
                                           "latency_ms": {"p50": r64["p50_ms"], "p99": r64["p99_ms"]},
                                           "stages_ms": {k: round(v, 5) for k, v in r64["stages_ms"].items()}},
        "accuracy": {"vs_oracle_subsample": acc, "fp32_vs_fp64": acc64},
        "roofline": roof,
        "cpu_baseline": base,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
