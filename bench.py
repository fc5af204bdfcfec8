"""Setup + solve time of the algebraic multilevel overlapping Schwarz
preconditioner on one MI355X.

A step = dd_setup (A and the partition already on the GPU) + PCG to a true
relative residual <= 1e-8, device-synchronised on both sides.  The default
workload is the 3-D high-contrast diffusion problem (64^3 grid, n = 262144,
log-normal coefficient sigma = 2 with eight 1e6 channels, 256 subdomains by
seeded greedy graph growing, overlap 2, lambda > 50, two levels).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "setup+solve sec to 1e-8 rel-res: learned/FP32/batched vs plain FP64, 1 MI355X"

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# The kernel whose roofline is reported: the trailing update C -= V_b W of the
# blocked Householder QR (MFMA FP64), the largest single kernel family of the
# setup.  Its HBM traffic per dispatch comes from two rocprofv3 PMC passes
# (FETCH_SIZE, WRITE_SIZE) over this same workload, scaled by what the counters
# read for a plain copy of known size; it is only reported while the kernel
# sources still hash to what was profiled.
ROOFLINE_KERNEL = "qr_blk_upd"
ROOFLINE_SOURCES = ["common.hpp", "dense.hpp", "dense.hip"]
TRAFFIC = {"sha256": "2b8863b42dd6ed06", "bytes_per_launch": 3.1845e9,
           "workload": "diffusion3d_7pt_64^3_lognormal_sigma2_channels1e6"}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", choices=["diffusion3d_64", "poisson2d_64"], default="diffusion3d_64")
    p.add_argument("--form", choices=["fp64", "fp32"], default="fp64")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-compare-forms", action="store_true",
                   help="skip timing the other local-solve precision form (after the timed steps)")
    p.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for the CPU baseline")
    p.add_argument("--achievable", action="store_true",
                   help="only measure the achievable copy bandwidth and FP64/FP32 GEMM rates on this GPU and exit")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only run a plain device copy of 1 GiB three times (PMC byte-counter calibration) and exit")
    return p.parse_args()


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ROOFLINE_SOURCES:
        with open(os.path.join(ROOT, "paper_2109_05908_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def calibrate_copy():
    import torch
    n = (1 << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        t0 = time.perf_counter()
        y.copy_(x)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"[bench] copy 1 GiB -> 1 GiB: {dt * 1e3:.3f} ms, {2 * n * 8 / dt / 1e9:.0f} GB/s", file=sys.stderr,
              flush=True)


def achievable():
    """Achievable rates on this GPU, for the fractions beside the published peaks:
    device-to-device copy of 4 GiB (read + write bytes) and square FP64 / FP32
    matrix products through the vendor BLAS (torch.matmul), timed with events."""
    import torch
    out = {}
    n = (4 << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    y.copy_(x)
    torch.cuda.synchronize()
    reps = 10
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    out["copy_GBs"] = 2 * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    for name, dt, m in (("gemm_fp64_TFs", torch.float64, 8192), ("gemm_fp32_TFs", torch.float32, 8192)):
        a = torch.randn(m, m, dtype=dt, device="cuda:0")
        b = torch.randn(m, m, dtype=dt, device="cuda:0")
        c = a @ b
        torch.cuda.synchronize()
        reps = 5
        e0.record()
        for _ in range(reps):
            c = a @ b
        e1.record()
        torch.cuda.synchronize()
        out[name] = 2.0 * m ** 3 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e12
        del a, b, c
    out.update({"peak_hbm_GBs": 8000.0, "peak_fp64_TFs": 78.6, "peak_fp32_TFs": 157.3})
    print(json.dumps(out), flush=True)


def workload(name):
    import workloads as W
    if name == "poisson2d_64":
        cfg = W.config_c1()
        return cfg, {"workload": "poisson2d_5pt_64x64", "n": cfg.A.n, "subdomains": 16, "partition": "4x4 geometric",
                     "overlap": 1, "lambda_threshold": 10, "tau": cfg.tau, "levels": 2}
    cfg = W.config_c2()
    return cfg, {"workload": "diffusion3d_7pt_64^3_lognormal_sigma2_channels1e6", "n": cfg.A.n, "subdomains": cfg.N,
                 "partition": "seeded greedy graph growing (seed 0)", "overlap": cfg.overlap,
                 "lambda_threshold": round(1 / cfg.tau), "tau": cfg.tau, "levels": cfg.levels}


def cpu_baseline(cfg, part, budget, pre_sizes, its):
    """The oracle (FP64 NumPy/SciPy, as committed) on a bounded sample of the
    same workload, extrapolated to the whole setup + solve.

    Setup: the index sets of all subdomains are computed in full; the local
    setup (extraction, SVD splitting and Schur complement, eigenproblem,
    Cholesky) runs on a size-stratified sample of subdomains and is scaled by
    sum(n_i^3); the coarse Cholesky (dense, as in the oracle) is timed at
    m <= 3000 and scaled by (n_C/m)^3.  Solve: one oracle PCG iteration costs a
    SpMV (timed in full), the sampled local cho_solve calls scaled by
    sum(n_i^2), and a dense coarse cho_solve timed at m and scaled by
    (n_C/m)^2; multiplied by the GPU's iteration count (the oracle's count
    agrees to +-1 in the parity tests)."""
    import numpy as np
    import scipy.linalg as sla

    import oracle as O
    A = O.as_scipy(cfg.A)
    N = cfg.N
    t0 = time.perf_counter()
    sets = O.subdomain_sets(A, part, N, cfg.overlap)
    t_sets = time.perf_counter() - t0
    ni = np.array([s.Omega.size for s in sets], dtype=float)
    order = np.argsort(ni)
    cost3, cost2 = float((ni ** 3).sum()), float((ni ** 2).sum())
    t_loc, t_sol, c3, c2, nsamp = 0.0, 0.0, 0.0, 0.0, 0
    p_sample = []
    stride = max(1, N // 16)
    idx = list(order[::stride]) + list(order[stride // 2::stride])
    rng = np.random.default_rng(0)
    for i in idx:
        if t_loc > budget * 0.6:
            break
        s = sets[i]
        t1 = time.perf_counter()
        Aii, Xi = O.extract(A, s)
        spl = O.local_splitting(Xi, s.I.size, s.Gamma.size)
        _, mk, _ = O.local_eigen(Aii, spl.S_I, s.I.size, cfg.tau)
        ch = sla.cho_factor(Aii, lower=True)
        t_loc += time.perf_counter() - t1
        r = rng.standard_normal(Aii.shape[0])
        t1 = time.perf_counter()
        sla.cho_solve(ch, r)
        t_sol += time.perf_counter() - t1
        nsamp += 1
        c3 += ni[i] ** 3
        c2 += ni[i] ** 2
        p_sample.append(mk.size)
    nC = int(pre_sizes[:, 3].sum()) if pre_sizes is not None else int(np.mean(p_sample) * N)
    m = min(nC, 3000)
    M = rng.standard_normal((m, m))
    M = M @ M.T + m * np.eye(m)
    t1 = time.perf_counter()
    chE = sla.cho_factor(M, lower=True)
    t_cf = time.perf_counter() - t1
    y = rng.standard_normal(m)
    t1 = time.perf_counter()
    for _ in range(5):
        sla.cho_solve(chE, y)
    t_cs = (time.perf_counter() - t1) / 5
    x = rng.standard_normal(A.shape[0])
    t1 = time.perf_counter()
    for _ in range(5):
        A @ x
    t_mv = (time.perf_counter() - t1) / 5
    setup_est = t_sets + t_loc * cost3 / c3 + t_cf * (nC / m) ** 3
    iter_est = t_mv + t_sol * cost2 / c2 + t_cs * (nC / m) ** 2
    est = setup_est + its * iter_est
    used = t_sets + t_loc + t_sol + t_cf + 5 * (t_cs + t_mv)
    threads = os.environ.get("OMP_NUM_THREADS") or str(len(os.sched_getaffinity(0)))
    return {
        "value": est, "unit": "s (setup+solve, extrapolated)", "cores": int(threads), "kind": "oracle",
        "setup_s": setup_est, "solve_s": its * iter_est,
        "sample": (f"index sets of all {N} subdomains ({t_sets:.1f}s); oracle local setup (extraction, SVD "
                   f"splitting + Schur, eigen, Cholesky) on {nsamp} size-stratified subdomains ({t_loc:.1f}s) "
                   f"scaled by sum n_i^3; dense coarse Cholesky at m={m} ({t_cf:.2f}s) scaled to n_C={nC} by "
                   f"(n_C/m)^3; per-iteration SpMV + sampled local cho_solve scaled by sum n_i^2 + coarse "
                   f"cho_solve scaled by (n_C/m)^2, times {its} iterations; {used:.1f}s of CPU work"),
    }


def roofline(met, workload_name):
    """Achieved FP64 MFMA rate of the metered kernel: algorithmic flops per
    dispatch / average event-timed dispatch duration, against the FP64 peak."""
    if met["launches"] == 0 or met["total_ms"] <= 0:
        return None
    avg_ms = met["total_ms"] / met["launches"]
    achieved = met["flops"] / (met["total_ms"] * 1e-3) / 1e12
    traffic = None
    if TRAFFIC and TRAFFIC["sha256"] == source_hash() and TRAFFIC["workload"] == workload_name:
        traffic = TRAFFIC["bytes_per_launch"]
    return {"bound": "mfma", "kernel": "k_tiles<OpBlkUpd> (" + ROOFLINE_KERNEL + ")", "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
            "launches": met["launches"], "avg_launch_ms": avg_ms,
            "flops_per_launch": met["flops"] / met["launches"],
            "algorithmic_bytes_per_launch": met["bytes"] / met["launches"],
            "achieved_algorithmic_GBs": met["bytes"] / (met["total_ms"] * 1e-3) / 1e9,
            "source_sha256": source_hash()}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    from paper_2109_05908_amd import (DD_FP32, DD_FP64, DD_SCHWARZ_ADDITIVE, DD_SCHWARZ_DEFLATED, DeviceCSR,
                                      Preconditioner, meter_read, meter_start, partition_ggg)

    if args.achievable:
        achievable()
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    cfg, conf = workload(args.workload)
    dev = "cuda:0"
    dA = DeviceCSR.from_workload(cfg.A, device=dev)
    if cfg.part is None:
        part = partition_ggg(dA, cfg.N, cfg.ggg_seed)
    else:
        part = torch.as_tensor(cfg.part, device=dev)
    b = torch.as_tensor(W.rhs(cfg.A.n, 0), device=dev)
    prec = DD_FP32 if args.form == "fp32" else DD_FP64
    torch.cuda.synchronize()

    def step(prec=prec, schwarz=DD_SCHWARZ_ADDITIVE):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pre = Preconditioner(dA, part, cfg.N, cfg.overlap, cfg.tau, levels=cfg.levels, local_prec=prec,
                             schwarz=schwarz)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if schwarz == DD_SCHWARZ_DEFLATED:  # the variant of the paper's experiments: GMRES(30)
            x, its, rr, code = pre.gmres(b, rtol=1e-8, maxit=1000, restart=30)
        else:
            x, its, rr, code = pre.pcg(b, rtol=1e-8, maxit=1000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        assert code == 0 and rr[0] <= 1e-8, (code, rr)
        ph = " ".join(f"{k}={v:.0f}" for k, v in pre.info()["phase_ms"].items() if v >= 1.0)
        print(f"[bench]   setup phases (ms): {ph}", file=sys.stderr, flush=True)
        return pre, t1 - t0, t2 - t1, its[0], rr[0]

    for w in range(args.warmup):
        pre, ts, tv, its, rr = step()
        print(f"[bench] warmup {w}: setup {ts:.3f}s solve {tv:.3f}s its {its} relres {rr:.2e}", file=sys.stderr,
              flush=True)
        del pre
    times = []
    last = None
    torch.cuda.synchronize()
    meter_start(ROOFLINE_KERNEL)
    t_all = time.perf_counter()
    for k in range(args.steps):
        pre, ts, tv, its, rr = step()
        times.append((ts, tv, its, rr))
        print(f"[bench] step {k}: setup {ts:.3f}s solve {tv:.3f}s its {its} relres {rr:.2e}", file=sys.stderr,
              flush=True)
        if k < args.steps - 1:
            del pre
        else:
            last = pre
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_all
    met = meter_read()
    meter_start(None)
    info = last.info()
    sizes = last.sizes()
    per = [t[0] + t[1] for t in times]
    value = float(np.median(per))
    conf.update({"local_precision": args.form, "n_C": info["n_C"], "grid_complexity": round(info["grid_complexity"], 4),
                 "pcg_iterations": times[-1][2], "final_relres": times[-1][3],
                 "setup_s_median": float(np.median([t[0] for t in times])),
                 "solve_s_median": float(np.median([t[1] for t in times])),
                 "setup_phase_ms_last": {k: round(v, 1) for k, v in info["phase_ms"].items()}})
    out = {
        "metric": METRIC, "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * wall / args.steps, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.form == "fp64" else "f64 (f32 local solves)",
        "data": "synthetic", "config": conf, "roofline": roofline(met, conf["workload"]),
    }
    forms = {args.form: {"setup_plus_solve_s": value, "pcg_iterations": times[-1][2], "final_relres": times[-1][3]}}
    if not args.no_compare_forms:
        other = "fp32" if args.form == "fp64" else "fp64"
        oprec = DD_FP32 if other == "fp32" else DD_FP64
        del last
        ot = []
        for k in range(1 + args.steps):
            pre, ts, tv, its, rr = step(oprec)
            del pre
            if k > 0:
                ot.append((ts + tv, its, rr))
            print(f"[bench] form {other} step {k}: {ts + tv:.3f}s its {its} relres {rr:.2e}", file=sys.stderr, flush=True)
        forms[other] = {"setup_plus_solve_s": float(np.median([t[0] for t in ot])), "pcg_iterations": ot[-1][1],
                        "final_relres": ot[-1][2]}
        # the deflated variant with the one-level restricted method under
        # right-preconditioned GMRES(30), as in the paper's experiments (same setup)
        ot = []
        for k in range(1 + args.steps):
            pre, ts, tv, its, rr = step(prec, DD_SCHWARZ_DEFLATED)
            del pre
            if k > 0:
                ot.append((ts, tv, its, rr))
            print(f"[bench] form deflated_gmres step {k}: setup {ts:.3f}s solve {tv:.3f}s its {its} relres {rr:.2e}",
                  file=sys.stderr, flush=True)
        forms[f"deflated_gmres_{args.form}"] = {
            "setup_plus_solve_s": float(np.median([t[0] + t[1] for t in ot])),
            "solve_s_median": float(np.median([t[1] for t in ot])), "gmres_iterations": ot[-1][2],
            "final_relres": ot[-1][3]}
    conf["forms"] = forms
    if not args.no_cpu_baseline:
        part_h = part.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(cfg, part_h, args.cpu_budget, sizes, times[-1][2])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
