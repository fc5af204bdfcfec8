"""Setup + solve time of the algebraic multilevel overlapping Schwarz
preconditioner on one MI355X: the learned / FP32 / batched form against the
plain FP64 form.

A step = dd_setup (A and the partition already on the GPU) + PCG to a true
relative residual <= 1e-8, device-synchronised on both sides.  Default
workload: a held-out member (coefficient seed 150) of the 64^3 high-contrast
diffusion family (n = 262144, log-normal coefficient sigma = 2 with eight 1e6
channels, 256 subdomains by seeded greedy graph growing, overlap 2, lambda > 50).
The timed form keeps at most 32 modes per subdomain, solves the local
eigenproblems by LOBPCG from the learned start (network trained on seeds
0..149), keeps FP32 local factors and solves and runs PCG as a replayed
graph; the plain FP64 form (every mode above the threshold, dense eigen
route, FP64, host-driven PCG) is timed beside it.  Prints one JSON line.

--workload batch64_mixed times the many-systems case instead: 64 independent
systems of log-uniform size in [2e4, 5e5] (2-D 5-point, 3-D high-contrast
7-point and 3-D layered elasticity in turn, 9.4M unknowns in all), 32
right-hand sides each, set up and solved in memory waves of batch handles.
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
TRAFFIC = {"sha256": "23bc9c5a8ddd54bb", "bytes_per_launch": 3.9638e9, "form": "learned",
           "workload": "diffusion3d_7pt_64^3_lognormal_sigma2_channels1e6_seed150 (held-out member of the coefficient "
                       "family)"}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", choices=["diffusion3d_64_family150", "diffusion3d_64", "poisson2d_64",
                                          "batch64_mixed"],
                   default="diffusion3d_64_family150")
    p.add_argument("--batch-form", choices=["learned", "plain_fp64", "both"], default="both",
                   help="batch64_mixed: the forms to time")
    p.add_argument("--wave-dofs", type=int, default=500000,
                   help="batch64_mixed: most unknowns set up together in one batch handle")
    p.add_argument("--batch-systems", type=int, default=64, help="batch64_mixed: number of systems")
    p.add_argument("--nrhs", type=int, default=32, help="batch64_mixed: right-hand sides per system")
    p.add_argument("--model", default=os.path.join(ROOT, "paper_2109_05908_amd", "warm_start_c4.json"))
    p.add_argument("--nev", type=int, default=32)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--form", choices=["learned", "plain_fp64"], default="learned",
                   help="form timed as the value (plain_fp64: the reference form alone, for profiling it)")
    p.add_argument("--no-compare-forms", action="store_true",
                   help="skip the plain FP64 and random-start forms (after the timed steps)")
    p.add_argument("--cpu-reps", type=int, default=5, help="runs of the sampled oracle pool (median)")
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
    seed = 150 if name == "diffusion3d_64_family150" else 0
    cfg = W.config_c2(seed=seed)
    wl = ("diffusion3d_7pt_64^3_lognormal_sigma2_channels1e6" if seed == 0 else
          f"diffusion3d_7pt_64^3_lognormal_sigma2_channels1e6_seed{seed} (held-out member of the coefficient family)")
    return cfg, {"workload": wl, "n": cfg.A.n, "subdomains": cfg.N,
                 "partition": "seeded greedy graph growing (seed 0)", "overlap": cfg.overlap,
                 "lambda_threshold": round(1 / cfg.tau), "tau": cfg.tau, "levels": cfg.levels}


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on the host cores (run before the GPU is touched, so
# that its worker processes never start from a process holding GPU state)
# ---------------------------------------------------------------------------
def _blas_threads_one():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
        os.environ[k] = "1"


def _warm_worker(_):
    _blas_threads_one()
    import scipy.linalg  # noqa: F401

    import oracle  # noqa: F401
    return 0


def _oracle_local(args):
    """One subdomain's local setup by the oracle (extraction, SVD splitting and
    Schur complement, eigenproblem (3.3), Cholesky), in a worker process with
    single-threaded BLAS; returns (seconds, kept count, cho_solve seconds)."""
    _blas_threads_one()
    import numpy as np
    import scipy.linalg as sla
    import scipy.sparse as sp

    import oracle as O
    rowptr, colind, val, n, I, G, D, tau = args
    A = sp.csr_matrix((val, colind, rowptr), shape=(n, n))
    s = O.Sets(I, G, D)
    t0 = time.perf_counter()
    Aii, Xi = O.extract(A, s)
    spl = O.local_splitting(Xi, I.size, G.size)
    _, mk, _ = O.local_eigen(Aii, spl.S_I, I.size, tau)
    ch = sla.cho_factor(Aii, lower=True)
    t1 = time.perf_counter()
    r = np.random.default_rng(0).standard_normal(Aii.shape[0])
    t2 = time.perf_counter()
    for _ in range(4):
        sla.cho_solve(ch, r)
    t3 = time.perf_counter()
    return t1 - t0, int(mk.size), (t3 - t2) / 4


def cpu_baseline_host(cfg, part, reps=5, sample=16):
    """The oracle (plain FP64 NumPy/SciPy, unchanged) on the host: the per-
    subdomain setup of a size-stratified sample of subdomains runs in a pool
    of worker processes, one per host core (up to 16), BLAS single-threaded in
    each; the sample's work is scaled by sum n_i^3 to all subdomains and divided
    over the cores (the paper's one-subdomain-per-process layout).  The coarse
    factor is the oracle's dense Cholesky of E (its cost depends on n_C only):
    timed at m = 4000 on all cores and scaled by (n_C / m)^3.  One PCG
    iteration: SpMV, the local solves (sampled cho_solve scaled by sum n_i^2,
    over the cores) and a dense coarse solve (timed at m, scaled by (n_C/m)^2);
    the iteration count comes from the GPU run of the same method.  Median of
    `reps` runs of the sampled pool."""
    import multiprocessing as mp

    import numpy as np
    import scipy.linalg as sla

    import oracle as O
    A = O.as_scipy(cfg.A)
    N = cfg.N
    cores = min(16, len(os.sched_getaffinity(0)))
    t0 = time.perf_counter()
    sets = O.subdomain_sets(A, part, N, cfg.overlap)
    t_sets = time.perf_counter() - t0
    ni = np.array([s.Omega.size for s in sets], dtype=float)
    nI = np.array([s.I.size for s in sets], dtype=float)
    order = np.argsort(ni)
    # the smaller 40 % of the subdomains, evenly spaced in size: a bounded sample (a few seconds per run)
    idx = [int(order[int(round(q))]) for q in np.linspace(0, 0.4 * (N - 1), sample)]
    jobs = [(A.indptr, A.indices, A.data, A.shape[0], sets[i].I, sets[i].Gamma, sets[i].Delta, cfg.tau) for i in idx]
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS",
                                            "BLIS_NUM_THREADS")}
    _blas_threads_one()  # inherited by the spawned workers
    walls, res = [], None
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(cores) as pool:
            pool.map(_warm_worker, range(cores))  # imports in every worker
            for _ in range(reps):
                t1 = time.perf_counter()
                res = pool.map(_oracle_local, jobs)
                walls.append(time.perf_counter() - t1)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    t_loc = np.array([r[0] for r in res])
    p_s = np.array([r[1] for r in res])
    t_cs = np.array([r[2] for r in res])
    c3 = float((ni[idx] ** 3).sum())
    work_setup = float(t_loc.sum()) * float((ni ** 3).sum()) / c3
    setup_local = max(work_setup / cores, float(t_loc.max()))
    nC = int(round(float((p_s / nI[idx]).mean()) * nI.sum()))
    m = 4000
    rng = np.random.default_rng(0)
    M = rng.standard_normal((m, m))
    M = M @ M.T + m * np.eye(m)
    t1 = time.perf_counter()
    chE = sla.cho_factor(M, lower=True)
    t_cf = time.perf_counter() - t1
    y = rng.standard_normal(m)
    t1 = time.perf_counter()
    for _ in range(5):
        sla.cho_solve(chE, y)
    t_csE = (time.perf_counter() - t1) / 5
    x = rng.standard_normal(A.shape[0])
    t1 = time.perf_counter()
    for _ in range(5):
        A @ x
    t_mv = (time.perf_counter() - t1) / 5
    c2 = float((ni[idx] ** 2).sum())
    iter_local = float(t_cs.sum()) * float((ni ** 2).sum()) / c2 / cores
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = "unknown"
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        if info:
            blas = f"{info[0].get('internal_api')} {info[0].get('version')}"
    except Exception:
        pass
    return {
        "cores": cores, "cpu_model": cpu, "blas": blas, "t_sets": t_sets, "setup_local_s": setup_local,
        "coarse_factor_s": t_cf * (nC / m) ** 3, "iter_s": t_mv + iter_local + t_csE * (nC / m) ** 2,
        "nC_est": nC, "sample_wall_median_s": float(np.median(walls)), "sample_walls": walls,
        "sample": (f"oracle local setup (extraction, SVD splitting + Schur, eigenproblem, Cholesky) of {sample} "
                   f"subdomains of {N} evenly spaced in size over the smaller 40 %, pool of {cores} worker processes with single-threaded BLAS, "
                   f"median of {reps} runs ({float(np.median(walls)):.1f}s wall each), scaled by sum n_i^3 and divided "
                   f"over the cores; coarse: dense Cholesky of E as the oracle does it, timed at m={m} on all cores and "
                   f"scaled to n_C={nC} (estimated from the sample's kept modes) by (n_C/m)^3; per PCG iteration: SpMV, "
                   f"sampled local cho_solve scaled by sum n_i^2 over the cores, dense coarse solve scaled by "
                   f"(n_C/m)^2"),
    }


def cpu_baseline_value(host, its):
    setup = host["t_sets"] + host["setup_local_s"] + host["coarse_factor_s"]
    solve = its * host["iter_s"]
    out = {"value": setup + solve, "unit": "s (setup+solve, plain FP64 method, extrapolated)",
           "cores": host["cores"], "kind": "oracle", "sample": host["sample"], "setup_s": setup, "solve_s": solve,
           "pcg_iterations_used": its, "cpu_model": host["cpu_model"], "blas": host["blas"],
           "sample_wall_median_s": host["sample_wall_median_s"]}
    return out


def roofline(met, workload_name, form):
    """Achieved FP64 MFMA rate of the metered kernel: algorithmic flops per
    dispatch / average event-timed dispatch duration, against the FP64 peak."""
    if met["launches"] == 0 or met["total_ms"] <= 0:
        return None
    avg_ms = met["total_ms"] / met["launches"]
    achieved = met["flops"] / (met["total_ms"] * 1e-3) / 1e12
    traffic = None
    if TRAFFIC and TRAFFIC["sha256"] == source_hash() and TRAFFIC["workload"] == workload_name \
            and TRAFFIC["form"] == form:
        traffic = TRAFFIC["bytes_per_launch"]
    return {"bound": "mfma", "kernel": "k_tiles<OpBlkUpd> (" + ROOFLINE_KERNEL + ")", "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
            "launches": met["launches"], "avg_launch_ms": avg_ms,
            "flops_per_launch": met["flops"] / met["launches"],
            "algorithmic_bytes_per_launch": met["bytes"] / met["launches"],
            "achieved_algorithmic_GBs": met["bytes"] / (met["total_ms"] * 1e-3) / 1e9,
            "source_sha256": source_hash(), "mapping": tuner_line(ROOFLINE_KERNEL)}


def tuner_line(name):
    """The launch-mapping tuner's candidates for one launch name (the chosen one starred)."""
    from paper_2109_05908_amd import autotune_report
    for ln in autotune_report().splitlines():
        if ln.startswith(name + ":"):
            return ln[len(name) + 1:].strip()
    return None


def pack_waves(sizes, kinds, cap):
    """Waves of one kind each (the production form's options depend on the kind), packed first-fit by
    decreasing size within a kind, at most cap[kind] unknowns per wave (a larger system alone).
    sizes: (kind, n) per system; returns lists of system indices, ascending within a wave."""
    waves = []
    for kind in kinds:
        bins, room = [], []
        for j in sorted((j for j in range(len(sizes)) if sizes[j][0] == kind), key=lambda j: -sizes[j][1]):
            n_j = sizes[j][1]
            k = next((k for k in range(len(bins)) if room[k] >= n_j), None)
            if k is None:
                bins.append([])
                room.append(cap[kind])
                k = len(bins) - 1
            bins[k].append(j)
            room[k] -= n_j
        waves += [sorted(w) for w in bins]
    return waves


def main_batch(args):
    """The many-systems workload: every system partitioned by seeded graph growing into parts of
    about 1024 unknowns (elasticity 648), overlap 1, lambda > 50, 2 levels; systems of one kind grouped
    into waves of at most --wave-dofs unknowns, each wave one batch handle (dd_setup_batch) solved for its
    right-hand sides by dd_pcg (one PCG per system and column, systems in lockstep; the learned
    form replays the iteration as a HIP graph).  A form's
    time is the sum over the waves of setup + solve; matrices, partitions and right-hand sides
    are on the GPU before each wave's clock starts."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2109_05908_amd import (DD_EIG_LOBPCG, DD_FP32, DD_SEL_THRESHOLD_CAP, DD_START_MODEL, DeviceCSR,
                                      Preconditioner, meter_read, meter_start, partition_ggg)
    from paper_2109_05908_amd.binding import DD_ERR_OOM, DDError
    from paper_2109_05908_amd.train_warm_start import load_model

    dev = "cuda:0"
    overlap, tau, levels = 1, 0.02, 2
    # unknowns per part: 1024 for the scalar kinds; elasticity takes the 648 of its 48^3 configuration,
    # whose dense local blocks (overlap 1 of a 27-node stencil) need less memory per unknown, and waves
    # of at most the size of that configuration
    per_part = {"elasticity3d_layered": 648}
    wave_cap = {"elasticity3d_layered": min(args.wave_dofs, 330000)}
    plan = W.batch_plan(args.batch_systems)
    systems = []
    for j, (kind, n_target, seed) in enumerate(plan):
        A = W.batch_system(kind, n_target, seed)
        systems.append((kind, A, max(1, int(round(A.n / per_part.get(kind, 1024))))))
        print(f"[batch] system {j}: {kind} n={A.n} parts={systems[-1][2]}", file=sys.stderr, flush=True)
    waves = pack_waves([(kind, A.n) for kind, A, _ in systems], W.C5_KINDS,
                       {k: wave_cap.get(k, args.wave_dofs) for k in W.C5_KINDS})
    n_total = sum(A.n for _, A, _ in systems)
    print(f"[batch] {len(systems)} systems, n = {n_total}, {len(waves)} waves", file=sys.stderr, flush=True)

    model, meta = load_model(args.model)
    learned_scalar = dict(select=DD_SEL_THRESHOLD_CAP, nev_cap=args.nev, eig_solver=DD_EIG_LOBPCG, lobpcg_tol=1e-4,
                          warm_start=DD_START_MODEL, model=model, local_prec=DD_FP32, graph_pcg=8)
    # elasticity: the network is trained on scalar diffusion with blocks of 8..32 modes, and 32 modes per
    # part leave most of the elastic near-kernel out (over 1000 iterations); the dense eigen route with at
    # most 256 modes per part keeps the iteration count near the threshold's
    learned_elastic = dict(select=DD_SEL_THRESHOLD_CAP, nev_cap=256, local_prec=DD_FP32, graph_pcg=8)
    # 2-D Poisson parts of about 1024 unknowns keep 43..161 modes above the threshold (oracle, 128^2 grid in
    # 16 parts): a cap of 32 left up to 313 iterations, so the dense route with at most 128 modes
    learned_2d = dict(select=DD_SEL_THRESHOLD_CAP, nev_cap=128, local_prec=DD_FP32, graph_pcg=8)
    per_kind = {"elasticity3d_layered": learned_elastic, "poisson2d_5pt": learned_2d}
    form_opts = {"learned": lambda kind: per_kind.get(kind, learned_scalar), "plain_fp64": lambda kind: {}}
    names = ["learned", "plain_fp64"] if args.batch_form == "both" else [args.batch_form]

    def load_wave(w):
        dAs = [DeviceCSR.from_workload(systems[j][1], device=dev) for j in waves[w]]
        parts = [partition_ggg(dA, systems[j][2], 0) for dA, j in zip(dAs, waves[w])]
        n_w = sum(dA.n for dA in dAs)
        g = torch.Generator(device=dev)
        g.manual_seed(w)
        b = torch.randn(n_w, args.nrhs, generator=g, device=dev, dtype=torch.float64)
        torch.cuda.synchronize()
        return dAs, parts, b

    def run_wave(w, opts, dAs, parts, b):
        Ns = [systems[j][2] for j in waves[w]]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pre = Preconditioner.batch(dAs, parts, Ns, overlap, tau, levels=levels, **opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, its, rr, code = pre.pcg(b, rtol=1e-8, maxit=3000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        inf = pre.info()
        del pre, x
        return t1 - t0, t2 - t1, its, rr, code, inf

    results, met = {}, None
    for name in names:
        opts_of = form_opts[name]

        def opts(w):
            return opts_of(systems[waves[w][0]][0])

        # untimed: the first wave of every kind once, so that the launch-mapping tuner samples its candidates
        firsts = sorted({min(w for w in range(len(waves)) if systems[waves[w][0]][0] == k)
                         for k in {systems[j][0] for j in range(len(systems))}})
        for w in firsts:
            dAs, parts, b = load_wave(w)
            try:
                ts, tv, its, rr, code, _ = run_wave(w, opts(w), dAs, parts, b)
                print(f"[batch] {name} tuning pass (wave {w}): setup {ts:.2f}s solve {tv:.2f}s", file=sys.stderr,
                      flush=True)
            except DDError as e:
                if e.code != DD_ERR_OOM:
                    raise
                print(f"[batch] {name} tuning pass (wave {w}): {e}", file=sys.stderr, flush=True)
            del dAs, parts, b
        if name == names[0]:
            meter_start(ROOFLINE_KERNEL)
        tot_setup = tot_solve = 0.0
        its_all, rr_max, n_c, per_wave = [], 0.0, 0, []
        failed = []
        for w in range(len(waves)):
            dAs, parts, b = load_wave(w)
            try:
                ts, tv, its, rr, code, inf = run_wave(w, opts(w), dAs, parts, b)
            except DDError as e:
                # a wave that does not fit the device is reported, and the form's total is then incomplete
                if e.code != DD_ERR_OOM:
                    raise
                del dAs, parts, b
                failed.append(w)
                per_wave.append({"systems": [systems[j][0] + f" n={systems[j][1].n}" for j in waves[w]],
                                 "n": sum(systems[j][1].n for j in waves[w]), "error": "out of device memory"})
                print(f"[batch] {name} wave {w}: {e}", file=sys.stderr, flush=True)
                continue
            del dAs, parts, b
            assert code == 0 and max(rr) <= 1e-8, (name, w, code, max(rr))
            tot_setup += ts
            tot_solve += tv
            its_all += list(its)
            rr_max = max(rr_max, max(rr))
            n_c += inf["n_C"]
            k_sys = len(waves[w])  # its: system j of right-hand side k at k * k_sys + j
            per_wave.append({"systems": [systems[j][0] + f" n={systems[j][1].n}" for j in waves[w]],
                             "n": sum(systems[j][1].n for j in waves[w]), "setup_s": round(ts, 3),
                             "solve_s": round(tv, 3),
                             "pcg_its_max_by_system": [int(max(its[j::k_sys])) for j in range(k_sys)]})
            print(f"[batch] {name} wave {w}: {len(waves[w])} systems setup {ts:.2f}s solve {tv:.2f}s "
                  f"its {min(its)}..{max(its)} relres <= {max(rr):.1e}", file=sys.stderr, flush=True)
        if name == names[0]:
            met = meter_read()
            meter_start(None)
        results[name] = {"setup_plus_solve_s": None if failed else tot_setup + tot_solve,
                         "setup_s_completed_waves": tot_setup, "solve_s_completed_waves": tot_solve,
                         "waves_out_of_memory": failed,
                         "pcg_its_mean": round(float(np.mean(its_all)), 2), "pcg_its_max": int(max(its_all)),
                         "relres_max": rr_max, "n_C": n_c, "waves": per_wave}
    first = results[names[0]]
    kinds = {k: sum(1 for kk, _, _ in systems if kk == k) for k in W.C5_KINDS}
    conf = {"workload": f"batch{len(systems)}_mixed: {len(systems)} systems, n log-uniform in [2e4, 5e5] (seed 0), "
                        f"{args.nrhs} right-hand sides each", "n_total": n_total, "systems_by_kind": kinds,
            "partition": "seeded greedy graph growing per system, about 1024 unknowns per part (elasticity: 648)",
            "overlap": overlap, "lambda_threshold": round(1 / tau), "tau": tau, "levels": levels,
            "waves": len(waves), "wave_dofs_max": args.wave_dofs, "nrhs_per_system": args.nrhs,
            "solver": "dd_pcg on each batch handle: one PCG per system and right-hand side, systems in lockstep",
            "learned_form": "3-D diffusion: learned warm start (LOBPCG to 1e-4, at most 32 modes per subdomain); "
                            "2-D Poisson and elasticity: dense eigen route, at most 128 and 256 modes per "
                            "subdomain; all with FP32 local factors and solves + PCG as a replayed HIP graph with "
                            "per-system scalars, autotuned launch mapping; waves of one kind each",
            "forms": results}
    if len(names) == 2 and results["plain_fp64"]["setup_plus_solve_s"] and first["setup_plus_solve_s"]:
        conf["speedup_vs_plain_fp64"] = results["plain_fp64"]["setup_plus_solve_s"] / first["setup_plus_solve_s"]
    line = {
        "metric": METRIC, "value": first["setup_plus_solve_s"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1000.0 * first["setup_plus_solve_s"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (f32 local factors and solves)" if names[0] == "learned" else "f64",
        "data": "synthetic", "config": conf, "roofline": roofline(met, conf["workload"], names[0]),
        "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    if args.achievable:
        achievable()
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload == "batch64_mixed":
        main_batch(args)
        return
    import numpy as np

    cfg, conf = workload(args.workload)
    host = None
    if not args.no_cpu_baseline:
        import oracle as O
        t0 = time.perf_counter()
        part_cpu = cfg.part if cfg.part is not None else O.ggg_partition(cfg.A, cfg.N, cfg.ggg_seed)
        host = cpu_baseline_host(cfg, np.asarray(part_cpu), reps=args.cpu_reps)
        print(f"[bench] CPU baseline sample: {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)

    import torch

    import workloads as W
    from paper_2109_05908_amd import (DD_EIG_LOBPCG, DD_FP32, DD_FP64, DD_SCHWARZ_ADDITIVE, DD_SCHWARZ_DEFLATED,
                                      DD_SEL_THRESHOLD_CAP, DD_START_MODEL, DD_START_RANDOM, DeviceCSR, Preconditioner,
                                      autotune_report, meter_read, meter_start, partition_ggg)
    from paper_2109_05908_amd.train_warm_start import load_model

    dev = "cuda:0"
    dA = DeviceCSR.from_workload(cfg.A, device=dev)
    if cfg.part is None:
        part = partition_ggg(dA, cfg.N, cfg.ggg_seed)
    else:
        part = torch.as_tensor(cfg.part, device=dev)
    b = torch.as_tensor(W.rhs(cfg.A.n, 0), device=dev)
    model, meta = load_model(args.model)
    learned = dict(select=DD_SEL_THRESHOLD_CAP, nev_cap=args.nev, eig_solver=DD_EIG_LOBPCG, lobpcg_tol=1e-4,
                   warm_start=DD_START_MODEL, model=model, local_prec=DD_FP32, graph_pcg=8)
    random_start = dict(learned, warm_start=DD_START_RANDOM, model=None)
    torch.cuda.synchronize()

    def step(opts):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pre = Preconditioner(dA, part, cfg.N, cfg.overlap, cfg.tau, levels=cfg.levels, **opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if opts.get("schwarz", DD_SCHWARZ_ADDITIVE) == DD_SCHWARZ_DEFLATED:  # not symmetric: GMRES(30)
            x, its, rr, code = pre.gmres(b, rtol=1e-8, maxit=3000, restart=30)
        else:
            x, its, rr, code = pre.pcg(b, rtol=1e-8, maxit=3000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        assert code == 0 and rr[0] <= 1e-8, (code, rr)
        inf = pre.info()
        ph = " ".join(f"{k}={v:.0f}" for k, v in inf["phase_ms"].items() if v >= 1.0)
        print(f"[bench]   setup phases (ms): {ph}", file=sys.stderr, flush=True)
        return pre, t1 - t0, t2 - t1, its[0], rr[0]

    def unsettled():
        # launch names of the tuner that have not picked a mapping yet (no starred candidate); names
        # never sampled (all counts 0) run only inside captured graphs, which use the fixed mapping
        out = []
        for ln in autotune_report().splitlines():
            if ln.strip() and "*" not in ln and any(not c.endswith("(0)") for c in ln.split()[1:]):
                out.append(ln.split(":")[0])
        return out

    tune_passes = {}

    def run_form(name, opts, steps, warmup, metered=False):
        # untimed: let the launch-mapping tuner finish sampling this form's kernels first, so that no
        # timed step runs candidate mappings (at most 8 setups; the count is reported)
        k = 0
        while k < 8 and (k == 0 or unsettled()):
            pre, ts, tv, its, rr = step(opts)
            del pre
            k += 1
        tune_passes[name] = k
        print(f"[bench] {name}: {k} tuning passes, unsettled: {unsettled()}", file=sys.stderr, flush=True)
        for w in range(warmup):
            pre, ts, tv, its, rr = step(opts)
            del pre
            print(f"[bench] {name} warmup {w}: setup {ts:.3f}s solve {tv:.3f}s its {its}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        if metered:
            meter_start(ROOFLINE_KERNEL)
        t_all = time.perf_counter()
        times, last = [], None
        for k in range(steps):
            pre, ts, tv, its, rr = step(opts)
            times.append((ts, tv, its, rr))
            print(f"[bench] {name} step {k}: setup {ts:.3f}s solve {tv:.3f}s its {its} relres {rr:.2e}",
                  file=sys.stderr, flush=True)
            if k < steps - 1:
                del pre
            else:
                last = pre
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_all
        met = meter_read() if metered else None
        if metered:
            meter_start(None)
        inf = last.info()
        res = {"setup_plus_solve_s": float(np.median([t[0] + t[1] for t in times])),
               "setup_s_median": float(np.median([t[0] for t in times])),
               "solve_s_median": float(np.median([t[1] for t in times])),
               "pcg_iterations": times[-1][2], "final_relres": times[-1][3], "n_C": inf["n_C"],
               "grid_complexity": round(inf["grid_complexity"], 4),
               "ms_per_pcg_iteration": round(1e3 * float(np.median([t[1] for t in times])) / max(1, times[-1][2]), 3),
               "coarse_factor_bytes": inf["coarse_factor_bytes"],
               "setup_phase_ms_last": {k: round(v, 1) for k, v in inf["phase_ms"].items()}}
        if inf["eig_iters_max"] > 0:
            res.update({"lobpcg_iters_mean": round(inf["eig_iters_mean"], 3), "lobpcg_iters_max": inf["eig_iters_max"]})
        del last
        return res, wall, met

    if args.form == "plain_fp64":
        main_res, wall, met = run_form("plain_fp64", {}, args.steps, args.warmup, metered=True)
        forms = {"plain_fp64": main_res}
    else:
        main_res, wall, met = run_form("learned", learned, args.steps, args.warmup, metered=True)
        forms = {"learned_fp32_graph": main_res}
    if not args.no_compare_forms and args.form == "learned":
        # the comparison forms run after the timed steps, at most 3 steps each (medians), so that a
        # long timed run does not hold the GPU five times as long
        cs = min(args.steps, 3)
        forms["plain_fp64"], _, _ = run_form("plain_fp64", {}, cs, 0)
        forms["random_start_fp32_graph"], _, _ = run_form("random_start", random_start, cs, 0)
        # one production feature taken away at a time
        forms["learned_fp64_local_graph"], _, _ = run_form("learned_fp64_local", dict(learned, local_prec=DD_FP64),
                                                           cs, 0)
        forms["learned_fp32_host_pcg"], _, _ = run_form("learned_host_pcg", dict(learned, graph_pcg=0), cs, 0)
        # the deflated variant of the experiments under GMRES(30), with the plain FP64 setup
        forms["deflated_gmres_fp64"], _, _ = run_form("deflated_gmres", dict(schwarz=DD_SCHWARZ_DEFLATED), cs, 0)
        conf["comparison_form_steps"] = cs
    value = main_res["setup_plus_solve_s"]
    conf.update({
        "form": (f"learned warm start (LOBPCG to 1e-4, at most {args.nev} modes per subdomain) + FP32 local "
                 "factors and solves + PCG as a replayed HIP graph") if args.form == "learned" else
                "plain FP64 (profiling run of the reference form alone)",
        "reference_form": "plain FP64: every mode with lambda > 50, dense eigen route, FP64 local solves, "
                          "host-driven PCG",
        "model": {"file": os.path.relpath(args.model, ROOT), "train_seeds": meta.get("train_seeds"),
                  "loss_last": meta.get("loss_last")},
        "pcg_iterations": main_res["pcg_iterations"], "n_C": main_res["n_C"], "forms": forms,
        "untimed_tuning_passes": tune_passes})
    if "plain_fp64" in forms:
        conf["speedup_vs_plain_fp64"] = forms["plain_fp64"]["setup_plus_solve_s"] / value
    out = {
        "metric": METRIC, "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * wall / args.steps, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (f32 local factors and solves)",
        "data": "synthetic", "config": conf, "roofline": roofline(met, conf["workload"], args.form),
    }
    if host is not None:
        its_plain = forms.get("plain_fp64", main_res)["pcg_iterations"]
        out["cpu_baseline"] = cpu_baseline_value(host, its_plain)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
