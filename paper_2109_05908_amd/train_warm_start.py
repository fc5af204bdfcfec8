"""Train the warm-start network of the block eigensolver on a family of
matrices and evaluate it on held-out members (GPU).

The family is the 64^3 high-contrast diffusion workload with its coefficient
field resampled per seed (same pattern, same 256-part partition).  Training
samples come from setups of the training seeds with the dense eigen route in
cap mode (their kept vectors are exact); the network is trained by the
library's own kernels (dd_model_train).  The parameters are written as JSON.

Evaluation on held-out seeds: the block eigensolver from a random start, from
the near-kernel range start without the network, and from the learned start,
each to an eigen-residual of 1e-4 (LOBPCG iterations, eigen phase time, PCG
iterations) and with a budget of two iterations (median eigen-residual).

    python -m paper_2109_05908_amd.train_warm_start --train 0:150 --eval 150:200:10
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_MODEL = os.path.join(HERE, "warm_start_c4.json")


def _range(spec: str) -> list[int]:
    parts = [int(x) for x in spec.split(":")]
    return list(range(*parts))


def load_model(path: str = DEFAULT_MODEL):
    """A WarmStartModel with the parameters stored at `path`."""
    from .binding import WarmStartModel
    with open(path) as f:
        meta = json.load(f)
    m = WarmStartModel(0)
    m.set_params(np.asarray(meta["params"], dtype=np.float64))
    return m, meta


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", default="0:150")
    ap.add_argument("--eval", default="150:200:10")
    ap.add_argument("--nev", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=600)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--report", default="")
    args = ap.parse_args()

    import torch

    import workloads as W
    from paper_2109_05908_amd import (DD_EIG_LOBPCG, DD_SEL_THRESHOLD_CAP, DD_START_MODEL, DD_START_RANDOM,
                                      DD_START_RANGE, DeviceCSR, Preconditioner, WarmStartModel, partition_ggg)

    cfg0 = W.config_c2(seed=0)
    dA0 = DeviceCSR.from_workload(cfg0.A)
    part = partition_ggg(dA0, cfg0.N, cfg0.ggg_seed)
    kw = dict(select=DD_SEL_THRESHOLD_CAP, nev_cap=args.nev)
    model = WarmStartModel(1)
    t0 = time.perf_counter()
    train = _range(args.train)
    for k, sd in enumerate(train):
        cfg = W.config_c2(seed=sd)
        P = Preconditioner(DeviceCSR.from_workload(cfg.A), part, cfg.N, cfg.overlap, cfg.tau, **kw)
        model.add_samples(P)
        del P
        print(f"[train] samples from matrix {sd} ({k + 1}/{len(train)}), {time.perf_counter() - t0:.0f}s", flush=True)
    t1 = time.perf_counter()
    losses = []
    for e in range(0, args.epochs, 50):
        losses.extend(model.train(min(50, args.epochs - e), args.lr).tolist())
        print(f"[train] epoch {e + 50}: loss {losses[-1]:.5f}", flush=True)
    t2 = time.perf_counter()
    meta = {"family": "diffusion3d_7pt_64^3_lognormal_sigma2_channels1e6, coefficients resampled per seed",
            "partition": "256 parts, seeded greedy graph growing (seed 0), overlap 2, lambda > 50",
            "nev_cap": args.nev, "train_seeds": [train[0], train[-1] + 1], "epochs": args.epochs, "lr": args.lr,
            "loss_first": losses[0], "loss_last": losses[-1], "sample_setup_s": t1 - t0, "train_s": t2 - t1,
            "params": model.params().tolist()}
    with open(args.out, "w") as f:
        json.dump(meta, f)
    print(f"[train] wrote {args.out}: loss {losses[0]:.4f} -> {losses[-1]:.4f}, training {t2 - t1:.1f}s", flush=True)

    rows = []
    for sd in _range(args.eval):
        cfg = W.config_c2(seed=sd)
        dA = DeviceCSR.from_workload(cfg.A)
        b = torch.as_tensor(W.rhs(cfg.A.n, 0), device="cuda")
        for name, ws, m in (("random", DD_START_RANDOM, None), ("range", DD_START_RANGE, None),
                            ("learned", DD_START_MODEL, model)):
            opts = dict(kw, eig_solver=DD_EIG_LOBPCG, warm_start=ws, model=m, seed=sd)
            P = Preconditioner(dA, part, cfg.N, cfg.overlap, cfg.tau, lobpcg_tol=1e-4, **opts)
            its, _ = P.eig_stats()
            inf = P.info()
            _, pits, rr, _ = P.pcg(b, rtol=1e-8, maxit=3000)
            del P
            Pb = Preconditioner(dA, part, cfg.N, cfg.overlap, cfg.tau, lobpcg_maxit=2, **opts)
            _, r2 = Pb.eig_stats()
            del Pb
            rows.append({"seed": sd, "start": name, "lobpcg_its_mean": float(its.mean()),
                         "lobpcg_its_max": int(its.max()), "eigen_ms": inf["phase_ms"]["eigen"],
                         "pcg_its": int(pits[0]), "relres": float(rr[0]), "median_resid_after_2": float(np.median(r2))})
            r = rows[-1]
            print(f"[eval] seed {sd} {name:8s}: LOBPCG its mean {r['lobpcg_its_mean']:.2f} max {r['lobpcg_its_max']}, "
                  f"eigen {r['eigen_ms']:.0f} ms, PCG its {r['pcg_its']}, residual after 2 "
                  f"{r['median_resid_after_2']:.2e}", flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump({"meta": {k: v for k, v in meta.items() if k != "params"}, "eval": rows}, f, indent=1)


if __name__ == "__main__":
    main()
