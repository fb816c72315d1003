#!/usr/bin/env python3
"""Throughput of the fused M1 transport + chemistry step on one MI355X.

One step = one rt_step call (fused kernel + one-block FP64 finalisation) over
the whole grid.  Default workload: the 1024^3 cosmological grid (10 Mpc/h box
at z = 9, lognormal density, 131072 sources in the densest cells, FP32
transport with FP64 chemistry for cells with xHI < 1e-3), inputs generated
on the device before the timed region.

Prints one JSON line with cell-updates/s, the roofline of the step kernel
(algorithmic 52 bytes per cell-update over its HIP-event duration) and the
FP64 oracle timed on the host cores over a bounded sample of the same state.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_CELL = 52          # read N,F,xHI,T,nH (28 B) + write N,F,xHI,T (24 B)
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
METRIC = "cell-updates/s (transport+chem) and % HBM peak, plain vs surrogate at 1024^3"
KERNEL_SRC = os.path.join(ROOT, "paper_1004_2503_amd", "csrc", "rt_step.hip")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(workload: str, nsub: int, prec: str):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"m1_step_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_sha") != kernel_hash() or d.get("nsub") != nsub or d.get("prec") != prec:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(G, w, dt, nsub, budget_s: float, seed: int = 20100417):
    """Time the FP64 oracle on sampled 32^3 sub-blocks (one step each, halo
    taken from the same device state)."""
    import torch

    import oracle

    oracle.lib()
    st = G.tensors()
    n = w.n
    B = 32
    rng = np.random.default_rng(seed)
    p = oracle.make_params((B, B, B), w.dx, chem=oracle.CHEM_FULL)
    cells = 0
    blocks = 0
    t_total = 0.0
    while t_total < budget_s and blocks < 512:
        z0, y0, x0 = (int(v) for v in rng.integers(0, n, 3))
        idx = [torch.arange(o - 1, o + B + 1, device=st["N"].device) % n for o in (z0, y0, x0)]

        def blk(t, halo):
            a = t.index_select(0, idx[0]).index_select(1, idx[1]).index_select(2, idx[2])
            if not halo:
                a = a[1:-1, 1:-1, 1:-1]
            return a.double().cpu().numpy()

        Np = blk(st["N"], True)
        Fp = [blk(st[k], True) for k in ("Fx", "Fy", "Fz")]
        xh, T, nh = blk(st["xHI"], False), blk(st["T"], False), blk(st["nH"], False)
        t0 = time.perf_counter()
        oracle.step_subblock(p, dt, nsub, Np, Fp, xh, T, nh)
        t_total += time.perf_counter() - t0
        cells += B ** 3
        blocks += 1
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    threads = min(threads, len(os.sched_getaffinity(0)))
    return {"value": cells / t_total, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{blocks} random {B}^3 sub-blocks of the {n}^3 state, one FP64 "
                      f"step each ({cells} cell-updates in {t_total:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cosmo1024",
                    choices=["cosmo128", "cosmo256", "cosmo512", "cosmo1024"])
    ap.add_argument("--nsub", type=int, default=1)
    ap.add_argument("--prec", default="mixed", choices=["fp32", "mixed"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the fused step kernel runs on a single "
              "MI355X holding the whole grid; multi-GPU runs are not supported.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1004_2503_amd import rt
    from paper_1004_2503_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = W.workload(args.workload)
    prec = rt.PREC_MIXED if args.prec == "mixed" else rt.PREC_FP32
    t_gen = time.perf_counter()
    nH, ijk, ndot = W.cosmo_inputs(w, device="cuda")
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    print(f"# inputs {w.name}: {w.n}^3, {len(ijk)} sources, generated in {t_gen:.1f} s",
          file=sys.stderr, flush=True)

    params = rt.make_params((w.n,) * 3, w.dx, chem=rt.CHEM_FULL, prec=prec)
    T0 = torch.full((w.n,) * 3, w.T0, dtype=torch.float32, device=dev)
    G = rt.RTGrid(params, dict(nH=nH, T=T0), device=dev)
    del nH, T0
    G.inject_sources(ijk, ndot)

    dt = w.dt
    G.step(dt, args.nsub, args.warmup)
    torch.cuda.synchronize()
    G.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.step(dt, args.nsub, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_kernel, launches = G.profile_read()
    G.profile(False)
    red = G.reduce()

    cells = w.cells
    wall = t1 - t0
    value = cells * args.steps / wall
    avg_ms = ms_kernel / max(launches, 1)
    achieved = BYTES_PER_CELL * cells / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(w.name, args.nsub, args.prec)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "m1_step_kernel", "avg_launch_ms": avg_ms,
            "bytes_per_cell": BYTES_PER_CELL}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(G, w, dt, args.nsub, args.cpu_seconds)
    G.close()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == rt.PREC_MIXED else "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n}^3 lognormal (sigma_ln 1.5, mean nH 2e-4), "
                               f"{len(ijk)} sources, plain exact chemistry",
                   "grid": w.n, "sources": len(ijk), "nsub": args.nsub,
                   "precision": args.prec, "dt_s": dt, "dx_cm": w.dx,
                   "parallelism": "single GPU, whole grid"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "hbm_frac_whole_step": BYTES_PER_CELL * value / (HBM_PEAK_GBS * 1e9),
        "state_after": {"xhi_vol": red["xhi_vol"], "xhi_mass": red["xhi_mass"],
                        "gamma_vol": red["gamma_vol"], "n_fp64": red["n_fp64"],
                        "n_nonfinite": red["n_nonfinite"]},
        "kernel_sha": kernel_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
