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
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_CELL = 52          # read N,F,xHI,T,nH (28 B) + write N,F,xHI,T (24 B)
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
METRIC = "cell-updates/s (transport+chem) and % HBM peak, plain vs surrogate at 1024^3"
KERNEL_SRC = [os.path.join(ROOT, "paper_1004_2503_amd", "csrc", f)
              for f in ("rt_step.hip", "rt_device.h", "rt_internal.h", "mlp_device.h")]


def kernel_hash() -> str:
    """Hash of the sources the step kernel is compiled from, with comments
    and whitespace removed (an edit of a comment leaves the kernel as it
    was)."""
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        with open(f) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, nsub: int, prec: str, flux: str = "lf"):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    name = f"m1_step_{workload}" if flux == "lf" else f"m1_step_{flux}_{workload}"
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_sha") != kernel_hash() or d.get("nsub") != nsub or d.get("prec") != prec:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(G, w, dt, nsub, budget_s: float, chem: str = "full", clump=None,
                 seed: int = 20100417):
    """Time the FP64 oracle on random 64^3 sub-blocks of the state (one step
    each, halo taken from the same device state) until budget_s of oracle
    time has been spent."""
    import torch

    import oracle

    oracle.lib()
    st = G.tensors()
    n = w.n
    B = 64
    rng = np.random.default_rng(seed)
    ochem = {"full": oracle.CHEM_FULL, "isothermal": oracle.CHEM_ISOTHERMAL,
             "off": oracle.CHEM_OFF}[chem]
    p = oracle.make_params((B, B, B), w.dx, chem=ochem, clump=clump)
    cells = 0
    blocks = 0
    t_total = 0.0
    while t_total < budget_s and blocks < 4096:
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


def _omp_threads(n: int):
    """Set the OpenMP thread count of this process (the oracle's parallel
    loops) through the OpenMP runtime it is linked with."""
    import ctypes

    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def _host_info() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            mem_kb = int(fh.readline().split()[1])
    except OSError:
        mem_kb = 0
    return {"cpu": model, "cpus_usable": len(os.sched_getaffinity(0)),
            "nproc_online": os.cpu_count(), "mem_GiB": round(mem_kb / 2 ** 20, 1)}


def cpu_baseline_configs(budget_s: float = 20.0):
    """The CPU baseline on the configurations themselves: the FP64 oracle on
    the Stromgren 32^3 test (200 steps), the 128^3 grid (1000 steps) and
    the 256^3 grid (500 steps), from their initial states, with one thread
    and with every usable host thread.  Each timing runs whole steps until
    the config's step count or budget_s of oracle time is reached; rates
    are cell-updates per second and the full-run times are extrapolated
    from them where the run was cut."""
    import oracle
    from paper_1004_2503_amd import workloads as W

    oracle.lib()
    full = max(1, int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0)))
    full = min(full, len(os.sched_getaffinity(0)))
    rows = []
    for name in ("stromgren32", "cosmo128", "cosmo256"):
        w = W.workload(name)
        n = w.n
        if name == "stromgren32":
            st = dict(xHI=np.ones((n,) * 3), T=np.full((n,) * 3, w.T0),
                      nH=np.full((n,) * 3, w.nH_mean))
            src = W.stromgren_sources(w)
            bc = w.bc
        else:
            nH, ijk, ndot = W.cosmo_inputs(w, device="cpu")
            nH = nH.numpy().astype(np.float64)
            st = dict(xHI=np.ones_like(nH), T=np.full_like(nH, w.T0), nH=nH)
            src = (ijk, ndot)
            bc = (0,) * 6
        for threads in (1, full):
            _omp_threads(threads)
            g = oracle.Grid(oracle.make_params((n,) * 3, w.dx, bc=bc, chem=oracle.CHEM_FULL))
            g.set_state(**st)
            g.set_sources(*src)
            done, t = 0, 0.0
            while done < w.steps and t < budget_s:
                t0 = time.perf_counter()
                g.step(w.dt, 1)
                t += time.perf_counter() - t0
                done += 1
            rate = n ** 3 * done / t
            rows.append({"config": name, "cells": n ** 3, "config_steps": w.steps,
                         "threads": threads, "steps_timed": done, "seconds": round(t, 3),
                         "cell_updates_per_s": rate,
                         "full_run_s": round(n ** 3 * w.steps / rate, 1),
                         "extrapolated": done < w.steps})
            print(f"# oracle {name} threads={threads}: {done} steps in {t:.1f} s, "
                  f"{rate:.3e} cell-updates/s", file=sys.stderr, flush=True)
    _omp_threads(full)
    return {"host": _host_info(), "rows": rows}


def surrogate_leg(args, G, w, dt, params, src):
    """Train the network on exact pairs (several dt, weighted towards the
    stiff and FP64 cells the step asks the network for) sampled from four
    states of the 256^3 run and from the 1024^3 state the comparison starts
    from, labelled by the exact adaptive operator with up to
    --label-cap sub-cycles; then time, from that state and for the same
    number of steps, the exact and the learned forms with fixed sub-cycling
    (nsub) and with adaptive sub-cycling (10% rule, capped at
    --adaptive-cap).  In both the learned forms and the exact adaptive form
    the stiff cells leave the bandwidth-bound step for the dense deferred
    kernel; the learned forms try the network there first."""
    import torch

    from paper_1004_2503_amd import rt, surrogate
    from paper_1004_2503_amd import workloads as W

    t0 = time.perf_counter()
    w256 = W.workload("cosmo256")
    nH, ijk, ndot = W.cosmo_inputs(w256, device="cuda")
    G2 = rt.RTGrid(rt.make_params((256,) * 3, w256.dx, prec=rt.PREC_MIXED), dict(nH=nH))
    del nH
    G2.inject_sources(ijk, ndot)
    states = []
    for _ in range(4):
        G2.step(w256.dt, 1, 125)
        t = G2.tensors()
        states.append({k: t[k].clone() for k in ("N", "xHI", "T", "nH")})
    G2.close()
    # the 1024^3 state the forms are compared from: its photon densities lie
    # far above the 256^3 run's near the sources (cells 64 times smaller)
    t = G.tensors()
    states.append({k: t[k].clone() for k in ("N", "xHI", "T", "nH")})
    pexact = rt.make_params((1, 1, 1), 1.0, chem=rt.CHEM_FULL, prec=rt.PREC_MIXED,
                            sub=rt.SUB_ADAPTIVE, sub_eps=0.1)
    dts = [W.courant_dt(W.cosmo_dx(n)) for n in (256, 512, 1024)]

    def make_pairs(total, seed, perturb=True):
        # twice as many cells sampled as kept: every stiff (or FP64) cell
        # among them is kept, the easy ones fill the rest
        per = total // (len(states) * len(dts))
        Xs, Us, Ys, n_hard = [], [], [], 0
        for i, st in enumerate(states):
            for j, d in enumerate(dts):
                c = surrogate.sample_cells(st, 2 * per, seed + 1000 * i + j)
                # half of them moved beyond the sampled states (hotter,
                # more ionised, brighter), where the run goes next
                if perturb:
                    c = surrogate.perturb_cells(c, seed + 77 + 1000 * i + j)
                X, U, Y, h = surrogate.candidate_pairs(pexact, c, d, per, args.label_cap,
                                                       fp64_thr=params.xhi_fp64_thr,
                                                       seed=seed + 1000 * i + j)
                Xs.append(X)
                Us.append(U)
                Ys.append(Y)
                n_hard += h
        return torch.cat(Xs), torch.cat(Us), torch.cat(Ys), n_hard

    X, U, _, n_hard = make_pairs(args.surrogate_pairs, 0)
    Xv, Uv, Yv, _ = make_pairs(1_000_000, 777_000, perturb=False)   # held out, as sampled
    n_pairs = int(X.shape[0])
    del states
    t_pairs = time.perf_counter() - t0
    s = surrogate.fit(X, U, steps=args.surrogate_steps, batch=65536, lr=2e-3,
                      grad_blocks=256, log_every=max(args.surrogate_steps // 6, 1),
                      verbose=False)
    t_train = time.perf_counter() - t0 - t_pairs
    del X, U
    P = surrogate.predict(s, Xv)
    dxv = (10 ** P[:, 0] - 10 ** Yv[:, 0]).abs()
    held = {"pairs": int(Xv.shape[0]), "mean_abs_dxHI": float(dxv.mean()),
            "p99_abs_dxHI": float(torch.quantile(dxv[:200_000].float(), 0.99)),
            "loss_untrained": surrogate.mse(surrogate.untrained(s), Xv, Uv),
            "loss_trained": surrogate.mse(s, Xv, Uv)}
    del Xv, Uv, Yv, P, dxv

    # the adaptive context starts from a copy of the same state
    snap = {k: v.clone() for k, v in G.tensors().items()}
    pad = rt.make_params((w.n,) * 3, w.dx, chem=params.chem, prec=params.prec,
                         sub=rt.SUB_ADAPTIVE, sub_eps=0.1)
    Ga = rt.RTGrid(pad, snap)
    Ga.inject_sources(*src)
    n_steps = max(args.steps // 2, 10)
    out = {}
    for form, GG, nsub, use in (("exact_fixed", G, args.nsub, False),
                                ("surrogate_fixed", G, args.nsub, True),
                                ("exact_adaptive", Ga, args.adaptive_cap, False),
                                ("surrogate_adaptive", Ga, args.adaptive_cap, True)):
        c = GG.current()                      # the buffer the next step reads
        for k in ("xHI", "T"):
            getattr(GG, k).copy_(snap[k])
        for k in ("N", "Fx", "Fy", "Fz"):
            getattr(GG, k)[c].copy_(snap[k])
        if use:
            rt.check(rt.rt_set_surrogate(GG.ctx, s.theta, s.norm_array(), 1e-3),
                     "rt_set_surrogate")
        r0 = GG.reduce()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        GG.step(dt, nsub, n_steps)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        r1 = GG.reduce()
        hist = [b - a for a, b in zip(r0["subcycle_hist"], r1["subcycle_hist"])]
        cs = w.cells * n_steps
        n_fb = r1["n_fallback"] - r0["n_fallback"]
        n_net = r1["n_learned"] - r0["n_learned"]
        n_rng = r1["n_fallback_range"] - r0["n_fallback_range"]
        out[form] = dict(ms_per_step=(tb - ta) / n_steps * 1e3,
                         value=cs / (tb - ta),
                         network_cells_per_step=(n_fb + n_net) / n_steps,
                         accepted_frac_of_network_cells=n_net / max(n_fb + n_net, 1),
                         fallback_frac=n_fb / cs,
                         out_of_range_frac_of_network_cells=n_rng / max(n_fb + n_net, 1),
                         fp64_cells_per_step=(r1["n_fp64"] - r0["n_fp64"]) / n_steps,
                         subcycle_hist=hist, xHI=GG.xHI.clone())
        rt.check(rt.rt_set_surrogate(GG.ctx, None, None, 0.0), "rt_set_surrogate off")
    Ga.close()
    del snap

    def dx(a, b):
        return float((out[a]["xHI"] - out[b]["xHI"]).abs().double().mean())

    forms = {k: {kk: vv for kk, vv in v.items() if kk != "xHI"} for k, v in out.items()}
    ms = {k: v["ms_per_step"] for k, v in out.items()}
    sp = ms["exact_adaptive"] / ms["surrogate_adaptive"]
    return {"value": out["surrogate_adaptive"]["value"], "unit": "cell-updates/s",
            "ms_per_step": ms["surrogate_adaptive"],
            "plain_ms_per_step_same_state": ms["exact_fixed"],
            "speedup_vs_plain": ms["exact_fixed"] / ms["surrogate_fixed"],
            "speedup_vs_adaptive_exact": sp,
            "fraction_of_2x_target": sp / 2.0,
            "adaptive_cap": args.adaptive_cap, "forms": forms, "steps": n_steps,
            "mean_abs_dxHI_vs_exact_after_steps": {"fixed": dx("surrogate_fixed", "exact_fixed"),
                                                   "adaptive": dx("surrogate_adaptive",
                                                                  "exact_adaptive")},
            "held_out": held,
            "train": {"pairs": n_pairs, "stiff_or_fp64_pairs": n_hard,
                      "sources": "4 states of the 256^3 run + the 1024^3 start state; "
                                 "half the cells perturbed in T, xHI and N",
                      "label_cap": args.label_cap,
                      "adam_steps": args.surrogate_steps,
                      "pair_gen_s": t_pairs, "train_s": t_train,
                      "loss_first_last": [s.history[0][1], s.history[-1][1]]}}


def diagnostics_leg(G, w, reps: int = 5):
    """Time rt_histogram (Sec. 3.1.5 distributions, 64 x 64 bins) over the
    whole grid for both quantities: one pass reading nH and xHI or N, 8
    bytes per cell; the call includes its small host copies and a stream
    wait.  Also reports the Thomson depth accumulated by the run."""
    import torch

    from paper_1004_2503_amd import rt

    out = {}
    xr = (-6.0, 1.0, 64)
    for name, q, yr in (("xHI", rt.HQ_XHI, (-7.0, 0.5, 64)),
                        ("gamma", rt.HQ_GAMMA, (-18.0, -8.0, 64))):
        G.histogram(q, xr, yr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            counts, sums = G.histogram(q, xr, yr)
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"ms": dt * 1e3, "GBs": 8.0 * w.cells / dt / 1e9,
                     "nonzero_bins": int(np.count_nonzero(counts))}
    out["tau_e"] = G.reduce()["tau_e"]
    # Sec. 3.1.5 analysis: plateau rate below 1e-3 cm^-3, then the equilibrium
    # neutral fraction under the plateau, J1 and J4 models at a few densities
    g0, _ = G.gamma_plateau(1e-3)
    dens = torch.tensor([1e-4, 1e-3, 1e-2, 1e-1], dtype=torch.float64, device=G.device)
    temp = torch.full_like(dens, 1e4)
    eq = {"gamma0": g0, "nH": dens.tolist()}
    for name, model, ns in (("J0", rt.JMODEL_UNIFORM, 0.0), ("J1", rt.JMODEL_EXP1, 0.007),
                            ("J4", rt.JMODEL_EXP4, 0.018)):
        eq[name] = rt.equilibrium_xhi(G.params, model, g0, ns, dens, temp).tolist()
    out["equilibrium_xhi"] = eq
    return out


def hll_leg(G, w, dt, params, src, nsub: int, prec: str, steps: int = 20):
    """Time the step with HLL intercell fluxes (Sec. 2.2) on a copy of the
    run's current state: same fields read and written (52 bytes per cell),
    the six signal speeds of every cell computed in the kernel.  Kernel time
    from the library's own events, as for the main step."""
    import torch

    from paper_1004_2503_amd import rt

    ph = rt.rt_params.from_buffer_copy(params)
    ph.flux = rt.FLUX_HLL
    H = rt.RTGrid(ph, {k: v for k, v in G.tensors().items()}, device=G.device)
    H.inject_sources(*src)
    H.step(dt, nsub, 2)
    torch.cuda.synchronize()
    H.profile(True)
    t0 = time.perf_counter()
    H.step(dt, nsub, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_kernel, launches = H.profile_read()
    H.profile(False)
    red = H.reduce()
    H.close()
    del H
    torch.cuda.empty_cache()
    avg = ms_kernel / max(launches, 1)
    gbs = BYTES_PER_CELL * w.cells / (avg * 1e-3) / 1e9
    return {"steps": steps, "ms_per_step": wall / steps * 1e3, "avg_launch_ms": avg,
            "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS,
            "traffic": measured_traffic(w.name, nsub, prec, "hll"),
            "n_nonfinite": red["n_nonfinite"]}


def sources_leg(G, w, nH_dev, n: int = 1_000_000, reps: int = 3):
    """Time rt_sources_from_particles: n seeded star particles in the
    densest cells of the grid (Sec. 2.3 pipeline: lifetimes, interval
    dilution, escape fraction and boost, NGP binning into the per-tile
    source lists).  Replaces the grid's sources, so it runs last."""
    import torch

    from paper_1004_2503_amd import workloads as W

    parts = W.star_particles(nH_dev, w.dx, n)
    d = {k: torch.tensor(v, dtype=torch.float64, device="cuda").contiguous()
         for k, v in parts.items()}
    myr = W.MYR_S
    args = (700 * myr, 703 * myr, 0.02, 1.2, 3000 * myr)
    G.sources_from_particles(d, *args)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        m = G.sources_from_particles(d, *args)
    dt = (time.perf_counter() - t0) / reps
    return {"particles": n, "emitting": m, "ms": dt * 1e3}


def stream_ceiling(dev, n: int = 1 << 30, reps: int = 10):
    """GB/s of the step's stream mix (7 float arrays of n read, 6 written)
    on plain grid-stride kernels for a few grid sizes and in the step
    kernel's tile-marching order, and of a device copy; the arrays are
    placed as RTGrid places the step's fields (one allocation, 256-byte
    stagger), and the tile-marching probe is repeated on separately
    allocated arrays.  The step kernel's rate is compared with them."""
    import torch

    from paper_1004_2503_amd import rt

    side = round(n ** (1.0 / 3.0))
    cubic = side ** 3 == n and side % 128 == 0

    def march_row(arr, label):
        rc, ms = rt.rt_march_probe(arr[:7], arr[7:13], (side,) * 3, reps)
        rt.check(rc, "rt_march_probe")
        gbs = 52 * n / (ms * 1e-3) / 1e9
        print(f"# tile-marching order, {side}^3, {label}: {ms:.3f} ms, {gbs:.1f} GB/s",
              file=sys.stderr, flush=True)
        return {"mix": f"7 read + 6 write in the step's tile-marching order, {label}",
                "blocks": (side // 64) * (side // 16) * (side // 128), "ms": ms, "GBs": gbs}

    rows = []
    march_separate = None
    if cubic:
        arr = [torch.zeros(n, dtype=torch.float32, device=dev) for _ in range(13)]
        rows.append(march_row(arr, "13 separate allocations"))
        march_separate = rows[-1]["GBs"]
        del arr
        torch.cuda.empty_cache()
    stride = (n + 63) // 64 * 64 + rt.FIELD_STAGGER
    slab = torch.zeros(stride * 12 + n, dtype=torch.float32, device=dev)
    arr = [slab[k * stride:k * stride + n] for k in range(13)]
    for blocks in (4096, 16384, 65536):
        for name, nin, nout in (("7 read + 6 write (the step's mix)", 7, 6),
                                ("7 read + 1 write", 7, 1)):
            rc, ms = rt.rt_stream_probe(arr[:nin], arr[7:7 + nout], blocks, reps)
            rt.check(rc, "rt_stream_probe")
            gbs = (nin + nout) * 4 * n / (ms * 1e-3) / 1e9
            rows.append({"mix": name, "blocks": blocks, "ms": ms, "GBs": gbs})
            print(f"# {name}, {blocks} blocks: {ms:.3f} ms, {gbs:.1f} GB/s", file=sys.stderr,
                  flush=True)
    march = None
    if cubic:
        rows.append(march_row(arr, "one allocation, 256-byte stagger"))
        march = rows[-1]["GBs"]
    # a device copy of 4 GiB (torch's copy_) for reference
    src, dst = arr[0], arr[7]
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    rows.append({"mix": "device copy (torch copy_)", "blocks": None, "ms": ms,
                 "GBs": 8 * n / (ms * 1e-3) / 1e9})
    best = max(r["GBs"] for r in rows if r["mix"].startswith("7 read + 6 write (the step"))
    return {"stream_ceiling": rows, "best_step_mix_GBs": best, "tile_march_GBs": march,
            "tile_march_separate_GBs": march_separate, "n_floats_per_array": n,
            "stagger_bytes": 4 * rt.FIELD_STAGGER, "reps": reps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cosmo1024",
                    choices=["cosmo128", "cosmo256", "cosmo512", "cosmo1024"])
    ap.add_argument("--nsub", type=int, default=1)
    ap.add_argument("--prec", default="mixed", choices=["fp32", "mixed"])
    ap.add_argument("--chem", default="full", choices=["full", "isothermal", "off"])
    ap.add_argument("--clump", default=None, choices=["A", "B"],
                    help="subgrid clumping laws in the chemistry (default: none)")
    ap.add_argument("--flux", default="lf", choices=["lf", "hll"],
                    help="intercell flux of the timed step (the paper's runs use LF)")
    ap.add_argument("--no-hll", action="store_true",
                    help="skip the extra timing of the HLL step on the evolved state")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="instead of the step, time a plain device copy of MIB MiB "
                         "(the reference for the HBM byte counters)")
    ap.add_argument("--stream-ceiling", action="store_true",
                    help="instead of the step, measure the bandwidth the step's stream mix "
                         "can reach: 7 arrays of 1024^3 floats read and 6 written by a "
                         "plain grid-stride kernel (rt_stream_probe), and plain copies")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-configs", action="store_true",
                    help="instead of the step, time the FP64 oracle on the 32^3, 128^3 and "
                         "256^3 configurations with one and with all host threads")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip training the learned chemistry on exact pairs from the "
                         "256^3 run and timing its forms against the exact ones on the "
                         "same 1024^3 state")
    ap.add_argument("--surrogate-pairs", type=int, default=10_000_000)
    ap.add_argument("--surrogate-steps", type=int, default=80000)
    ap.add_argument("--label-cap", type=int, default=1024,
                    help="sub-cycle cap of the exact adaptive operator that labels the "
                         "surrogate's training pairs")
    ap.add_argument("--adaptive-cap", type=int, default=32,
                    help="sub-cycle cap of the adaptive forms in the surrogate comparison")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the fused step kernel runs on a single "
              "MI355X holding the whole grid; multi-GPU runs are not supported.",
              file=sys.stderr)
        sys.exit(2)

    if args.cpu_baseline_configs:
        print(json.dumps(cpu_baseline_configs(args.cpu_seconds)), flush=True)
        return

    import torch

    from paper_1004_2503_amd import rt
    from paper_1004_2503_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(args.warmup):
            dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        dtc = (time.perf_counter() - t0) / args.steps
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                          "ms": dtc * 1e3, "GBs": 8 * n / dtc / 1e9}), flush=True)
        return
    if args.stream_ceiling:
        print(json.dumps(stream_ceiling(dev)), flush=True)
        return
    w = W.workload(args.workload)
    prec = rt.PREC_MIXED if args.prec == "mixed" else rt.PREC_FP32
    t_gen = time.perf_counter()
    nH, ijk, ndot = W.cosmo_inputs(w, device="cuda")
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    print(f"# inputs {w.name}: {w.n}^3, {len(ijk)} sources, generated in {t_gen:.1f} s",
          file=sys.stderr, flush=True)

    chem = {"full": rt.CHEM_FULL, "isothermal": rt.CHEM_ISOTHERMAL, "off": rt.CHEM_OFF}[args.chem]
    clump = None if args.clump is None else W.CLUMP_LAWS[args.clump]
    flux = rt.FLUX_HLL if args.flux == "hll" else rt.FLUX_LF
    params = rt.make_params((w.n,) * 3, w.dx, chem=chem, prec=prec, clump=clump, flux=flux)
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
    traffic = measured_traffic(w.name, args.nsub, args.prec, args.flux)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "m1_step_kernel (+ defer_chem_kernel in the mixed LF form)",
            "avg_launch_ms": avg_ms,
            "bytes_per_cell": BYTES_PER_CELL}

    diag = diagnostics_leg(G, w)
    hll = None
    if flux == rt.FLUX_LF and not args.no_hll:
        hll = hll_leg(G, w, dt, params, (ijk, ndot), args.nsub, args.prec)

    surr = None
    if not args.no_surrogate:
        surr = surrogate_leg(args, G, w, dt, params, (ijk, ndot))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(G, w, dt, args.nsub, args.cpu_seconds, args.chem, clump)
    srcs = sources_leg(G, w, G.nH)
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
                               f"{len(ijk)} sources, plain exact chemistry"
                               + ("" if args.chem == "full" else f" (chemistry {args.chem})")
                               + ("" if clump is None else
                                  f", subgrid clumping {args.clump} laws {clump}")
                               + ("" if flux == rt.FLUX_LF else ", HLL fluxes"),
                   "grid": w.n, "sources": len(ijk), "nsub": args.nsub, "chem": args.chem,
                   "clump": args.clump, "flux": args.flux,
                   "precision": args.prec, "dt_s": dt, "dx_cm": w.dx,
                   "parallelism": "single GPU, whole grid"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "diagnostics": diag,
        "source_pipeline": srcs,
        "hll_step": hll,
        "surrogate": surr,
        "hbm_frac_whole_step": BYTES_PER_CELL * value / (HBM_PEAK_GBS * 1e9),
        "state_after": {"xhi_vol": red["xhi_vol"], "xhi_mass": red["xhi_mass"],
                        "gamma_vol": red["gamma_vol"], "n_fp64": red["n_fp64"],
                        "n_nonfinite": red["n_nonfinite"]},
        "kernel_sha": kernel_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
