#!/usr/bin/env python3
"""Benchmark of the stencil hot path on one MI355X.

Step = one advec_u + diff_uvw pair (configurations selected from the wisdom
files) over a 512^3 FP32 staggered grid: sinusoidal modes n = 1..8 plus 0.1
seeded noise (seed 2), z walls with zero-gradient w, tanh-stretched z,
viscosity 1e-5.  Inputs are resident in HBM before the timed region.

Prints one JSON line: grid-points/s of the pair, HBM GB/s of the
algorithmic bytes (14 values per point), the dominant kernel's roofline
entry (per-launch duration from HIP events on the launch stream), the
untuned default configurations on the same grid, and the CPU oracle timed on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-points/s & HBM GB/s (% peak), advec_u+diff_uvw 512^3 FP32; p99 latency"
PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E, published
KERNEL_SOURCES = ["paper_2303_12374_amd/csrc/stencil.hpp", "paper_2303_12374_amd/csrc/variants.hpp",
                  "paper_2303_12374_amd/csrc/variants_f32.hip", "paper_2303_12374_amd/csrc/variants_f64.hip"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_name, workload_key, variant):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel sources and configuration."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        rec = data.get(f"{kernel_name}:{workload_key}")
        if not rec or rec.get("source_hash") != kernel_source_hash() or rec.get("variant") != variant:
            return None
        return float(rec["hbm_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def cpu_baseline(itot, jtot, k_sample, seed, visc, reps=7):
    """The CPU oracle (FP64, OpenMP over k) on a 512 x 512 x k_sample slab of
    the same field recipe; grid-points/s of one advec_u + diff_uvw pair."""
    import numpy as np

    import oracle
    from paper_2303_12374_amd import inputs
    lib = oracle.load()
    zg = inputs.zgrid(k_sample, inputs.domain_height(itot, jtot, k_sample), 1.5)
    fs = inputs.sinusoid_fields(seed, itot, jtot, k_sample, zg)
    off, js, ks, alloc = inputs.plain_layout(itot, jtot, k_sample)
    g = oracle.Grid(itot, jtot, k_sample, off, js, ks, alloc, float(np.float32(itot)), float(np.float32(jtot)),
                    zg["dzi"].astype(np.float32).astype(np.float64),
                    zg["dzhi"].astype(np.float32).astype(np.float64), 0)
    host = [inputs.embed(f.astype(np.float32).astype(np.float64), off, js, ks, alloc) for f in fs]
    oracle.fill_ghosts(g, *host)
    tend = [np.zeros(alloc) for _ in range(3)]
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        oracle.advec_u(g, tend[0], *host)
        oracle.diff_uvw(g, tend[0], tend[1], tend[2], *host, visc)
        times.append(time.perf_counter() - t0)
    best = float(np.median(times))
    threads = lib.ora_threads() if hasattr(lib, "ora_threads") else os.cpu_count()
    npts = itot * jtot * k_sample
    return {"value": npts / best, "unit": "grid-points/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{itot}x{jtot}x{k_sample} slab of the same recipe, FP64 oracle, one advec_u+diff_uvw "
                      f"pair, median of {reps} runs ({best:.3f} s each, {sum(times):.1f} s total)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", default="512,512,512")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--recipe", default="sinusoid", choices=["sinusoid", "random"])
    ap.add_argument("--wisdom", default=os.path.join(ROOT, "wisdom"))
    ap.add_argument("--tune", action="store_true", help="tune both kernels first (appends to --wisdom)")
    ap.add_argument("--tune-budget", type=float, default=60.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-k", type=int, default=128)
    ap.add_argument("--no-untuned", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent grids shard by grid, one process per GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2303_12374_amd import inputs, kl

    itot, jtot, ktot = (int(x) for x in args.size.split(","))
    dtype = kl.F32 if args.dtype == "f32" else kl.F64
    s = 4 if dtype == kl.F32 else 8
    seed, visc = 2, 1e-5
    torch.cuda.set_device(0)
    kl.kl_set_wisdom_dir(args.wisdom)

    log(f"generating {itot}x{jtot}x{ktot} {args.dtype} {args.recipe} fields (seed {seed})")
    g = kl.Grid(itot, jtot, ktot, dtype=dtype, bc=kl.BC_ZWALL_ZEROGRAD)
    if args.recipe == "sinusoid":
        fs = inputs.sinusoid_fields(seed, itot, jtot, ktot, g.zg)
    else:
        fs = inputs.random_fields(seed, itot, jtot, ktot)
    dev = []
    for f in fs:
        dev.append(g.upload(f.astype(kl.NP_DTYPE[dtype])))
    del fs
    kl.kl_fill_ghosts(g, *dev)
    tend = [g.zeros_interior(fill=0.0) for _ in range(3)]
    u, v, w = dev
    ut, vt, wt = tend
    torch.cuda.synchronize()

    if args.tune:
        log("tuning advec_u and diff_uvw")
        kl.kl_tune(g, dev + tend, 3, args.wisdom, args.tune_budget)
        torch.cuda.synchronize()

    sel = {name: kl.kl_selected_variant(g, k) for name, k in (("advec_u", kl.ADVEC_U), ("diff_uvw", kl.DIFF_UVW))}
    sel_names = {n: kl.kl_variant_name(k, dtype, sel[n]) for n, k in (("advec_u", kl.ADVEC_U), ("diff_uvw", kl.DIFF_UVW))}
    log(f"selected configurations: {sel_names}")

    stream = torch.cuda.current_stream()

    def sel_advec():
        kl.kl_advec_u(g, ut, u, v, w, stream)

    def sel_diff():
        kl.kl_diff_uvw(g, ut, vt, wt, u, v, w, visc, stream)

    def timed(advec_fn, diff_fn, steps, warmup):
        """Per-launch durations from HIP events recorded on the launch stream."""
        for _ in range(warmup):
            advec_fn()
            diff_fn()
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        t_start.record(stream)
        for e in ev:
            e[0].record(stream)
            advec_fn()
            e[1].record(stream)
            diff_fn()
            e[2].record(stream)
        t_end.record(stream)
        torch.cuda.synchronize()
        total_ms = t_start.elapsed_time(t_end)
        adv = [e[0].elapsed_time(e[1]) for e in ev]
        dif = [e[1].elapsed_time(e[2]) for e in ev]
        return total_ms, float(np.mean(adv)), float(np.mean(dif)), float(np.median(adv)), float(np.median(dif))

    log(f"timing {args.steps} steps after {args.warmup} warm-up steps")
    total_ms, adv_ms, dif_ms, adv_med, dif_med = timed(sel_advec, sel_diff, args.steps, args.warmup)
    npts = itot * jtot * ktot
    ms_per_step = total_ms / args.steps
    value = npts * args.steps / (total_ms * 1e-3)
    bytes_adv = 5 * npts * s
    bytes_dif = 9 * npts * s
    pair_gbps = (bytes_adv + bytes_dif) / (ms_per_step * 1e6)
    dominant = "diff_uvw" if dif_ms >= adv_ms else "advec_u"
    dom_bytes, dom_ms = (bytes_dif, dif_ms) if dominant == "diff_uvw" else (bytes_adv, adv_ms)
    achieved = dom_bytes / (dom_ms * 1e6)
    wkey = f"{itot}x{jtot}x{ktot}_{args.dtype}"
    traffic = load_traffic(dominant, wkey, sel_names[dominant])

    untuned = None
    if not args.no_untuned and (sel["advec_u"] != 0 or sel["diff_uvw"] != 0):
        k = max(3, args.steps // 2)
        t_ms, a_ms, f_ms, _, _ = timed(
            lambda: kl.kl_launch_variant(g, kl.ADVEC_U, 0, dev + tend, visc, stream),
            lambda: kl.kl_launch_variant(g, kl.DIFF_UVW, 0, dev + tend, visc, stream), k, 2)
        untuned = {"ms_per_step": t_ms / k, "advec_u_ms": a_ms, "diff_uvw_ms": f_ms,
                   "grid_points_per_s": npts * k / (t_ms * 1e-3),
                   "speedup_tuned_vs_untuned": (t_ms / k) / ms_per_step}

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"advec_u+diff_uvw {itot}x{jtot}x{ktot} {args.dtype.upper()}, "
                               f"{args.recipe} fields seed {seed}, z walls zero-gradient w, tanh z, visc 1e-5",
                   "grid": [itot, jtot, ktot], "configurations": sel_names},
        "hbm_gbps": pair_gbps,
        "hbm_frac_of_peak": pair_gbps / PEAK_HBM_GBPS,
        "kernels": {"advec_u": {"ms": adv_ms, "median_ms": adv_med, "gbps": bytes_adv / (adv_ms * 1e6)},
                    "diff_uvw": {"ms": dif_ms, "median_ms": dif_med, "gbps": bytes_dif / (dif_ms * 1e6)}},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBPS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": dom_bytes},
        "untuned": untuned,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(itot, jtot, args.cpu_sample_k, seed, float(np.float32(visc)))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
