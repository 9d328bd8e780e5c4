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
_CSRC = "paper_2303_12374_amd/csrc/"
# device sources whose change invalidates a kernel's recorded counters
KERNEL_SOURCES = {
    "advec_u": [_CSRC + "stencil.hpp", _CSRC + "stencil_zl.hpp"],
    "diff_uvw": [_CSRC + "stencil.hpp", _CSRC + "stencil_zl.hpp"],
    "advec_u_2i5": [_CSRC + "stencil.hpp", _CSRC + "stencil_zl.hpp", _CSRC + "stencil_les.hpp",
                    _CSRC + "stencil_les_zl.hpp"],
    "diff_smag": [_CSRC + "stencil.hpp", _CSRC + "stencil_zl.hpp", _CSRC + "stencil_les.hpp",
                  _CSRC + "stencil_les_zl.hpp"],
    "step": [_CSRC + "stencil.hpp", _CSRC + "stencil_zl.hpp", _CSRC + "stencil_step.hpp"],
    "advec_diff": [_CSRC + "stencil.hpp", _CSRC + "stencil_zl.hpp", _CSRC + "stencil_step.hpp"],
}


def kernel_of_symbol(sym):
    """Library kernel a rocprofv3 kernel symbol belongs to, or None.  The
    step tile serves both the fused step (last template argument 0) and the
    fused advec_u + diff_uvw pass (1)."""
    import re
    m = re.search(r"kl::(\w+?)_(zl3|zlp|zl|zr|zc|plain)(_batch)?<([^>]*)>", sym)
    if not m:
        m = re.search(r"kl::(step)_zl(_batch)?<([^>]*)>", sym)
        if not m:
            return None
        return "advec_diff" if m.group(3).split(",")[-1].strip() == "1" else "step"
    name = m.group(1)
    if name == "step":
        return "advec_diff" if m.group(4).split(",")[-1].strip() == "1" else "step"
    return name if name in KERNEL_SOURCES else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(kernel_name):
    h = hashlib.sha256()
    for p in KERNEL_SOURCES[kernel_name]:
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
        if not rec or rec.get("source_hash") != kernel_source_hash(kernel_name) or rec.get("variant") != variant:
            return None
        return float(rec["hbm_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def cpu_info():
    """Host CPU model and the thread counts available to this process."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"model": model, "logical_cpus": os.cpu_count(), "cpus_in_affinity": affinity}


def cpu_baseline(itot, jtot, k_sample, seed, visc, min_reps=7, min_seconds=10.0, threads=None):
    """The CPU oracle (FP64, OpenMP over k) on a 512 x 512 x k_sample slab of
    the same field recipe; grid-points/s of one advec_u + diff_uvw pair,
    repeated until at least min_seconds of oracle work (and min_reps runs).
    threads: OpenMP threads (None = the OpenMP default, all host threads)."""
    import numpy as np

    import oracle
    from paper_2303_12374_amd import inputs
    lib = oracle.load()
    default_threads = lib.ora_threads()
    if threads is not None:
        lib.ora_set_threads(int(threads))
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
    while len(times) < min_reps or sum(times) < min_seconds:
        t0 = time.perf_counter()
        oracle.advec_u(g, tend[0], *host)
        oracle.diff_uvw(g, tend[0], tend[1], tend[2], *host, visc)
        times.append(time.perf_counter() - t0)
    best = float(np.median(times))
    used = lib.ora_threads()
    lib.ora_set_threads(default_threads)
    npts = itot * jtot * k_sample
    return {"value": npts / best, "unit": "grid-points/s", "cores": int(used), "kind": "oracle",
            "sample": f"{itot}x{jtot}x{k_sample} slab of the same recipe, FP64 oracle, one advec_u+diff_uvw "
                      f"pair, median of {len(times)} runs ({best:.3f} s each, {sum(times):.1f} s total)"}


def batched_leg(kl, inputs, torch, steps=10, warmup=3, tune_dir=None):
    """56 grids (48 with each axis from {32,64,96,128,192}, seed 3, plus 8 of
    256x256x32), FP32: one graph replay of the persistent tile-walking kernels
    of the fused advec_u + diff_uvw pass versus 56 x (advec_u + diff_uvw)
    single-grid launches (default and selected configurations) and 56
    single-grid fused launches."""
    import numpy as np
    shapes = inputs.batch_shapes(3)
    grids, fields = [], []
    for n, sh in enumerate(shapes):
        g = kl.Grid(*sh, dtype=kl.F32)
        f = [g.full(0.0) for _ in range(6)]
        kl.kl_generate_fields(g, 3000 + n, *f[:3])
        kl.kl_fill_ghosts(g, *f[:3])
        grids.append(g)
        fields.append(f)
    npts = sum(g.npoints for g in grids)
    b = kl.kl_batch_create(grids, fields, 1e-5, False)
    stream = torch.cuda.current_stream()
    tuned = None
    if tune_dir:
        tuned = kl.kl_batch_tune(b, tune_dir, 120.0, stream)
    nk, nt = kl.kl_batch_info(b)
    groups = kl.kl_batch_groups(b)

    def time_it(fn, k):
        settle_gpu(torch, fn)
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    batched_ms = time_it(lambda: kl.kl_batch_run(b, stream), steps)

    def plain():
        for g, f in zip(grids, fields):
            kl.kl_launch_variant(g, kl.ADVEC_U, 0, f, 1e-5, stream)
            kl.kl_launch_variant(g, kl.DIFF_UVW, 0, f, 1e-5, stream)

    def selected():
        for g, f in zip(grids, fields):
            kl.kl_advec_u(g, f[3], *f[:3], stream)
            kl.kl_diff_uvw(g, *f[3:], *f[:3], 1e-5, stream)

    def fused():
        for g, f in zip(grids, fields):
            kl.kl_advec_diff(g, *f[3:], *f[:3], 1e-5, stream)

    plain_ms = time_it(plain, max(3, steps // 2))
    sel_ms = time_it(selected, max(3, steps // 2))
    fused_ms = time_it(fused, max(3, steps // 2))
    kl.kl_batch_destroy(b)
    # the whole graph of the plan: ghost fill of every grid, tendencies := 0,
    # the fused pass, FP64 conservation sums of every grid
    sums = torch.zeros(3 * len(grids), dtype=torch.float64, device="cuda")
    flags = kl.BATCH_FILL_GHOSTS | kl.BATCH_ZERO_TENDENCIES | kl.BATCH_SUMS
    bf = kl.kl_batch_create_ex(grids, fields, 1e-5, flags, sums)
    nkf, _ = kl.kl_batch_info(bf)
    full_ms = time_it(lambda: kl.kl_batch_run(bf, stream), steps)
    kl.kl_batch_destroy(bf)
    del fields
    torch.cuda.empty_cache()
    return {"workload": "56 grids FP32 (48 x {32,64,96,128,192}^3 per axis, seed 3; 8 x 256x256x32)",
            "points": npts, "graph_kernels": nk, "tiles": nt,
            "configurations": [name for _, name, _ in groups],
            "tuned_now": None if tuned is None else
            {kl.kl_variant_name(kl.ADVEC_DIFF, kl.F32, i) if i >= 0 else "per_grid": ms for i, ms in tuned},
            "batched_ms": batched_ms, "batched_grid_points_per_s": npts / (batched_ms * 1e-3),
            "plain_112_launches_ms": plain_ms, "selected_112_launches_ms": sel_ms,
            "fused_56_launches_ms": fused_ms,
            "speedup_vs_plain": plain_ms / batched_ms, "speedup_vs_selected": sel_ms / batched_ms,
            "speedup_vs_fused_launches": fused_ms / batched_ms,
            "hbm_gbps_algorithmic": 9 * 4 * npts / (batched_ms * 1e6),
            "hbm_frac_of_peak": 9 * 4 * npts / (batched_ms * 1e6) / PEAK_HBM_GBPS,
            "bytes_note": "the graph runs the fused pass: 9 values per point (u, v, w, ut, vt, wt read; "
                          "ut, vt, wt written); the two separate kernels move 14",
            "hbm_gbps_14_value_equivalent": 14 * 4 * npts / (batched_ms * 1e6),
            "full_graph": {"steps": "ghost fill -> tendencies := 0 -> fused pass -> FP64 conservation sums",
                           "graph_kernels": nkf, "ms": full_ms,
                           "grid_points_per_s": npts / (full_ms * 1e-3)}}


def served_trace(n=2000, seed=4, rate=None):
    """Requests of the served workload: grids uniform over {64^3, 128^3, 256^3,
    512x512x128}, FP32 with probability 0.75 else FP64, 1..10 steps, Poisson
    arrivals (exponential gaps) -- all drawn from SplitMix64 counters of seed."""
    import numpy as np
    from paper_2303_12374_amd import inputs
    with np.errstate(over="ignore"):
        keys = inputs.field_key_base(seed, 6) + np.arange(4 * n, dtype=np.uint64)
        r = inputs.uniform01(keys).reshape(n, 4)
    shapes = [(64, 64, 64), (128, 128, 128), (256, 256, 256), (512, 512, 128)]
    reqs = []
    for q in range(n):
        sh = shapes[min(int(r[q, 0] * 4), 3)]
        dtype = 0 if r[q, 1] < 0.75 else 1
        steps = 1 + min(int(r[q, 2] * 10), 9)
        gap = -np.log1p(-r[q, 3])  # unit-rate exponential
        reqs.append({"shape": sh, "dtype": dtype, "steps": steps, "gap": gap, "seed": 40000 + q})
    return reqs


def served_leg(kl, torch, wisdom, n_req=2000, budget_gib=8.0, load=0.8, sweep=(0.5, 1.0, 1.2)):
    """Continuous batching server on the Poisson trace versus serial plain
    execution of the same trace; p50/p99 latency of (done - arrival), at the
    main offered load and at the loads of `sweep` (fractions of the served
    capacity)."""
    import threading
    import numpy as np
    reqs = served_trace(n_req)
    # calibrate the service rate: serial plain cost of one request of each kind
    cost = {}
    plain_dir = os.path.join("/tmp", "kl_empty_wisdom")
    kl.kl_set_wisdom_dir(plain_dir)
    stream = torch.cuda.current_stream()
    for sh in {r["shape"] for r in reqs}:
        for dt in (0, 1):
            g = kl.Grid(*sh, dtype=dt)
            f = [g.full(0.0) for _ in range(6)]
            kl.kl_generate_fields(g, 1, *f[:3])
            kl.kl_fill_ghosts(g, *f[:3])
            kl.kl_step(g, 1e-5, 1e-4, *f, stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(3):
                kl.kl_step(g, 1e-5, 1e-4, *f, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            cost[(sh, dt)] = e0.elapsed_time(e1) / 3 * 1e-3
            del f
    mean_service = float(np.mean([cost[(r["shape"], r["dtype"])] * r["steps"] for r in reqs]))
    serial_capacity = 1.0 / mean_service  # requests per second, serial plain
    kl.kl_set_wisdom_dir(wisdom)
    # served capacity: the first 400 requests of the trace submitted at once
    served_capacity = served_run(kl, torch, reqs[:400], np.zeros(400), budget_gib)["requests_per_s"]
    rate = load * served_capacity
    t_arr = np.cumsum([r["gap"] for r in reqs]) / rate
    pts_steps = sum(r["shape"][0] * r["shape"][1] * r["shape"][2] * r["steps"] for r in reqs)

    def serial(t_arr):
        """Serial plain execution of the trace (measured per-request costs)."""
        t_free, lat = 0.0, []
        for r, ta in zip(reqs, t_arr):
            start = max(ta, t_free)
            t_free = start + cost[(r["shape"], r["dtype"])] * r["steps"]
            lat.append(t_free - ta)
        return np.array(lat) * 1e3, t_free

    ls, serial_makespan = serial(t_arr)
    # the first requests of the same trace, at the same arrival times: serial
    # plain execution run on the GPU, and the server on exactly those requests
    n_pre = min(200, len(reqs))
    pre_serial = serial_plain_run(kl, torch, np, reqs[:n_pre], t_arr[:n_pre], plain_dir)
    kl.kl_set_wisdom_dir(wisdom)
    pre_served = served_run(kl, torch, reqs[:n_pre], t_arr[:n_pre], budget_gib)
    run = served_run(kl, torch, reqs, t_arr, budget_gib)
    # the same trace with a budget that never holds a request back (64 GiB
    # against a peak of about 9 GB in flight): what admission costs
    unl_gib = 64.0
    run_unl = served_run(kl, torch, reqs, t_arr, unl_gib)
    sweep_out = []
    for ld in sweep:
        ta = np.cumsum([r["gap"] for r in reqs]) / (ld * served_capacity)
        rr = served_run(kl, torch, reqs, ta, budget_gib)
        sl, _ = serial(ta)
        sweep_out.append({"load": ld, "p50_ms": rr["p50_ms"], "p99_ms": rr["p99_ms"],
                          "grid_point_steps_per_s": rr["grid_point_steps_per_s"],
                          "serial_plain_p50_ms": float(np.percentile(sl, 50)),
                          "serial_plain_p99_ms": float(np.percentile(sl, 99))})
    return {"workload": f"{n_req} requests, Poisson (seed 4) at {load:.1f} x the served capacity, grids "
                        "{64^3,128^3,256^3,512x512x128}, 75% FP32, 1-10 steps, budget "
                        f"{budget_gib:g} GiB",
            "arrival_rate_per_s": rate, "served_capacity_req_per_s": served_capacity,
            "serial_plain_capacity_req_per_s": serial_capacity,
            "p50_ms": run["p50_ms"], "p99_ms": run["p99_ms"], "mean_ms": run["mean_ms"],
            "grid_point_steps_per_s": run["grid_point_steps_per_s"], "makespan_s": run["makespan_s"],
            "ticks": run["ticks"], "launches": run["launches"], "peak_bytes": run["peak_bytes"],
            "serial_plain_simulated": {
                "p50_ms": float(np.percentile(ls, 50)), "p99_ms": float(np.percentile(ls, 99)),
                "grid_point_steps_per_s": pts_steps / serial_makespan, "makespan_s": serial_makespan,
                "method": "SIMULATED over the full trace: each request's plain kl_step time (measured per grid "
                          "and dtype) x steps, queued serially on the same arrival times; excludes set-up, "
                          "ghost fill, checksums and host synchronisation"},
            "prefix_measured": {
                "requests": n_pre,
                "serial_plain": dict(pre_serial, method="RUN on the GPU: per request, in arrival order after "
                                     "its arrival, allocate, generate, ghost fill, nsteps plain kl_step "
                                     "(default configurations), FP64 checksums, synchronise"),
                "served": {k: pre_served[k] for k in ("p50_ms", "p99_ms", "mean_ms", "grid_point_steps_per_s",
                                                        "makespan_s")},
                "arrivals": f"the first {n_pre} requests of the trace at the same arrival times"},
            "unlimited_budget": {"budget_gib": unl_gib,
                                 **{k: run_unl[k] for k in ("p50_ms", "p99_ms", "mean_ms", "grid_point_steps_per_s",
                                                            "makespan_s", "peak_bytes")}},
            "load_sweep": sweep_out}


def serial_plain_run(kl, torch, np, reqs, t_arr, plain_wisdom):
    """Serial plain execution of requests, run on the GPU (not simulated):
    in arrival order, once a request has arrived, the plain path does the
    work the server does for it -- allocate its six arrays, the seeded
    initial state (kl_generate_fields), ghost fill, nsteps kl_step with the
    default configurations, FP64 checksums -- and waits for it.  Latency is
    completion minus arrival, as for the server."""
    kl.kl_set_wisdom_dir(plain_wisdom)
    stream = torch.cuda.current_stream()
    cs = torch.zeros(9, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lat, first_arr, last_done = [], None, None
    base = time.perf_counter()
    for r, ta in zip(reqs, t_arr):
        while time.perf_counter() - base < ta:
            time.sleep(min(0.0005, max(0.0, ta - (time.perf_counter() - base))))
        g = kl.Grid(*r["shape"], dtype=r["dtype"], bc=kl.BC_ZWALL_ZEROGRAD)
        f = [torch.empty(g.alloc, dtype=g.tdtype, device="cuda") for _ in range(6)]
        kl.kl_generate_fields(g, r["seed"], *f[:3], stream)
        kl.kl_fill_ghosts(g, *f[:3], stream)
        for _ in range(r["steps"]):
            kl.kl_step(g, 1e-5, 1e-4, *f, stream)
        kl.kl_reduce_fp64(g, 1, *f[:3], cs, stream)
        stream.synchronize()
        done = time.perf_counter() - base
        lat.append((done - ta) * 1e3)
        first_arr = ta if first_arr is None else first_arr
        last_done = done
        del f, g
    pts_steps = sum(r["shape"][0] * r["shape"][1] * r["shape"][2] * r["steps"] for r in reqs)
    span = last_done - first_arr
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(np.mean(lat)), "grid_point_steps_per_s": pts_steps / span, "makespan_s": span}


def served_run(kl, torch, reqs, t_arr, budget_gib):
    """Submit reqs at times t_arr (s, from start) to a server and collect latencies."""
    import threading
    import numpy as np
    arena_bytes = int((budget_gib + 0.5) * (1 << 30))
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    srv = kl.kl_server_create(arena, arena_bytes, int(budget_gib * (1 << 30)))
    tickets = [None] * len(reqs)
    done = threading.Event()

    def client():
        base = time.perf_counter()
        for q, (r, ta) in enumerate(zip(reqs, t_arr)):
            while time.perf_counter() - base < ta:
                time.sleep(min(0.0005, max(0.0, ta - (time.perf_counter() - base))))
            sh = r["shape"]
            tickets[q] = kl.kl_submit(srv, sh[0], sh[1], sh[2], r["dtype"], 0, r["steps"], 1e-4, 1e-5, r["seed"])
        done.set()

    th = threading.Thread(target=client)
    wall0 = time.perf_counter()
    th.start()
    lat, first_arr, last_done = [], None, None
    pending = set()
    nxt = 0
    while len(lat) < len(reqs):
        while nxt < len(reqs) and tickets[nxt] is not None:
            pending.add(tickets[nxt])
            nxt += 1
        for tk in list(pending):
            rc, res = kl.kl_poll(srv, tk)
            if rc == kl.OK:
                if res.state != 2:
                    raise RuntimeError(f"served request {tk} failed: {res.err}")
                lat.append((res.t_done_ns - res.t_arrive_ns) * 1e-6)
                first_arr = res.t_arrive_ns if first_arr is None else min(first_arr, res.t_arrive_ns)
                last_done = res.t_done_ns if last_done is None else max(last_done, res.t_done_ns)
                kl.kl_release(srv, tk)
                pending.discard(tk)
        time.sleep(0.0002)
    th.join()
    wall = time.perf_counter() - wall0
    stats = kl.kl_server_stats(srv)
    kl.kl_server_destroy(srv)
    del arena
    torch.cuda.empty_cache()
    pts_steps = sum(r["shape"][0] * r["shape"][1] * r["shape"][2] * r["steps"] for r in reqs)
    span = (last_done - first_arr) * 1e-9
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(np.mean(lat)), "grid_point_steps_per_s": pts_steps / span, "makespan_s": span,
            "requests_per_s": len(reqs) / span, "wall_s": wall, "ticks": stats[0], "launches": stats[1],
            "peak_bytes": stats[3]}


STREAM_MIXES = {"r1w1 (copy)": (1, 1), "r2w1": (2, 1), "r3w3 (fused step)": (3, 3), "r4w1 (advec_u)": (4, 1),
                "r6w3 (diff_uvw)": (6, 3), "r7w3 (diff_smag)": (7, 3)}


def ceiling_leg(kl, torch, np, nbytes=1 << 29, reps=10):
    """HBM rate of plain streaming kernels (kl_stream_probe) in this process:
    the copy and each tendency kernel's read/write mix with no stencil, with
    cached and with non-temporal accesses; median of reps launches each.
    Arrays of nbytes (512 MiB) each: far beyond the 256 MB Infinity Cache."""
    bufs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(10)]
    for b in bufs:
        b.fill_(1)
    stream = torch.cuda.current_stream()
    out = {}
    for name, (nr, nw) in STREAM_MIXES.items():
        src, dst = bufs[:nr], bufs[nr:nr + nw]
        row = {}
        for nt in (False, True):
            for _ in range(2):
                kl.kl_stream_probe(src, dst, nbytes, nt, stream)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for e0, e1 in ev:
                e0.record(stream)
                kl.kl_stream_probe(src, dst, nbytes, nt, stream)
                e1.record(stream)
            torch.cuda.synchronize()
            ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
            row["nontemporal_gbps" if nt else "cached_gbps"] = (nr + nw) * nbytes / (ms * 1e6)
        row["best_gbps"] = max(row["cached_gbps"], row["nontemporal_gbps"])
        out[name] = row
    del bufs
    torch.cuda.empty_cache()
    return {"arrays_bytes": nbytes, "mixes": out, "copy_gbps": out["r1w1 (copy)"]["best_gbps"],
            "note": "kl_stream_probe: 16-byte accesses, 4 chunks per thread per pass, XOR of the sources "
                    "to every destination; no stencil and no reuse"}


def precision_leg(kl, torch, np, shape, host_fields, visc):
    """Normwise error of the FP32 path against the FP64 path on the whole
    grid: one advec_u + diff_uvw pair (selected configurations) on the same
    FP64 field recipe, in FP32 (fields, metrics and viscosity rounded to FP32)
    and in FP64.  The FP64 path is held to the FP64 oracle at 1e-12 by the
    parity tests, so this is the FP32 path's error against the oracle to
    that accuracy."""
    outs = {}
    for dtype in (kl.F32, kl.F64):
        g = kl.Grid(*shape, dtype=dtype, bc=kl.BC_ZWALL_ZEROGRAD)
        dev = [g.upload(f.astype(kl.NP_DTYPE[dtype])) for f in host_fields]
        kl.kl_fill_ghosts(g, *dev)
        t = [g.zeros_interior(fill=0.0) for _ in range(4)]
        kl.kl_advec_u(g, t[0], *dev)
        kl.kl_diff_uvw(g, t[1], t[2], t[3], *dev, visc)
        torch.cuda.synchronize()
        del dev
        outs[dtype] = (g, t)
    res = {}
    g32, t32 = outs[kl.F32]
    g64, t64 = outs[kl.F64]
    for n, name in enumerate(("advec_u", "diff_uvw_u", "diff_uvw_v", "diff_uvw_w")):
        a = g32.interior(t32[n]).to(torch.float64)
        b = g64.interior(t64[n])
        den = float(b.abs().max())
        a.sub_(b)
        res[name] = float(a.abs().max()) / den if den > 0 else float(a.abs().max())
        del a
    del outs, t32, t64
    torch.cuda.empty_cache()
    return {"normwise_rel_err": res, "max": max(res.values()),
            "definition": "max|f32 - f64| / max|f64| per output over the whole interior, both GPU paths on "
                          "the same FP64 sinusoid fields; the FP64 path meets the oracle to 1e-12",
            "grid": list(shape)}


def settle_gpu(torch, fn, min_ms=60.0, max_calls=200):
    """Run fn until at least min_ms of wall time has passed (at most
    max_calls calls): a leg that follows host-side work (field generation,
    oracle sums) otherwise starts timing while the GPU's clocks are still
    rising from idle, which measured up to 12% slow over the first ten
    calls of a 0.7 ms kernel."""
    import time as _t
    t0 = _t.perf_counter()
    for n in range(1, max_calls + 1):
        fn()
        if n % 4 == 0:
            torch.cuda.synchronize()
            if (_t.perf_counter() - t0) * 1e3 >= min_ms:
                break
    torch.cuda.synchronize()


def pair_leg(kl, torch, np, inputs, shape, dtype, recipe, seed, visc, steps, warmup=3):
    """advec_u + diff_uvw on one grid: the configurations selected from the
    wisdom files against the default (untuned) configurations, per-launch
    durations from HIP events on the launch stream."""
    g = kl.Grid(*shape, dtype=dtype, bc=kl.BC_ZWALL_ZEROGRAD)
    if recipe == "sinusoid":
        fs = inputs.sinusoid_fields(seed, *shape, g.zg)
    else:
        fs = inputs.random_fields(seed, *shape)
    dev = [g.upload(f.astype(kl.NP_DTYPE[dtype])) for f in fs]
    del fs
    kl.kl_fill_ghosts(g, *dev)
    tend = [g.zeros_interior(fill=0.0) for _ in range(3)]
    stream = torch.cuda.current_stream()
    s = 4 if dtype == kl.F32 else 8
    npts = shape[0] * shape[1] * shape[2]

    def run(adv_fn, dif_fn):
        settle_gpu(torch, lambda: (adv_fn(), dif_fn()))
        for _ in range(warmup):
            adv_fn()
            dif_fn()
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        for e in ev:
            e[0].record(stream)
            adv_fn()
            e[1].record(stream)
            dif_fn()
            e[2].record(stream)
        torch.cuda.synchronize()
        adv = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
        dif = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
        pair = float(np.mean([e[0].elapsed_time(e[2]) for e in ev]))
        return {"ms_per_pair": pair, "advec_u_ms": adv, "diff_uvw_ms": dif,
                "grid_points_per_s": npts / (pair * 1e-3), "hbm_gbps": 14 * s * npts / (pair * 1e6),
                "hbm_frac_of_peak": 14 * s * npts / (pair * 1e6) / PEAK_HBM_GBPS,
                "advec_u_gbps": 5 * s * npts / (adv * 1e6), "diff_uvw_gbps": 9 * s * npts / (dif * 1e6)}

    tuned = run(lambda: kl.kl_advec_u(g, tend[0], *dev, stream),
                lambda: kl.kl_diff_uvw(g, *tend, *dev, visc, stream))
    untuned = run(lambda: kl.kl_launch_variant(g, kl.ADVEC_U, 0, dev + tend, visc, stream),
                  lambda: kl.kl_launch_variant(g, kl.DIFF_UVW, 0, dev + tend, visc, stream))
    names = {n: kl.kl_variant_name(k, dtype, kl.kl_selected_variant(g, k))
             for n, k in (("advec_u", kl.ADVEC_U), ("diff_uvw", kl.DIFF_UVW))}
    del dev, tend
    torch.cuda.empty_cache()
    return {"workload": f"advec_u+diff_uvw {shape[0]}x{shape[1]}x{shape[2]} "
                        f"{'F32' if dtype == kl.F32 else 'F64'}, {recipe} fields seed {seed}, z walls, tanh z",
            "tuned": tuned, "untuned": untuned, "speedup_tuned_vs_untuned": untuned["ms_per_pair"] / tuned["ms_per_pair"],
            "configurations": names, "steps": steps}


def copy_probe(torch, nelem=1 << 27, reps=5):
    """A plain elementwise copy of known size (torch's multiply-by-one
    kernel: reads and writes nelem FP32 values), for scaling the HBM byte
    counters: FETCH_SIZE and WRITE_SIZE of one dispatch should each read
    4 * nelem bytes."""
    src = torch.ones(nelem, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 4 * nelem, "reps": reps}), flush=True)


def other_dtype_leg(kl, torch, np, shape, dtype, host_fields, visc, steps):
    """The advec_u + diff_uvw pair on the same grid and fields in the other
    precision, configurations selected from the wisdom files."""
    g = kl.Grid(*shape, dtype=dtype, bc=kl.BC_ZWALL_ZEROGRAD)
    s = 4 if dtype == kl.F32 else 8
    dev = [g.upload(f.astype(kl.NP_DTYPE[dtype])) for f in host_fields]
    kl.kl_fill_ghosts(g, *dev)
    tend = [g.zeros_interior(fill=0.0) for _ in range(3)]
    stream = torch.cuda.current_stream()
    settle_gpu(torch, lambda: (kl.kl_advec_u(g, tend[0], *dev, stream), kl.kl_diff_uvw(g, *tend, *dev, visc, stream)))
    for _ in range(3):
        kl.kl_advec_u(g, tend[0], *dev, stream)
        kl.kl_diff_uvw(g, *tend, *dev, visc, stream)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for e in ev:
        e[0].record(stream)
        kl.kl_advec_u(g, tend[0], *dev, stream)
        e[1].record(stream)
        kl.kl_diff_uvw(g, *tend, *dev, visc, stream)
        e[2].record(stream)
    torch.cuda.synchronize()
    adv = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    dif = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    pair = float(np.mean([e[0].elapsed_time(e[2]) for e in ev]))

    npts = shape[0] * shape[1] * shape[2]
    names = {n: kl.kl_variant_name(k, dtype, kl.kl_selected_variant(g, k))
             for n, k in (("advec_u", kl.ADVEC_U), ("diff_uvw", kl.DIFF_UVW))}
    del dev, tend
    torch.cuda.empty_cache()
    return {"dtype": "f64" if dtype == kl.F64 else "f32", "ms_per_pair": pair, "advec_u_ms": adv, "diff_uvw_ms": dif,
            "grid_points_per_s": npts / (pair * 1e-3), "hbm_gbps": 14 * s * npts / (pair * 1e6),
            "hbm_frac_of_peak": 14 * s * npts / (pair * 1e6) / PEAK_HBM_GBPS, "configurations": names,
            "steps": steps}


def les_leg(kl, torch, np, inputs, shape, host_fields, seed, steps):
    """The paper's own schemes on the same grid and fields: advec_u_2i5
    (fifth-order interpolated advection, three ghost cells in x and y) and
    diff_smag (stress divergence with a cell-center eddy viscosity), FP32,
    configurations selected from the wisdom files.  Algorithmic values per
    point: 5 (advection) and 10 (diffusion: u, v, w, evisc, ut, vt, wt read;
    ut, vt, wt written)."""
    g = kl.Grid(*shape, dtype=kl.F32, bc=kl.BC_ZWALL_ZEROGRAD, gc=3)
    dev = [g.upload(f.astype(np.float32)) for f in host_fields]
    dev.append(g.upload(inputs.evisc_field(seed, *shape).astype(np.float32)))
    kl.kl_fill_ghosts(g, *dev[:3])
    kl.kl_fill_scalar(g, dev[3])
    tend = [g.zeros_interior(fill=0.0) for _ in range(3)]
    stream = torch.cuda.current_stream()
    settle_gpu(torch, lambda: (kl.kl_advec_u_2i5(g, tend[0], *dev[:3], stream), kl.kl_diff_smag(g, *tend, *dev, stream)))
    for _ in range(3):
        kl.kl_advec_u_2i5(g, tend[0], *dev[:3], stream)
        kl.kl_diff_smag(g, *tend, *dev, stream)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for e in ev:
        e[0].record(stream)
        kl.kl_advec_u_2i5(g, tend[0], *dev[:3], stream)
        e[1].record(stream)
        kl.kl_diff_smag(g, *tend, *dev, stream)
        e[2].record(stream)
    torch.cuda.synchronize()
    adv = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    dif = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    pair = float(np.mean([e[0].elapsed_time(e[2]) for e in ev]))

    def alone(fn):
        """Mean duration of one kernel launched back to back (as the tuner
        times it), beside its duration inside the alternating pair above."""
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    adv_alone = alone(lambda: kl.kl_advec_u_2i5(g, tend[0], *dev[:3], stream))
    dif_alone = alone(lambda: kl.kl_diff_smag(g, *tend, *dev, stream))
    npts = shape[0] * shape[1] * shape[2]
    names = {n: kl.kl_variant_name(k, kl.F32, kl.kl_selected_variant(g, k))
             for n, k in (("advec_u_2i5", kl.ADVEC_U_2I5), ("diff_smag", kl.DIFF_SMAG))}
    b_adv, b_dif = 5 * 4 * npts, 10 * 4 * npts
    wkey = f"{shape[0]}x{shape[1]}x{shape[2]}_f32"
    del dev, tend
    torch.cuda.empty_cache()
    return {"workload": f"advec_u_2i5+diff_smag {shape[0]}x{shape[1]}x{shape[2]} F32, same fields, "
                        f"eddy viscosity 1e-3 (1 +- 0.5 noise), 3 ghost cells in x and y",
            "ms_per_pair": pair, "grid_points_per_s": npts / (pair * 1e-3),
            "hbm_gbps": (b_adv + b_dif) / (pair * 1e6),
            "hbm_frac_of_peak": (b_adv + b_dif) / (pair * 1e6) / PEAK_HBM_GBPS,
            "kernels": {"advec_u_2i5": {"ms": adv, "ms_back_to_back": adv_alone, "gbps": b_adv / (adv * 1e6),
                                        "frac": b_adv / (adv * 1e6) / PEAK_HBM_GBPS,
                                        "algorithmic_bytes_per_launch": b_adv,
                                        "traffic": load_traffic("advec_u_2i5", wkey, names["advec_u_2i5"])},
                        "diff_smag": {"ms": dif, "ms_back_to_back": dif_alone, "gbps": b_dif / (dif * 1e6),
                                      "frac": b_dif / (dif * 1e6) / PEAK_HBM_GBPS,
                                      "algorithmic_bytes_per_launch": b_dif,
                                      "traffic": load_traffic("diff_smag", wkey, names["diff_smag"])}},
            "configurations": names, "steps": steps}


def launch_overhead_leg(kl, torch, np, shape=(256, 256, 256), calls=200):
    """Host time of one kl_advec_u call: the first call for a problem size
    (reads the wisdom file, runs the selection heuristic, launches) and the
    mean of later calls (cached selection; launch only), as in the paper's
    measurement of its first and subsequent launches.  No runtime compilation
    is involved: every configuration is compiled ahead of time."""
    import time as _t
    g = kl.Grid(*shape, dtype=kl.F32)
    f = [g.full(0.0) for _ in range(4)]
    kl.kl_fill_ghosts(g, *f[:3])
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    firsts = []
    for _ in range(5):
        kl.kl_clear_plan_cache()
        t0 = _t.perf_counter()
        kl.kl_advec_u(g, f[3], *f[:3], stream)
        firsts.append(_t.perf_counter() - t0)
        torch.cuda.synchronize()
    t0 = _t.perf_counter()
    for _ in range(calls):
        kl.kl_advec_u(g, f[3], *f[:3], stream)
    later = (_t.perf_counter() - t0) / calls
    torch.cuda.synchronize()
    return {"grid": list(shape), "first_call_ms": 1e3 * float(np.median(firsts)),
            "later_call_us": 1e6 * later, "calls": calls,
            "note": "host time per call through the Python binding; the first call reads advec_u.wisdom"}


def summarize_counters(fetch_csv, write_csv, workload_key, out_json, out_txt, command, elem="float"):
    """Per-dispatch HBM bytes of the tendency kernels from two rocprofv3 --pmc
    runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what
    the same counter reads for the copy probe of known size."""
    import csv
    import statistics

    def per_kernel(path, counter):
        acc = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return acc

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    copy_name = [k for k in fetch if "MulFunctor" in k and len(fetch[k]) >= 5]
    nbytes = 4 << 27
    out = {}
    lines = [f"# HBM byte counters, {workload_key}", "", f"command: {command}", ""]
    if copy_name:
        cf = statistics.median(fetch[copy_name[0]]) * 1024
        cw = statistics.median(write[copy_name[0]]) * 1024
        fs, ws = nbytes / cf, nbytes / cw
        lines.append(f"copy probe ({nbytes} B): FETCH_SIZE reads {cf:.0f} B -> scale {fs:.3f}; "
                     f"WRITE_SIZE reads {cw:.0f} B -> scale {ws:.3f}")
    else:
        fs = ws = 1.0
        lines.append("copy probe not found: scale 1")
    lines.append("")
    lines.append("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) |")
    lines.append("|---|---|---|---|---|")
    for k in fetch:
        if "kl::" not in k or k not in write:
            continue
        f_kib = statistics.median(fetch[k])
        w_kib = statistics.median(write[k])
        hbm = f_kib * 1024 * fs + w_kib * 1024 * ws
        name = kernel_of_symbol(k)
        if name and (f"<{elem}," not in k or "_batch" in k or "_plain" in k):
            name = None
        lines.append(f"| `{k[:90]}` | {len(fetch[k])} | {f_kib:.0f} | {w_kib:.0f} | {hbm:.4g} |")
        if name:
            # a configuration that splits one call into several dispatches (one
            # kernel symbol each) is summed over its symbols: bytes per call
            rec = out.setdefault(f"{name}:{workload_key}", {"kernel_symbols": [], "fetch_kib": 0.0,
                                                            "write_kib": 0.0, "fetch_scale": fs,
                                                            "write_scale": ws, "hbm_bytes_per_launch": 0.0})
            rec["kernel_symbols"].append(k)
            rec["fetch_kib"] += f_kib
            rec["write_kib"] += w_kib
            rec["hbm_bytes_per_launch"] += hbm
    for key, rec in out.items():
        if len(rec["kernel_symbols"]) > 1:
            lines.append(f"| **{key.split(':')[0]}** (one call = {len(rec['kernel_symbols'])} dispatches) | | "
                         f"{rec['fetch_kib']:.0f} | {rec['write_kib']:.0f} | {rec['hbm_bytes_per_launch']:.4g} |")
    return out, "\n".join(lines) + "\n"


def summarize_trace(trace_csv, bench_json, command):
    """Markdown summary of a rocprofv3 kernel trace of a bench.py run: per
    dispatch durations of the kernels each timed leg selected, per call (a
    split configuration runs several dispatches per call), beside the HIP
    event times the same run reported."""
    import csv
    import statistics
    with open(bench_json) as f:
        line = json.loads([ln for ln in f if ln.startswith("{")][-1])
    durs = {}
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            durs.setdefault(r["Kernel_Name"], []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    grid = line["config"]["grid"]
    legs = [("advec_u", line["config"]["configurations"]["advec_u"], line["kernels"]["advec_u"]["ms"]),
            ("diff_uvw", line["config"]["configurations"]["diff_uvw"], line["kernels"]["diff_uvw"]["ms"])]
    if line.get("pair_fused"):
        legs.append(("advec_diff", line["pair_fused"]["configuration"], line["pair_fused"]["ms"]))
    if line.get("step"):
        legs.append(("step", line["step"]["fused_configuration"], line["step"]["fused_ms"]))
    for k in ("advec_u_2i5", "diff_smag"):
        if line.get("les"):
            legs.append((k, line["les"]["configurations"][k], line["les"]["kernels"][k]["ms_back_to_back"]))
    elem = "float" if line["dtype"] == "f32" else "double"
    out = [f"# Kernel trace: bench.py, {'x'.join(map(str, grid))} {line['dtype'].upper()} (MI355X)", "",
           f"command: `{command}`", "",
           "Per dispatch durations from the profiler (ns).  A call of a split configuration (zl3) is three",
           "dispatches, one per velocity component.  `bench ms` is the same run's mean per call from HIP events",
           "on the launch stream (the fifth-order kernels: back to back).", "",
           "| call | configuration | kernel symbol | dispatches | average ns | min ns | max ns |",
           "|---|---|---|---|---|---|---|"]
    summary = []
    for call, cfg, bench_ms in legs:
        syms = [s for s in durs if kernel_of_symbol(s) == call and f"<{elem}," in s and "_batch" not in s
                and "_plain" not in s]
        # the selected configuration's symbols: template arguments vx, by, kb (and the z-march order)
        try:
            parts = cfg.split("_")
            vx, by, kb, xcd = int(parts[1][1:]), int(parts[2].split("x")[1]), int(parts[3][1:]), int(parts[4][1:])
        except (IndexError, ValueError):
            continue  # the default configuration: no tile parameters to match
        pick = [s for s in syms if s.split("<", 1)[1].replace(" ", "").startswith(f"{elem},{vx},{by},{kb},{xcd},")]
        total = 0.0
        for s in pick:
            d = durs[s]
            out.append(f"| {call} | `{cfg}` | `{s[:80]}` | {len(d)} | {statistics.mean(d):.0f} | {min(d)} | {max(d)} |")
            total += statistics.mean(d)
        summary.append((call, cfg, total / 1e6, bench_ms))
    out += ["", "| call | configuration | trace ms per call | bench ms per call | trace / bench |", "|---|---|---|---|---|"]
    for call, cfg, tms, bms in summary:
        out.append(f"| {call} | `{cfg}` | {tms:.4f} | {bms:.4f} | {tms / bms if bms else float('nan'):.3f} |")
    if line.get("batched"):
        syms = [s for s in durs if "_batch<" in s and "step_zl_batch" in s]
        out += ["", "Batched form (one graph replay per call):", "",
                "| kernel symbol | dispatches | average ns |", "|---|---|---|"]
        for s in syms:
            out.append(f"| `{s[:90]}` | {len(durs[s])} | {statistics.mean(durs[s]):.0f} |")
        out.append(f"\nbench: {line['batched']['batched_ms']:.4f} ms per replay ({line['batched']['configurations']})")
    return "\n".join(out) + "\n"


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
    ap.add_argument("--tune-batch", action="store_true",
                    help="tune the batched workload as a whole first (kl_batch_tune; appends to --wisdom)")
    ap.add_argument("--tune-budget", type=float, default=60.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-k", type=int, default=128)
    ap.add_argument("--no-untuned", action="store_true")
    ap.add_argument("--no-other-dtype", action="store_true", help="skip the pair in the other precision")
    ap.add_argument("--no-les", action="store_true", help="skip the fifth-order advection + Smagorinsky pair")
    ap.add_argument("--no-overhead", action="store_true", help="skip the first-launch overhead measurement")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=2000)
    ap.add_argument("--no-ceiling", action="store_true", help="skip the streaming-probe ceilings")
    ap.add_argument("--no-precision", action="store_true", help="skip the FP32-vs-FP64 error of the pair")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 256^3 FP32/FP64 and 1024x1024x128 FP32 pair legs")
    ap.add_argument("--copy-probe", action="store_true", help="run only the copy probe used to scale counters")
    ap.add_argument("--with-copy-probe", action="store_true", help="run the copy probe first")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_CSV", "BENCH_JSON"),
                    help="write profiles/kernel_trace_bench_<grid>_<dtype>.md from a rocprofv3 --kernel-trace run "
                         "of bench.py and that run's JSON line (no GPU work)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON"),
                    help="write profiles/counters.json from two rocprofv3 --pmc runs of "
                         "'bench.py --with-copy-probe' and that run's JSON line (no GPU work)")
    args = ap.parse_args()

    if args.summarize_trace:
        itot, jtot, ktot = (int(x) for x in args.size.split(","))
        cmd = ("rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o trace -- python3 bench.py "
               "--no-cpu-baseline")
        txt = summarize_trace(args.summarize_trace[0], args.summarize_trace[1], cmd)
        with open(os.path.join(ROOT, "profiles", f"kernel_trace_bench_{itot}x{jtot}x{ktot}_{args.dtype}.md"), "w") as f:
            f.write(txt)
        print(txt)
        return

    if args.summarize_counters:
        itot, jtot, ktot = (int(x) for x in args.size.split(","))
        wkey = f"{itot}x{jtot}x{ktot}_{args.dtype}"
        cmd = ("rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -d <dir> -o bench -- python3 "
               "bench.py --with-copy-probe --steps 3 --warmup 1 --no-cpu-baseline --no-untuned --no-batched "
               "--no-served --no-other-dtype --no-overhead --no-precision --no-configs --no-ceiling")
        fetch_csv, write_csv, bench_json = args.summarize_counters
        out, txt = summarize_counters(fetch_csv, write_csv, wkey, None, None, cmd,
                                      "float" if args.dtype == "f32" else "double")
        with open(bench_json) as f:
            line = json.loads([ln for ln in f if ln.startswith("{")][-1])
        sel = dict(line["config"]["configurations"])
        sel.update((line.get("les") or {}).get("configurations", {}))
        if line.get("step"):
            sel["step"] = line["step"]["fused_configuration"]
        if line.get("pair_fused"):
            sel["advec_diff"] = line["pair_fused"]["configuration"]
        path = os.path.join(ROOT, "profiles", "counters.json")
        old = json.load(open(path)) if os.path.exists(path) else {}
        for k, v in out.items():
            if k.split(":")[0] not in sel:
                continue
            v["source_hash"] = kernel_source_hash(k.split(":")[0])
            v["variant"] = sel[k.split(":")[0]]
            old[k] = v
        json.dump(old, open(path, "w"), indent=1)
        with open(os.path.join(ROOT, "profiles", f"hbm_counters_{wkey}.md"), "w") as f:
            f.write(txt)
        print(txt)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent grids shard by grid, one process per GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe or args.with_copy_probe:
        copy_probe(torch)
        if args.copy_probe:
            return
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
    if args.no_other_dtype and args.no_les and args.no_precision:
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
        """Per-launch durations from HIP events recorded on the launch stream.
        The untimed clock settle (the GPU idles while the host generates the
        fields) comes before the warm-up steps; exactly `steps` pairs are timed."""
        settle_gpu(torch, lambda: (advec_fn(), diff_fn()))
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

    # the same pair as one fused pass (kl_advec_diff): bitwise the same
    # tendencies, 9 values per point moved instead of 14
    k_f = max(5, args.steps // 2)
    settle_gpu(torch, lambda: kl.kl_advec_diff(g, ut, vt, wt, u, v, w, visc, stream))
    for _ in range(2):
        kl.kl_advec_diff(g, ut, vt, wt, u, v, w, visc, stream)
    torch.cuda.synchronize()
    ev_f = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev_f[0].record(stream)
    for _ in range(k_f):
        kl.kl_advec_diff(g, ut, vt, wt, u, v, w, visc, stream)
    ev_f[1].record(stream)
    torch.cuda.synchronize()
    fused_ms = ev_f[0].elapsed_time(ev_f[1]) / k_f
    pair_fused = {"ms": fused_ms, "grid_points_per_s": npts / (fused_ms * 1e-3),
                  "hbm_gbps": 9 * npts * s / (fused_ms * 1e6),
                  "hbm_frac_of_peak": 9 * npts * s / (fused_ms * 1e6) / PEAK_HBM_GBPS,
                  "speedup_vs_separate_pair": ms_per_step / fused_ms,
                  "configuration": kl.kl_variant_name(kl.ADVEC_DIFF, dtype, kl.kl_selected_variant(g, kl.ADVEC_DIFF)),
                  "note": "advec_u then diff_uvw as one pass (kl_advec_diff), bitwise the separate kernels' "
                          "tendencies; 9 values per point (u, v, w, ut, vt, wt read, ut, vt, wt written)"}

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
                     "algorithmic_bytes_per_launch": dom_bytes,
                     "dispatches_per_launch": 3 if sel_names[dominant].startswith("zl3") else 1},
        "untuned": untuned,
        "pair_fused": pair_fused,
    }
    if not args.no_ceiling:
        log("streaming ceilings: copy and the kernels' read/write mixes")
        ceil = ceiling_leg(kl, torch, np)
        mixes = ceil["mixes"]
        ceil["kernel_frac_of_own_mix"] = {
            "advec_u": (bytes_adv / (adv_ms * 1e6)) / mixes["r4w1 (advec_u)"]["best_gbps"],
            "diff_uvw": (bytes_dif / (dif_ms * 1e6)) / mixes["r6w3 (diff_uvw)"]["best_gbps"]}
        ceil["kernel_frac_of_copy"] = {"advec_u": (bytes_adv / (adv_ms * 1e6)) / ceil["copy_gbps"],
                                       "diff_uvw": (bytes_dif / (dif_ms * 1e6)) / ceil["copy_gbps"],
                                       "pair": pair_gbps / ceil["copy_gbps"]}
        result["ceiling"] = ceil
        result["roofline"]["copy_ceiling_gbps"] = ceil["copy_gbps"]
        result["roofline"]["frac_of_copy_ceiling"] = achieved / ceil["copy_gbps"]
    if not args.no_precision:
        log("FP32 path against the FP64 path on the whole grid")
        result["precision"] = precision_leg(kl, torch, np, (itot, jtot, ktot), fs, visc)
    if not args.no_other_dtype:
        other = kl.F64 if dtype == kl.F32 else kl.F32
        log(f"the same pair in {'FP64' if other == kl.F64 else 'FP32'}")
        result["other_dtype"] = other_dtype_leg(kl, torch, np, (itot, jtot, ktot), other, fs, visc,
                                                max(5, args.steps // 2))
    if not args.no_les:
        log("the paper's schemes: advec_u_2i5 + diff_smag")
        result["les"] = les_leg(kl, torch, np, inputs, (itot, jtot, ktot), fs, seed, max(5, args.steps // 2))
    if not (args.no_other_dtype and args.no_les and args.no_precision):
        del fs
    # one time step: separate kernels (kl_step) versus the fused step kernel
    log("time step: kl_step (zero, advec_u, diff_uvw, Euler) vs kl_step_fused")
    out = [g.full() for _ in range(3)]
    dt_step = 1e-5

    def time_fn(fn, k=10):
        settle_gpu(torch, fn)
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    fused_ms = time_fn(lambda: kl.kl_step_fused(g, visc, dt_step, u, v, w, *out, stream))
    sep_ms = time_fn(lambda: kl.kl_step(g, visc, dt_step, u, v, w, ut, vt, wt, stream))
    result["step"] = {"fused_ms": fused_ms, "separate_ms": sep_ms, "speedup": sep_ms / fused_ms,
                      "fused_configuration": kl.kl_variant_name(kl.STEP, dtype, kl.kl_selected_variant(g, kl.STEP)),
                      "fused_grid_points_per_s": npts / (fused_ms * 1e-3),
                      "fused_hbm_gbps_6_values": 6 * s * npts / (fused_ms * 1e6),
                      "separate_hbm_gbps_26_values": 26 * s * npts / (sep_ms * 1e6)}
    # FP64 reductions over the same grid: conservation sums of the tendencies
    # and checksums of the fields (3 fields read each, accumulated in double)
    log("FP64 reductions: conservation sums and checksums")
    red = torch.zeros(9, dtype=torch.float64, device="cuda")
    cons_ms = time_fn(lambda: kl.kl_reduce_fp64(g, 0, ut, vt, wt, red, stream))
    chk_ms = time_fn(lambda: kl.kl_reduce_fp64(g, 1, u, v, w, red, stream))
    result["reductions"] = {"conservation_ms": cons_ms, "checksums_ms": chk_ms,
                            "conservation_hbm_gbps": 3 * s * npts / (cons_ms * 1e6),
                            "checksums_hbm_gbps": 3 * s * npts / (chk_ms * 1e6),
                            "note": "3 fields read per call (algorithmic bytes 3*N*s), sums in FP64"}
    del dev, tend, u, v, w, ut, vt, wt, out
    torch.cuda.empty_cache()
    if not args.no_configs:
        legs = {}
        for key, shape, dt, recipe, sd in (("256x256x256_f32", (256, 256, 256), kl.F32, "random", 1),
                                           ("256x256x256_f64", (256, 256, 256), kl.F64, "random", 1),
                                           ("1024x1024x128_f32", (1024, 1024, 128), kl.F32, "sinusoid", 2)):
            log(f"pair leg {key}: tuned vs untuned")
            legs[key] = pair_leg(kl, torch, np, inputs, shape, dt, recipe, sd, visc, max(5, args.steps // 2))
        result["configs"] = legs
    if not args.no_overhead:
        log("launch overhead: first call per problem size vs later calls")
        result["launch_overhead"] = launch_overhead_leg(kl, torch, np)
    if not args.no_batched:
        log("batched form: 56 grids in one graph vs 112 single-grid launches")
        result["batched"] = batched_leg(kl, inputs, torch, tune_dir=args.wisdom if args.tune_batch else None)
    if not args.no_served:
        log(f"served form: {args.served_requests} requests")
        result["served"] = served_leg(kl, torch, args.wisdom, args.served_requests)
        result["p99_latency_ms"] = result["served"]["p99_ms"]
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample (all host threads, then one thread)")
        cb = cpu_baseline(itot, jtot, args.cpu_sample_k, seed, float(np.float32(visc)))
        one = cpu_baseline(itot, jtot, args.cpu_sample_k, seed, float(np.float32(visc)), min_reps=3,
                           min_seconds=10.0, threads=1)
        cb["single_thread"] = {"value": one["value"], "cores": one["cores"], "sample": one["sample"]}
        cb["cpu"] = cpu_info()
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
