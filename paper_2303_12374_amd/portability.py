"""Performance-portability study of the tuned configurations (Section
"Experimental Evaluation": "Tuning Results" and "Performance Portability").

A *scenario* is one (kernel, grid size, precision) on this GPU.  For every
scenario the tuner measures every compiled configuration (kl_tune's
per-configuration timings).  From those timings this module derives what the
paper reports:

* per scenario, each configuration's performance as a fraction of the
  scenario's optimum (t_opt / t_cfg), a histogram of those fractions, the
  share of configurations within 10 % of the optimum, the default
  configuration's fraction, and the fraction reached by one fixed
  configuration C (the optimum of the first scenario);
* a matrix: the optimum of scenario A run in scenario B, as a fraction of
  B's optimum (a configuration that cannot run in B is replaced by the
  default configuration, which is what the library launches then);
* the performance-portability metric of Pennycook et al. (2016): for a
  configuration and a set of scenarios H, PPM = |H| / sum_{s in H} 1 / e_s,
  the harmonic mean of its efficiencies e_s, and 0 if any e_s is 0 (not
  supported); rows for the default configuration, for each scenario's
  optimum applied everywhere, and for runtime selection (always the
  scenario's own optimum, PPM 1).

The analysis functions take plain dictionaries and run on the CPU; only
``collect`` needs the GPU.

    python -m paper_2303_12374_amd.portability --out profiles/portability_mi355x \\
        --kernels advec_u,diff_uvw,advec_diff,advec_u_2i5,diff_smag \\
        --shapes 256x256x256,512x512x512,1024x1024x128 --dtypes f32,f64
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

BINS = [i / 10 for i in range(11)]  # fraction-of-optimum histogram edges 0.0 .. 1.0


# ---------------------------------------------------------------------------
# analysis (no GPU)
# ---------------------------------------------------------------------------

def scenario_key(kernel: str, shape, dtype: str) -> str:
    return f"{kernel}-{'x'.join(map(str, shape))}-{dtype}"


def fractions(times: dict) -> dict:
    """Fraction of the optimum t_opt / t for every configuration with a time."""
    ok = {c: t for c, t in times.items() if t is not None and t > 0}
    if not ok:
        return {}
    best = min(ok.values())
    return {c: best / t for c, t in ok.items()}


def optimum(times: dict) -> str:
    ok = {c: t for c, t in times.items() if t is not None and t > 0}
    return min(ok, key=lambda c: (ok[c], c))


def histogram(fr: dict, edges=BINS) -> list:
    """Counts of fractions per bin [e_i, e_i+1) (the last bin includes 1.0)."""
    counts = [0] * (len(edges) - 1)
    for f in fr.values():
        b = min(int(f * (len(edges) - 1)), len(edges) - 2)
        counts[b] += 1
    return counts


def efficiency(times: dict, config: str, default: str = "default") -> float:
    """Fraction of the optimum reached by `config` in a scenario; a
    configuration without a time there is replaced by the default one; 0 if
    neither ran."""
    fr = fractions(times)
    if config in fr:
        return fr[config]
    return fr.get(default, 0.0)


def ppm(effs) -> float:
    """Pennycook's metric: harmonic mean of the efficiencies, 0 if any is 0."""
    effs = list(effs)
    if not effs or any(e <= 0 for e in effs):
        return 0.0
    return len(effs) / sum(1.0 / e for e in effs)


def analyze(data: dict) -> dict:
    """data: {scenario key: {"kernel", "shape", "dtype", "times": {config: ms or None}}}."""
    keys = list(data)
    out = {"scenarios": {}, "matrix": {}, "ppm": {}}
    first = {}
    for k in keys:
        kern = data[k]["kernel"]
        first.setdefault(kern, k)
    for k in keys:
        t = data[k]["times"]
        fr = fractions(t)
        kern = data[k]["kernel"]
        c_conf = optimum(data[first[kern]]["times"])
        out["scenarios"][k] = {
            "kernel": kern, "shape": data[k]["shape"], "dtype": data[k]["dtype"],
            "configurations": len(t), "measured": len(fr), "optimum": optimum(t),
            "optimum_ms": min(v for v in t.values() if v is not None and v > 0),
            "default_fraction": efficiency(t, "default"),
            "within_10pct": sum(1 for f in fr.values() if f >= 0.9) / max(1, len(fr)),
            "histogram": histogram(fr), "config_C": c_conf, "config_C_fraction": efficiency(t, c_conf)}
    for kern in dict.fromkeys(data[k]["kernel"] for k in keys):
        ks = [k for k in keys if data[k]["kernel"] == kern]
        out["matrix"][kern] = {a: {b: efficiency(data[b]["times"], optimum(data[a]["times"])) for b in ks}
                               for a in ks}
        rows = {"(default configuration)": [efficiency(data[b]["times"], "default") for b in ks]}
        for a in ks:
            rows[a] = [out["matrix"][kern][a][b] for b in ks]
        rows["runtime selection"] = [1.0 for _ in ks]
        out["ppm"][kern] = {name: {"best": max(e), "worst": min(e), "ppm": ppm(e)} for name, e in rows.items()}
    return out


def report_markdown(rep: dict, meta: dict) -> str:
    L = [f"# Performance portability of the tuned configurations ({meta.get('device', '?')})", "",
         f"command: `{meta.get('command', '')}`", "",
         "Scenario = kernel-grid-precision on this GPU. Fractions are t_opt / t (1 = the scenario's optimum).",
         ""]
    L += ["## Per scenario", "",
          "| scenario | configs measured | optimum | optimum ms | within 10% | default | config C | C's fraction |",
          "|---|---|---|---|---|---|---|---|"]
    for k, s in rep["scenarios"].items():
        L.append(f"| {k} | {s['measured']}/{s['configurations']} | `{s['optimum']}` | {s['optimum_ms']:.4f} | "
                 f"{100 * s['within_10pct']:.1f}% | {s['default_fraction']:.2f} | `{s['config_C']}` | "
                 f"{s['config_C_fraction']:.2f} |")
    L += ["", "Histograms (share of configurations per fraction-of-optimum bin 0.0-0.1 ... 0.9-1.0):", ""]
    for k, s in rep["scenarios"].items():
        n = max(1, s["measured"])
        L.append(f"- {k}: " + " ".join(f"{100 * c / n:.0f}" for c in s["histogram"]))
    for kern, m in rep["matrix"].items():
        ks = list(m)
        L += ["", f"## Matrix: {kern} (row = scenario tuned for, column = scenario run)", "",
              "| tuned for \\ run | " + " | ".join(ks) + " |", "|---" * (len(ks) + 1) + "|"]
        for a in ks:
            L.append(f"| {a} | " + " | ".join(f"{m[a][b]:.2f}" for b in ks) + " |")
    for kern, rows in rep["ppm"].items():
        L += ["", f"## PPM: {kern}", "", "| configuration tuned for | best | worst | PPM |", "|---|---|---|---|"]
        for name, r in rows.items():
            L.append(f"| {name} | {r['best']:.2f} | {r['worst']:.2f} | {r['ppm']:.2f} |")
    return "\n".join(L) + "\n"


# ---------------------------------------------------------------------------
# collection (GPU)
# ---------------------------------------------------------------------------

def collect(kl, kernels, shapes, dtypes, budget=120.0, log=None) -> dict:
    """Every configuration's time in every scenario, through kl_tune (each
    kernel timed on its own, as the paper tunes captured launches one by
    one); records go to a scratch wisdom directory."""
    import torch
    names = {"advec_u": kl.ADVEC_U, "diff_uvw": kl.DIFF_UVW, "advec_u_2i5": kl.ADVEC_U_2I5,
             "diff_smag": kl.DIFF_SMAG, "advec_diff": kl.ADVEC_DIFF}
    bits = {kl.ADVEC_U: kl.TUNE_ADVEC_U, kl.DIFF_UVW: kl.TUNE_DIFF_UVW, kl.ADVEC_U_2I5: kl.TUNE_ADVEC_U_2I5,
            kl.DIFF_SMAG: kl.TUNE_DIFF_SMAG, kl.ADVEC_DIFF: kl.TUNE_ADVEC_DIFF}
    data = {}
    with tempfile.TemporaryDirectory() as tmp:
        for shape in shapes:
            for d in dtypes:
                dtype = kl.F32 if d == "f32" else kl.F64
                for gc in (1, 3):
                    ks = [n for n in kernels if (gc == 3) == (n in ("advec_u_2i5", "diff_smag"))]
                    if not ks:
                        continue
                    g = kl.Grid(*shape, dtype=dtype, bc=kl.BC_ZWALL_ZEROGRAD, gc=gc)
                    f = [g.full(0.0) for _ in range(7)]
                    kl.kl_generate_fields(g, 12345, *f[:3])
                    kl.kl_fill_ghosts(g, *f[:3])
                    f[6].fill_(1e-3)
                    for name in ks:
                        kern = names[name]
                        t0 = time.time()
                        res = kl.kl_tune(g, f, bits[kern], tmp, budget, max_timings=1024)
                        times = {kl.kl_variant_name(kern, dtype, i): (ms if ms > 0 else None) for i, ms in res}
                        key = scenario_key(name, shape, d)
                        data[key] = {"kernel": name, "shape": list(shape), "dtype": d, "times": times}
                        if log:
                            log(f"{key}: {len(times)} configurations in {time.time() - t0:.1f} s")
                    del f, g
                    torch.cuda.empty_cache()
    return data


def merge_collections(blobs):
    """Scenario tables of several collection runs on one device as one table
    (a later run's scenario replaces an earlier one of the same key); the
    commands are kept in order."""
    data, cmds = {}, []
    for b in blobs:
        data.update(b["data"])
        cmds.append(b["meta"].get("command", ""))
    meta = dict(blobs[0]["meta"])
    devices = {b["meta"].get("device") for b in blobs}
    if len(devices) > 1:
        raise SystemExit(f"collections from different devices: {sorted(map(str, devices))}")
    meta["command"] = " ; ".join(cmds)
    return data, meta


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True, help="output prefix: writes <out>.md and <out>.json")
    ap.add_argument("--kernels", default="advec_u,diff_uvw,advec_diff,advec_u_2i5,diff_smag")
    ap.add_argument("--shapes", default="256x256x256,512x512x512,1024x1024x128")
    ap.add_argument("--dtypes", default="f32,f64")
    ap.add_argument("--budget", type=float, default=120.0, help="seconds per scenario")
    ap.add_argument("--from-json", default="",
                    help="re-analyse collected JSON files (comma-separated, merged; no GPU)")
    a = ap.parse_args(argv)
    if a.from_json:
        data, meta = merge_collections([json.load(open(p)) for p in a.from_json.split(",")])
    else:
        from paper_2303_12374_amd import kl
        shapes = [tuple(int(x) for x in s.split("x")) for s in a.shapes.split(",")]
        log = lambda m: print(f"[portability] {m}", flush=True)
        data = collect(kl, a.kernels.split(","), shapes, a.dtypes.split(","), a.budget, log)
        import torch
        meta = {"device": torch.cuda.get_device_name(0), "arch": "gfx950",
                "command": "python -m paper_2303_12374_amd.portability " + " ".join(argv or sys.argv[1:]),
                "date": time.strftime("%Y-%m-%dT%H:%M:%SZ", time.gmtime())}
    rep = analyze(data)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out + ".json", "w") as f:
        json.dump({"meta": meta, "data": data, "report": rep}, f, indent=1)
    with open(a.out + ".md", "w") as f:
        f.write(report_markdown(rep, meta))
    return 0


if __name__ == "__main__":
    sys.exit(main())
