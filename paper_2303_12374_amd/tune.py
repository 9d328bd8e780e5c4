"""Tuning command line: measure every compiled configuration of advec_u and
diff_uvw for a list of grid shapes and dtypes on this GPU and append the
best ones to the wisdom files (the tune step of the capture -> tune ->
wisdom -> select flow; Section "Kernel Tuning").

Fields are the library's seeded initial state (kl_generate_fields): stencil
timings do not depend on the field values.

    python -m paper_2303_12374_amd.tune --wisdom wisdom \\
        --shapes 512x512x512,256x256x256 --dtypes f32,f64 --budget 60
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def parse_shape(s: str):
    parts = [int(x) for x in s.lower().split("x")]
    if len(parts) != 3:
        raise argparse.ArgumentTypeError(f"bad shape {s!r}")
    return tuple(parts)


def tune_shape(kl, shape, dtype, wisdom, budget, bc=0, log=None):
    import torch
    g = kl.Grid(*shape, dtype=dtype, bc=bc)
    f = [g.full(0.0) for _ in range(6)]
    kl.kl_generate_fields(g, 12345, *f[:3])
    kl.kl_fill_ghosts(g, *f[:3])
    out = {}
    kl.kl_set_wisdom_dir(wisdom)
    for kern, name in ((kl.ADVEC_U, "advec_u"), (kl.DIFF_UVW, "diff_uvw"), (kl.STEP, "step")):
        t0 = time.time()
        # diff_uvw is timed after the advec_u just tuned (it follows it in a step)
        mask = (1 << kern) | (8 if kern == kl.DIFF_UVW else 0)
        res = kl.kl_tune(g, f, mask, wisdom, budget)
        ok = [(ms, i) for i, ms in res if ms > 0]
        best_ms, best = min(ok)
        default_ms = dict((i, ms) for i, ms in res).get(0, float("nan"))
        out[name] = {"best": kl.kl_variant_name(kern, dtype, best), "ms": best_ms, "default_ms": default_ms,
                     "evaluated": len(res), "bitwise_failures": len(res) - len(ok), "seconds": time.time() - t0}
        if log:
            log(f"{name} {'x'.join(map(str, shape))} {'f32' if dtype == kl.F32 else 'f64'}: "
                f"{out[name]['best']} {best_ms:.4f} ms (default {default_ms:.4f} ms, "
                f"{len(res)} configurations)")
    del f
    torch.cuda.synchronize()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--wisdom", required=True, help="wisdom directory (records are appended)")
    ap.add_argument("--shapes", required=True, help="comma-separated IxJxK shapes")
    ap.add_argument("--dtypes", default="f32,f64")
    ap.add_argument("--budget", type=float, default=60.0, help="seconds per kernel and shape")
    ap.add_argument("--json", default="", help="write a summary here")
    a = ap.parse_args(argv)
    from paper_2303_12374_amd import kl
    log = lambda m: print(f"[tune] {m}", flush=True)
    summary = []
    for s in a.shapes.split(","):
        shape = parse_shape(s)
        for d in a.dtypes.split(","):
            dtype = kl.F32 if d == "f32" else kl.F64
            summary.append({"shape": shape, "dtype": d, **tune_shape(kl, shape, dtype, a.wisdom, a.budget, log=log)})
    if a.json:
        with open(a.json, "w") as f:
            json.dump(summary, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
