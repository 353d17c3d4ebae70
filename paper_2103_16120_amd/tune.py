"""Per-workload choice, by measurement, of the launch options that change
only speed: member groups on two streams or the whole batch on one stream,
and graph replay of the iterations (results are bitwise the same under every
choice).

    python -m paper_2103_16120_amd.tune [--steps 5]

times the benchmark batch (64 x 512x256), 64 x 1024x512 and the uneven
64-member batch in the float64 and the mixed half-precision-preconditioner
forms under the four combinations, and writes the fastest per workload to
paper_2103_16120_amd/_tuned.json (per machine, not versioned), keyed by
tune_key().  lib.Solver(..., tuned=True) applies the stored choice for its
workload and the defaults when none is stored.
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED_FILE = os.path.join(HERE, "_tuned.json")
CHOICES = [(False, False), (True, False), (False, True), (True, True)]   # (one_stream, graph)


def tune_key(sizes, precision):
    """Workload key: the precision form and the histogram of member sizes
    (member order does not matter)."""
    hist = collections.Counter((int(nx), int(ny)) for nx, ny in sizes)
    return f"{int(precision)}:" + ",".join(f"{nx}x{ny}*{n}" for (nx, ny), n in sorted(hist.items()))


def tuned_options(sizes, precision, path=None):
    """{"one_stream": bool, "graph": bool} stored for this workload, or the
    defaults (member groups, no graphs) when the file or the key is absent."""
    try:
        with open(TUNED_FILE if path is None else path) as fh:
            rec = json.load(fh).get(tune_key(sizes, precision))
    except (OSError, ValueError):
        rec = None
    if not rec:
        return {"one_stream": False, "graph": False}
    return {"one_stream": bool(rec.get("one_stream")), "graph": bool(rec.get("graph"))}


def _time(lib, torch, sizes, depth, dts, rhs, precision, one_stream, graph, steps):
    s = lib.Solver(sizes, precision=precision, rtol=1e-8, one_stream=one_stream, graph=graph)
    xs = [torch.zeros_like(r) for r in rhs]
    members = list(range(len(sizes)))

    def step():
        s.set_operators(members, depth, dts)
        for x in xs:
            x.zero_()
        s.solve(rhs, xs)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    s.close()
    return ms


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--steps", type=int, default=5)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    from paper_2103_16120_amd import lib
    from workloads import problem, batch_problems
    workloads = {
        "bench 64 x 512x256": [problem(2, 512, 256, instance=m, dt=600.0) for m in range(64)],
        "bench 64 x 1024x512": [problem(2, 1024, 512, instance=m, dt=100.0) for m in range(64)],
        "uneven 64": batch_problems(3, 64),
    }
    try:
        with open(TUNED_FILE) as fh:
            table = json.load(fh)
    except (OSError, ValueError):
        table = {}
    for name, probs in workloads.items():
        sizes = [(p["nx"], p["ny"]) for p in probs]
        depth = [torch.from_numpy(p["depth"]).cuda() for p in probs]
        dts = [p["dt"] for p in probs]
        f = lib.Solver(sizes, precision=lib.FP64)
        f.set_operators(list(range(len(probs))), depth, dts)
        rhs = [f.apply_operator(m, torch.from_numpy(p["x_true"]).cuda()) for m, p in enumerate(probs)]
        f.close()
        for precision in (lib.FP64, lib.MIXED_HALF_PC):
            ms = {f"one_stream={o},graph={g}": round(_time(lib, torch, sizes, depth, dts, rhs, precision, o, g,
                                                             args.steps), 4)
                  for o, g in CHOICES}
            best = min(CHOICES, key=lambda c: ms[f"one_stream={c[0]},graph={c[1]}"])
            table[tune_key(sizes, precision)] = {"workload": name, "precision": int(precision),
                                                 "one_stream": best[0], "graph": best[1], "ms": ms}
            print(json.dumps(table[tune_key(sizes, precision)]), flush=True)
    with open(TUNED_FILE, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
