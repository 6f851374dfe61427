#!/usr/bin/env python3
"""Benchmark of the IMDP hot path on one MI355X.

One step = the whole path on one batch of synthetic input: build the
abstraction (bounds in HBM) and run interval iteration (both passes, to eps
or the sweep cap) for the workload's specification.  The default workload is
the 3D unicycle reach-avoid system (50x50x24 cells, 20 inputs, +-6 sigma
windows, eps 1e-8).

Prints one JSON line.  ``value`` is (state, input)-row LP updates per second
over the whole timed step (build included); the line also carries the bound
construction rate, the roofline of the dominant kernel (the policy-pass sweep,
timed with HIP events on the library's stream) and the CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IMDP bound entries/s; interval-iter (s,u)-updates/s; served p99 query latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="unicycle3d",
                    choices=["unicycle3d", "robot2d", "room5d"])
    ap.add_argument("--storage", default="bounds", choices=["bounds", "factors"])
    ap.add_argument("--sweep-mode", default="auto", choices=["auto", "per_row", "state_box"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def workload(name):
    from paper_2401_03555_amd import workloads as W
    system, spec = getattr(W, name)()
    desc = {
        "unicycle3d": "3D unicycle reach-avoid, 50x50x24 cells, 20 inputs, +-6 sigma windows, "
                      "eps 1e-8",
        "robot2d": "2D robot reach-avoid, 20x20 cells, 9 inputs, dense rows, eps 1e-8",
        "room5d": "5D room safety, 10^5 cells, 4 inputs, +-6 sigma windows, 50 sweeps per pass",
    }[name]
    return system, spec, desc


def algorithmic_bytes(imdp, policy, n_states, d):
    """HBM bytes one policy-pass sweep must move (see the roofline notes).

    Per (SAFE state, input) row: 16 B per window cell (lo, hi) + 32 B OUT/TAIL
    bounds + 8 B row offset + 8*d B window origin and widths.  Per SAFE state:
    16 B (V0, V1) written + 4 B policy written + 4 B SAFE-list entry read.
    Plus one read of the (V0, V1) vector, 16 B per cell; the per-entry value
    gathers re-read it from cache and are not counted.
    """
    import numpy as np
    info = imdp.info()
    nu = info["n_inputs"]
    counts = imdp.export_rows(0, info["n_rows"], entries=False)["counts"].reshape(-1, nu)
    safe = policy >= 0
    cells = int(counts[safe].sum())
    rows = int(safe.sum()) * nu
    per_pass1 = 16 * cells + rows * (32 + 8 + 8 * d) + int(safe.sum()) * 24 + 16 * n_states
    return per_pass1, cells, rows


def cpu_baseline(system, spec, budget_s=25.0):
    """The oracle as it stands, single-threaded, on a bounded sample."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    m = oracle.build(system, system["k_sigma"])
    t_build = time.perf_counter() - t0
    cls = oracle.label(system, spec["target"], spec["avoid"])
    t1 = time.perf_counter()
    r = oracle.iterate(m["n_states"], m["n_inputs"], m["row_ptr"], m["target"], m["lo"],
                       m["hi"], cls, spec["kind"], spec["eps"], 1)
    t_it = time.perf_counter() - t1
    n_safe = int(r["n_safe"])
    updates = n_safe * m["n_inputs"] + n_safe  # one sweep of each pass
    return {
        "value": updates / t_it,
        "unit": "(s,u)-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle build of all {m['row_ptr'].size - 1} rows "
                   f"({m['row_ptr'][-1]} entries, {t_build:.1f} s, "
                   f"{m['row_ptr'][-1] / t_build:.3g} entries/s) then one sweep of each pass "
                   f"({updates} updates, {t_it:.1f} s)"),
        "build_entries_per_s": m["row_ptr"][-1] / t_build,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding "
              "is a design note, not built", file=sys.stderr)
        return 2
    import numpy as np
    import torch
    from paper_2401_03555_amd import impact

    assert torch.cuda.is_available(), "no GPU visible"
    impact.lib()
    system, spec, desc = workload(args.workload)
    max_sweeps = spec["max_sweeps"]

    def step(timing=False):
        imdp = impact.build_imdp(system, storage=args.storage, timing=timing,
                                 sweep_mode=args.sweep_mode)
        r = imdp.iterate(spec, max_sweeps=max_sweeps)
        return imdp, r

    for _ in range(args.warmup):
        imdp, r = step()
        imdp.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        imdp, r = step()
        infos.append((imdp.info(), r["info"], r["status"]))
        imdp.free()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    # one instrumented step (HIP events around every kernel launch), outside the timed region
    imdp, r = step(timing=True)
    binfo, iinfo = imdp.info(), r["info"]
    policy = r["policy"].cpu().numpy()
    d = binfo["dim"]
    bytes_sweep, cells, rows = algorithmic_bytes(imdp, policy, binfo["n_states"], d)
    sweeps0, launches0 = iinfo["sweeps"][0], iinfo["launches"][0]
    avg_launch_ms = iinfo["launch_ms"][0] / max(1, launches0)
    achieved = bytes_sweep * sweeps0 / max(1, launches0) / (avg_launch_ms * 1e-3) / 1e9
    updates = sum(iinfo["updates"])
    value = updates / (ms_per_step * 1e-3)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "(s,u)-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "storage": args.storage,
            "sweep_mode": args.sweep_mode,
            "max_row": binfo["max_row"],
            "max_box": binfo["max_box"],
            "n_states": binfo["n_states"],
            "n_inputs": binfo["n_inputs"],
            "n_entries": binfo["n_entries"],
            "n_safe": iinfo["n_safe"],
            "sweeps": list(iinfo["sweeps"]),
            "converged": list(iinfo["converged"]),
            "status": r["status"],
        },
        "components": {
            "bound_entries_per_s": binfo["n_entries"] / (binfo["build_ms"] * 1e-3),
            "build_ms": binfo["build_ms"],
            "iter_updates_per_s": updates / (iinfo["iterate_ms"] * 1e-3),
            "iterate_ms": iinfo["iterate_ms"],
            "served_p99_ms": None,
        },
        "roofline": {
            "kernel": ("k_sweep_sb" if (args.sweep_mode != "per_row" and binfo["max_row"] <= 512)
                       else "k_sweep") + " policy pass (all inputs per SAFE state)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "bytes_per_sweep": bytes_sweep,
            "avg_launch_ms": avg_launch_ms,
            "launches": launches0,
            "sweeps": sweeps0,
        },
    }
    imdp.free()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(system, dict(spec))
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
