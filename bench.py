#!/usr/bin/env python3
"""Benchmark of the IMDP hot path on one MI355X.

One step = the whole path on one batch of synthetic input: build the
abstraction (bounds in HBM) and run interval iteration (both passes, to eps
or the sweep cap) for the workload's specification.  The default workload is
the largest single-GPU configuration: the 5D room safety system (10^5 cells,
4 inputs, rows of up to 3,127 entries, 50 sweeps per pass since its second
pass does not converge); the 3D unicycle reach-avoid system (50x50x24 cells,
20 inputs, eps 1e-8, run to convergence) is measured beside it under
``components``.

Prints one JSON line.  ``value`` is (state, input)-row LP updates per second
over the whole timed step (build included); the line also carries the bound
construction rate, the roofline of the dominant kernel (the policy-pass sweep,
timed with HIP events on the library's stream), a bounded served leg (p50 /
p99 latency and queries/s of the continuous-batching loop at a sustainable
arrival rate, against serial plain solves) and the CPU oracle timed on a
bounded sample of the same workload on one core and on all of the host's
cores (at most 16).  The storage mode and the per-pass entry order come from
the autotuner unless given.

``--forms`` adds the systems forms at full size, each against its plain
counterpart on the same GPU at the same eps:
  batched: seeded random 2D/3D linear instances built with one batch build
           and iterated together by the graph-captured engine, against a
           loop of plain build + iterate calls, one instance at a time;
  served : the Poisson request trace of the served configuration;
  disturbed: the disturbance player (the 2D robot with 11 disturbances).
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
    ap.add_argument("--workload", default="room5d",
                    choices=["unicycle3d", "robot2d", "room5d", "robot2d_correlated"])
    ap.add_argument("--components", default="unicycle3d,robot2d_correlated",
                    help="comma list of further workloads measured beside the headline one")
    ap.add_argument("--no-served", action="store_true",
                    help="skip the bounded served leg of the default line")
    ap.add_argument("--served-rate", type=float, default=1.0,
                    help="arrivals per second of the bounded served leg")
    ap.add_argument("--served-seconds", type=float, default=20.0,
                    help="length of the bounded served leg's trace")
    ap.add_argument("--served-max-sweeps", type=int, default=1000)
    ap.add_argument("--cpu-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--storage", default="tuned", choices=["tuned", "bounds", "factors"])
    ap.add_argument("--sweep-mode", default="tuned",
                    choices=["tuned", "auto", "per_row", "state_box"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="", help="comma list of: batched, served, disturbed")
    ap.add_argument("--dist-max-sweeps", type=int, default=5000,
                    help="sweep cap per pass of the disturbed form")
    ap.add_argument("--instances", type=int, default=384)
    ap.add_argument("--batch-max-sweeps", type=int, default=1000)
    ap.add_argument("--batch-horizon", default="0",
                    help='horizon of the batched queries: 0 (infinite, stop on eps) or "auto" '
                         "(Remark 5.2: self-convergence, then that many sweeps)")
    ap.add_argument("--batch-dims", default="2,3",
                    help="keep only the seeded instances of these dimensions")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-max-sweeps", type=int, default=1000)
    ap.add_argument("--tune-cache", default=None, help="JSON file for autotuner results")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (a known-size kernel "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


WORKLOADS = {
    "unicycle3d": "3D unicycle reach-avoid, 50x50x24 cells, 20 inputs, +-6 sigma windows, "
                  "eps 1e-8",
    "robot2d": "2D robot reach-avoid, 20x20 cells, 9 inputs, dense rows, eps 1e-8",
    "room5d": "5D room safety, 10^5 cells, 4 inputs, +-6 sigma windows, 50 sweeps per pass",
    "robot2d_correlated": "2D robot reach-avoid with correlated noise (Cov = 0.75 [[1, .5], "
                          "[.5, 1]]), 40x40 cells, 9 inputs, +-6 marginal sigma windows, "
                          "Monte Carlo cell masses (256 points, 2x2 candidate means, "
                          "3 standard errors), eps 1e-8",
}


def workload(name):
    """(system, spec, description, Monte Carlo noise or None) of a workload."""
    from paper_2401_03555_amd import workloads as W
    out = getattr(W, name)()
    system, spec = out[0], out[1]
    mc = out[2] if len(out) > 2 else None
    return system, spec, WORKLOADS[name], mc


def algorithmic_bytes(imdp, policy, n_states, d):
    """HBM bytes one policy-pass sweep must move (see the roofline notes).

    Per (SAFE state, input) row: the row's bounds -- 16 B per window cell
    (lo, hi) when stored, or 16 B per per-dimension factor (sum of the window
    widths) when recomputed -- + 32 B OUT/TAIL bounds + 8 B row offset + 8*d B
    window origin and widths.  Per SAFE state: 16 B (V0, V1) written + 4 B
    policy written + 4 B SAFE-list entry read.  Plus one read of the (V0, V1)
    vector, 16 B per cell; the per-entry value gathers re-read it from cache
    and are not counted.
    """
    info = imdp.info()
    nu = info["n_inputs"] * info.get("n_dist", 1)   # rows per state in the policy pass
    ex = imdp.export_rows(0, info["n_rows"], entries=False)
    safe = policy >= 0
    counts = ex["counts"].reshape(-1, nu)
    if info["storage"] == 2:
        counts = ex["win"][:, d:].sum(axis=1).reshape(-1, nu)
    cells = int(counts[safe].sum())
    rows = int(safe.sum()) * nu
    per_pass1 = 16 * cells + rows * (32 + 8 + 8 * d) + int(safe.sum()) * 24 + 16 * n_states
    return per_pass1, cells, rows


FP64_PEAK_TFLOPS = 78.6


# the sources each recorded kernel family is compiled from, besides the C
# header and the build flags
KERNEL_SOURCES = {
    "k_sweep_sb": [f"sweep_sb_d{d}.hip" for d in (0, 2, 3, 5)] + [
        "sweep_sb.hpp", "sweep_common.hpp", "impact_internal.hpp", "impact_device.hpp"],
    "k_sweep_sel": ["sweep_sel.hip", "sweep_common.hpp", "impact_internal.hpp",
                    "impact_device.hpp"],
    "k_mc_rows": ["build_mc.hip", "build_mc.hpp", "impact_internal.hpp", "impact_device.hpp"],
    "build": ["build.hip", "impact_internal.hpp", "impact_device.hpp"],
}


def kernel_source_hash(kernel="k_sweep_sb"):
    """Digest of what a kernel family is compiled from (its sources, the
    headers they include and the build flags), comments and blank space
    removed: identifies the build whose hardware counters are recorded under
    profiles/, and ignores edits to documentation only."""
    import hashlib
    import re
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2401_03555_amd")
    csrc = os.path.join(pkg, "csrc")
    names = KERNEL_SOURCES.get(kernel, KERNEL_SOURCES["k_sweep_sb"])
    files = [os.path.join(csrc, n) for n in names] + [
        os.path.join(ROOT, "include", "impact.h"), os.path.join(pkg, "build_lib.py")]
    for f in files:
        with open(f) as fh:
            text = fh.read()
        if not f.endswith(".py"):
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def _recorded(tag, field, kernel, storage, workload):
    """A per-launch figure of ``kernel`` recorded under profiles/ (lines
    ``<tag>: key=value ...``) for this kernel build, or None."""
    import glob
    src = kernel_source_hash(kernel)
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(f) as fh:
            for line in fh:
                if not line.startswith(tag + ":"):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:] if "=" in x)
                if (kv.get("kernel") == kernel and kv.get("storage") == storage
                        and kv.get("workload") == workload and kv.get("src") == src):
                    return float(kv[field])
    return None


def recorded_traffic(kernel, storage, workload):
    """HBM bytes per launch of ``kernel`` from the FETCH_SIZE / WRITE_SIZE
    summaries under profiles/ (lines ``traffic: ...``), or None."""
    v = _recorded("traffic", "bytes_per_launch", kernel, storage, workload)
    return None if v is None else int(v)


# wave64 VALU instructions per second the chip can issue: one per SIMD every
# 4 cycles, 1,024 SIMDs (256 CUs x 4), 2.4 GHz
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4


def recorded_valu(kernel, storage, workload):
    """Wave64 VALU instructions per launch of ``kernel`` from the SQ counter
    summary under profiles/ (lines ``valu: ...``), or None."""
    return _recorded("valu", "valu_per_launch", kernel, storage, workload)


def recorded_build_flops(storage, workload, kernel="build"):
    """FP64 operations per build (k_row_geom + k_expand, or the Monte Carlo
    entry kernel) counted by the SQ counters recorded under profiles/ (lines
    ``fp64: ...``), or None."""
    return _recorded("fp64", "flops_per_build", kernel, storage, workload)


def mc_build_roofline(imdp, d, mc, workload):
    """The Monte Carlo construction against the FP64 vector units that bind it.

    Evaluations: one density evaluation per (window cell, candidate mean,
    sample point).  The factored kernel (grids of at most 5 dimensions, at
    most 16 candidates) forms each evaluation as a product of d table entries
    that share prefixes across candidates, and adds it and its square to two
    running sums: algorithmic FP64 work d + 2 per evaluation (d - 1 products,
    one add, one fused multiply-add counted as 2), besides the per-point
    tables and the per-candidate epilogue.  The fraction of the FP64 vector
    peak uses the FP64 instructions counted by the SQ counters of this kernel
    build when they are recorded under profiles/.
    """
    info = imdp.info()
    ex = imdp.export_rows(0, info["n_rows"], entries=False)
    cells = int(ex["counts"].sum())
    n_cand = int(mc["grid_pts"]) ** d
    n_pts = len(mc["samples"])
    evals = cells * n_cand * n_pts
    t = info["build_ms"] * 1e-3
    per_eval = d + 2
    flops = recorded_build_flops("bounds", workload, "k_mc_rows")
    return {
        "kernels": "k_row_geom + scan + k_mc_prep + k_mc_rows",
        "bound": "alu",
        "build_ms": info["build_ms"],
        "entries_per_s": info["n_entries"] / t,
        "evaluations": evals,
        "evals_per_s": evals / t,
        "algorithmic_flops_per_eval": per_eval,
        "algorithmic_tflops": evals * per_eval / t / 1e12,
        "fp64_counted_tflops": None if flops is None else flops / t / 1e12,
        "fp64_frac": None if flops is None else flops / t / (FP64_PEAK_TFLOPS * 1e12),
        "peak_tflops": FP64_PEAK_TFLOPS,
    }


def build_roofline(imdp, d, workload):
    """Construction against its two ceilings.

    HBM: bytes the build must write -- per row 8*d B window + 32 B OUT/TAIL +
    8 B row offset, plus 16 B per entry (bounds storage) or 16 B per factor
    (sum of the window widths; factor storage).  FP64: the work the chosen
    storage performs -- the erfc evaluations at both ends of every window edge
    of every dimension (2 (W_i + 1) per dimension and row), and, with bounds
    storage only, the 2(d-1) multiplies that form each entry's (lo, hi) from
    its factors (factor storage leaves them to the sweeps) -- and, when the
    SQ counters of this build are recorded, the fraction of the FP64 vector
    peak they give.  Entries are counted as implied entries whatever the
    storage.
    """
    info = imdp.info()
    ex = imdp.export_rows(0, info["n_rows"], entries=False)
    cells = int(ex["counts"].sum())
    rows = info["n_rows"]
    widths = ex["win"][:, d:]
    fac = int(widths.sum())
    bounds = info["storage"] != 2
    payload = 16 * (cells if bounds else fac)
    nbytes = payload + rows * (8 * d + 32 + 8)
    t = info["build_ms"] * 1e-3
    products = 2 * max(0, d - 1) * cells if bounds else 0
    erfc = int(2 * (widths + 1).sum())
    storage = "bounds" if bounds else "factors"
    flops = recorded_build_flops(storage, workload)
    return {
        "kernels": "k_row_geom + scan + k_expand",
        "build_ms": info["build_ms"],
        "entries_per_s": info["n_entries"] / t,
        "hbm_bytes": nbytes,
        "hbm_gbs": nbytes / t / 1e9,
        "hbm_frac": nbytes / t / 1e9 / HBM_PEAK_GBS,
        "fp64_products": products,
        "erfc_evals": erfc,
        "erfc_per_s": erfc / t,
        "fp64_frac": None if flops is None else flops / t / (FP64_PEAK_TFLOPS * 1e12),
    }


# states of the bounded CPU-oracle sample per workload (about 10-15 s of
# single-core oracle work: its build of the sample's rows and one sweep of
# each pass over them)
CPU_SAMPLE_STATES = {"room5d": 12000, "unicycle3d": 30000, "robot2d": 400,
                     "robot2d_correlated": 200}


def cpu_worker(job):
    """Child process of cpu_baseline: the oracle on one shard of the sample.

    Builds the rows of states [s0, s1) and times one sweep of each pass over
    them (the states outside the shard are labelled unsafe and carry no rows,
    so every row the oracle solves is a row of the workload).
    """
    import numpy as np
    import oracle
    from paper_2401_03555_amd import workloads as W
    out = getattr(W, job["workload"])()
    system, spec = out[0], out[1]
    mc = out[2] if len(out) > 2 else None
    s0, s1 = job["states"]
    nu = len(system["inputs"])
    N = int(np.prod(system["n"]))
    states = np.arange(s0, s1, dtype=np.int64)
    rows = (states[:, None] * nu + np.arange(nu)[None, :]).ravel()
    t0 = time.perf_counter()
    if mc is not None:
        m = oracle.build_mc(system, mc, system["k_sigma"], rows=rows)
    else:
        m = oracle.build(system, system["k_sigma"], rows=rows)
    t_build = time.perf_counter() - t0
    counts = np.zeros(N * nu, dtype=np.int64)
    counts[rows] = np.diff(m["row_ptr"])
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    cls = np.full(N, 2, dtype=np.int8)   # outside the shard: unsafe, never swept
    cls[states] = 0
    t1 = time.perf_counter()
    r = oracle.iterate(N, nu, row_ptr, m["target"], m["lo"], m["hi"], cls, spec["kind"],
                       spec["eps"], 1)
    t_sweep = time.perf_counter() - t1
    n_safe = int(r["n_safe"])
    return {"build_s": t_build, "sweep_s": t_sweep, "entries": int(m["row_ptr"][-1]),
            "updates": n_safe * nu + n_safe}


def _run_workers(jobs):
    """Run cpu_worker jobs in concurrent child processes; (results, wall s)."""
    import subprocess
    t0 = time.perf_counter()
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker",
                               json.dumps(j)], stdout=subprocess.PIPE, text=True) for j in jobs]
    out = []
    for p in procs:
        o, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"oracle worker failed ({p.returncode})")
        out.append(json.loads(o.strip().splitlines()[-1]))
    return out, time.perf_counter() - t0


def cpu_baseline(workload):
    """The oracle as it stands on a bounded sample of the workload: one core,
    then the same sample split over all of the host's cores (at most 16), each
    shard in its own process."""
    from paper_2401_03555_amd import workloads as W
    system, _ = getattr(W, workload)()
    import numpy as np
    N = int(np.prod(system["n"]))
    S = min(N, CPU_SAMPLE_STATES.get(workload, 10000))
    s0 = (N - S) // 2                      # a block of states from the middle of the grid
    one, _ = _run_workers([{"workload": workload, "states": [s0, s0 + S]}])
    one = one[0]
    host = os.cpu_count() or 1
    P = max(1, min(16, host))
    cuts = [s0 + (S * k) // P for k in range(P + 1)]
    shards, wall = _run_workers([{"workload": workload, "states": [cuts[k], cuts[k + 1]]}
                                 for k in range(P)])
    upd = sum(x["updates"] for x in shards)
    sweep_wall = max(x["sweep_s"] for x in shards)
    build_wall = max(x["build_s"] for x in shards)
    return {
        "value": upd / sweep_wall,
        "unit": "(s,u)-updates/s",
        "cores": P,
        "kind": "oracle",
        "sample": (f"{S} of {N} states ({one['entries']} entries): oracle build of their rows, "
                   f"then one sweep of each pass over them; single core {one['build_s']:.1f} s "
                   f"+ {one['sweep_s']:.1f} s, {P} processes {build_wall:.1f} s + "
                   f"{sweep_wall:.1f} s"),
        "host_cores": host,
        "single_core": {"value": one["updates"] / one["sweep_s"], "cores": 1,
                        "build_entries_per_s": one["entries"] / one["build_s"]},
        "build_entries_per_s": sum(x["entries"] for x in shards) / build_wall,
    }


def _progress(label, every):
    state = {"last": 0}

    def cb(n, total):
        if n - state["last"] >= every or n == total:
            state["last"] = n
            print(f"# {label}: {n}/{total}", file=sys.stderr, flush=True)
    return cb


def run_batched(args, tuner):
    """Batched form vs a per-instance plain loop, same instances, eps and sweep cap."""
    import numpy as np
    import torch
    from paper_2401_03555_amd import impact, workloads as W
    dims = {int(x) for x in args.batch_dims.split(",")}
    insts = [x for x in W.batched(count=args.instances) if len(x[0]["n"]) in dims]
    systems = [s for s, _ in insts]
    hz = "auto" if args.batch_horizon == "auto" else int(args.batch_horizon)
    specs = [dict(spec, max_sweeps=args.batch_max_sweeps, horizon=hz) for _, spec in insts]
    # schedule choice (untimed): storage of the batch and engine graph chunk
    probe = impact.build_imdp_batch(systems, storage="factors")
    infos = [v.info() for v in probe]
    for v in probe:
        v.free()
    choice = tuner.choose_batch(systems, infos=infos)
    storage, chunk = choice["storage"], choice["chunk"]
    print(f"# batched: {len(systems)} instances, storage {storage}, chunk {chunk}",
          file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    views = impact.build_imdp_batch(systems, storage=storage)
    eng = impact.Engine(max_queries=len(views))
    ids = [eng.submit(v, sp) for v, sp in zip(views, specs)]
    res = {}
    t_print = time.perf_counter()
    while len(res) < len(ids):
        eng.run(chunk)
        for r in eng.poll():
            res[r["id"]] = r
        if time.perf_counter() - t_print > 15:
            t_print = time.perf_counter()
            print(f"# batched engine: {len(res)}/{len(ids)} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    eng.free()
    print(f"# batched done in {t_batched:.2f} s", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    worst = 0.0
    plain_updates = 0
    prog = _progress("plain loop", 32)
    for k, (system, sp) in enumerate(zip(systems, specs)):
        im = impact.build_imdp(system, storage=storage)
        r = im.iterate(sp)
        prog(k + 1, len(systems))
        plain_updates += sum(r["info"]["updates"])
        b = res[ids[k]]
        worst = max(worst, float((r["lo"] - b["lo"]).abs().max()),
                    float((r["hi"] - b["hi"]).abs().max()))
        im.free()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for v in views:
        v.free()
    updates = sum(sum(r["info"]["updates"]) for r in res.values())
    sweeps = np.array([r["info"]["sweeps"] for r in res.values()])
    return {
        "workload": (f"{len(systems)} of {args.instances} seeded random linear instances "
                     f"(dimensions {args.batch_dims}), reach-avoid, eps 1e-8, horizon "
                     f"{args.batch_horizon}, at most {args.batch_max_sweeps} sweeps per pass"),
        "instances": len(systems),
        "n_states": int(sum(i["n_states"] for i in infos)),
        "n_rows": int(sum(i["n_rows"] for i in infos)),
        "n_entries": int(sum(i["n_entries"] for i in infos)),
        "storage": storage, "chunk": chunk, "tuner": choice,
        "batched_s": t_batched, "plain_loop_s": t_plain,
        "speedup_vs_plain_loop": t_plain / t_batched,
        "batched_updates_per_s": updates / t_batched,
        "plain_updates_per_s": plain_updates / t_plain,
        "instances_per_s": len(systems) / t_batched,
        "converged": int(sum(r["status"] == 0 for r in res.values())),
        "self_converged": (int(sum(all(r["info"]["self_sweeps"][k] < args.batch_max_sweeps
                                       for k in (0, 1)) for r in res.values()))
                           if hz == "auto" else None),
        "sweeps_p50": [float(x) for x in np.percentile(sweeps, 50, axis=0)],
        "sweeps_max": [int(x) for x in sweeps.max(axis=0)],
        "max_abs_diff_vs_plain": worst,
    }


def run_disturbed(args):
    """The disturbance player (eq. (5.1)) on the 2D robot with 11 disturbances:
    build + iterate timed like the plain step; the per-row policy-pass sweep's
    roofline; the oracle on one sweep of each pass."""
    import numpy as np
    import torch
    import oracle
    from paper_2401_03555_amd import impact, workloads as W
    system, spec = W.robot2d_disturbed()
    spec = dict(spec, max_sweeps=args.dist_max_sweeps)

    def step(timing=False):
        imdp = impact.build_imdp(system, storage="bounds", timing=timing)
        return imdp, imdp.iterate(spec)

    imdp, r = step()
    imdp.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        imdp, r = step()
        imdp.free()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    imdp, r = step(timing=True)
    info, it = imdp.info(), r["info"]
    policy = r["policy"].cpu().numpy()
    bytes_sweep, cells, rows = algorithmic_bytes(imdp, policy, info["n_states"], info["dim"])
    launch_ms = it["launch_ms"][0] / max(1, it["launches"][0])
    achieved = bytes_sweep * it["sweeps"][0] / max(1, it["launches"][0]) / (launch_ms * 1e-3) / 1e9
    imdp.free()
    updates = sum(it["updates"])
    # the oracle, one sweep of each pass (bounded sample)
    m = oracle.build(system, system["k_sigma"])
    cls = oracle.label(system, spec["target"], spec["avoid"])
    t1 = time.perf_counter()
    ro = oracle.iterate(m["n_states"], len(system["inputs"]), m["row_ptr"], m["target"], m["lo"],
                        m["hi"], cls, spec["kind"], spec["eps"], 1, n_dist=info["n_dist"])
    t_o = time.perf_counter() - t1
    o_updates = int(ro["n_safe"]) * info["n_dist"] * (len(system["inputs"]) + 1)
    return {
        "workload": ("2D robot reach-avoid with a disturbance player: 20x20 cells, 9 inputs, "
                     "11 disturbances (drift along x in [-0.5, 0.5]), dense rows, eps 1e-8, "
                     f"at most {args.dist_max_sweeps} sweeps per pass"),
        "ms_per_step": ms,
        "value": updates / (ms * 1e-3),
        "unit": "(s,u,w)-row updates/s",
        "sweeps": list(it["sweeps"]),
        "converged": list(it["converged"]),
        "rows_per_sweep_pass1": rows,
        "roofline": {"kernel": ("k_sweep_sb" if info["max_box"] <= 512 and info["max_row"] <= 512
                                else "k_sweep") + " policy pass (all (u, w) rows per SAFE state)",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_sweep": bytes_sweep, "avg_launch_ms": launch_ms},
        "cpu_baseline": {"value": o_updates / t_o, "unit": "(s,u,w)-row updates/s", "cores": 1,
                         "kind": "oracle",
                         "sample": f"one sweep of each pass ({o_updates} row updates, {t_o:.1f} s)"},
        "vs_oracle": (updates / (ms * 1e-3)) / (o_updates / t_o),
    }


def run_served(args):
    """Served form vs serial plain solves over the same request trace."""
    import torch
    from paper_2401_03555_amd import serve, workloads as W
    pool = W.served_pool()
    trace = W.served_trace(pool, rate=args.serve_rate, duration=args.serve_seconds,
                           max_sweeps=args.serve_max_sweeps)
    budget = int(torch.cuda.mem_get_info()[0] * 0.5)
    # both legs start from an empty cache of the same budget
    cache = serve.AbstractionCache(pool, budget, storage="factors")
    srv = serve.Server(cache, max_active=64, steps=8)
    done, st = srv.run(trace, progress=_progress("served", 25))
    srv.free()
    served = serve.latency_stats(done, st["makespan"])
    served.update(peak_active=st["peak_active"], cache=cache.stats())
    cache.clear()
    print(f"# served: {served}", file=sys.stderr, flush=True)
    cache = serve.AbstractionCache(pool, budget, storage="factors")
    sdone, sst = serve.serve_serial(cache, trace, progress=_progress("serial", 25))
    serial = serve.latency_stats(sdone, sst["makespan"])
    serial.update(cache=cache.stats())
    cache.clear()
    return {
        "workload": (f"64-system pool (robot2d, unicycle3d, room5d variants, random linear), "
                     f"Poisson {args.serve_rate:g} req/s for {args.serve_seconds:g} s, "
                     f"safety/reach/reach-avoid, eps 1e-6/1e-8, at most "
                     f"{args.serve_max_sweeps} sweeps per pass"),
        "requests": len(trace),
        "served": served,
        "serial_plain": serial,
        "p99_speedup": serial["p99_ms"] / served["p99_ms"],
        "qps_ratio": served["qps"] / serial["qps"],
    }


def measured_peaks(impact, mib=1024, reps=5):
    """This device's copy bandwidth (a 1 GiB device-to-device copy, read +
    write bytes) and FP64 FMA rate (the library's probe kernel), measured
    outside the timed region; the roofline quotes the published peaks."""
    import torch
    src = torch.ones((mib << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    copy_gbs = 2.0 * src.numel() * 8 / (best * 1e-3) / 1e9
    del src, dst
    fp64 = impact.probe_fp64_fma()
    return {"copy_gbs": copy_gbs, "copy_frac_of_peak": copy_gbs / HBM_PEAK_GBS,
            "fp64_fma_tflops": fp64, "fp64_frac_of_peak": fp64 / 78.6}


def sweep_kernel_name(binfo, modes):
    """The kernel family of the policy-pass sweep for this abstraction."""
    if binfo["max_row"] > 512:
        return "k_sweep_sel"
    if modes[0] in ("state_box", "auto"):
        return "k_sweep_sb"
    return "k_sweep"


def measure_plain(args, tuner, name, steps, warmup):
    """Steps of one workload (build + iterate, timed as a whole) and the
    roofline of its policy-pass sweep from one instrumented step."""
    import torch
    from paper_2401_03555_amd import impact
    system, spec, desc, mc = workload(name)
    max_sweeps = spec["max_sweeps"]
    storage, modes, choice = args.storage, (args.sweep_mode, args.sweep_mode), None
    if mc is not None:
        # correlated noise: stored bounds only; the library's per-pass order
        storage = "bounds"
        modes = tuple("auto" if m == "tuned" else m for m in modes)
    elif "tuned" in (args.storage, args.sweep_mode):
        # measured per-sweep times, weighted by the sweeps each pass runs on
        # this query (from one untimed solve under the equal-weight choice)
        choice = tuner.choose(system)
        im = impact.build_imdp(system, storage=choice["storage"])
        im.set_sweep_modes(choice["policy_pass"], choice["fixed_pass"])
        sw = im.iterate(spec, max_sweeps=max_sweeps)["info"]["sweeps"]
        im.free()
        choice = tuner.choose(system, weights=sw)
        if args.storage == "tuned":
            storage = choice["storage"]
        if args.sweep_mode == "tuned":
            modes = (choice["policy_pass"], choice["fixed_pass"])
    print(f"# {name}: storage {storage}, sweep modes {modes}", file=sys.stderr, flush=True)

    def step(timing=False):
        if mc is not None:
            imdp = impact.build_imdp_mc(system, mc, timing=timing)
        else:
            imdp = impact.build_imdp(system, storage=storage, timing=timing)
        imdp.set_sweep_modes(*modes)
        r = imdp.iterate(spec, max_sweeps=max_sweeps)
        return imdp, r

    for _ in range(warmup):
        imdp, r = step()
        imdp.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        imdp, r = step()
        imdp.free()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / max(1, steps)

    # one instrumented step (HIP events around every sweep launch), outside the timed region
    imdp, r = step(timing=True)
    binfo, iinfo = imdp.info(), r["info"]
    policy = r["policy"].cpu().numpy()
    d = binfo["dim"]
    bytes_sweep, cells, rows = algorithmic_bytes(imdp, policy, binfo["n_states"], d)
    sweeps0, launches0 = iinfo["sweeps"][0], iinfo["launches"][0]
    avg_launch_ms = iinfo["launch_ms"][0] / max(1, launches0)
    achieved = bytes_sweep * sweeps0 / max(1, launches0) / (avg_launch_ms * 1e-3) / 1e9
    updates = sum(iinfo["updates"])
    kernel = sweep_kernel_name(binfo, modes)
    st_name = "bounds" if binfo["storage"] != 2 else "factors"
    out = {
        "workload": desc,
        "ms_per_step": ms_per_step,
        "value": updates / (ms_per_step * 1e-3),
        "config": {
            "workload": desc,
            "storage": storage,
            "sweep_modes": list(modes),
            "tuner": choice,
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
        "bound_entries_per_s": binfo["n_entries"] / (binfo["build_ms"] * 1e-3),
        "build_ms": binfo["build_ms"],
        "iter_updates_per_s": updates / (iinfo["iterate_ms"] * 1e-3),
        "iterate_ms": iinfo["iterate_ms"],
        "fixed_pass_launch_ms": iinfo["launch_ms"][1] / max(1, iinfo["launches"][1]),
        "build_roofline": (build_roofline(imdp, d, name) if mc is None
                           else mc_build_roofline(imdp, d, mc, name)),
        "roofline": {
            "kernel": kernel + " policy pass (all inputs per SAFE state)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": recorded_traffic(kernel, st_name, name),
            "bytes_per_sweep": bytes_sweep,
            "avg_launch_ms": avg_launch_ms,
            "launches": launches0,
            "sweeps": sweeps0,
            # what binds it instead: VALU issue, from the recorded SQ_INSTS_VALU
            # of this kernel build over the live launch time
            "valu_issue_frac": (lambda v: None if v is None else
                                v / (avg_launch_ms * 1e-3) / VALU_ISSUE_PEAK)(
                recorded_valu(kernel, st_name, name)),
        },
    }
    imdp.free()
    if mc is None and binfo["storage"] == 2:
        # the same sweep with stored bounds, whose bytes are the ones the HBM
        # roofline prices (factor storage trades them for VALU work)
        im2 = impact.build_imdp(system, storage="bounds", timing=True)
        im2.set_sweep_modes(*modes)
        r2 = im2.iterate(spec, max_sweeps=max_sweeps)
        i2 = r2["info"]
        b2, _, _ = algorithmic_bytes(im2, r2["policy"].cpu().numpy(), binfo["n_states"], d)
        l2 = i2["launch_ms"][0] / max(1, i2["launches"][0])
        a2 = b2 * i2["sweeps"][0] / max(1, i2["launches"][0]) / (l2 * 1e-3) / 1e9
        out["roofline"]["stored_bounds"] = {
            "achieved": a2, "frac": a2 / HBM_PEAK_GBS, "bytes_per_sweep": b2,
            "avg_launch_ms": l2, "traffic": recorded_traffic(kernel, "bounds", name),
            "valu_issue_frac": (lambda v: None if v is None else
                                v / (l2 * 1e-3) / VALU_ISSUE_PEAK)(
                recorded_valu(kernel, "bounds", name)),
        }
        im2.free()
    return out


def run_served_leg(args):
    """The bounded served leg of the default line: a short Poisson trace over
    the served pool at an arrival rate the GPU sustains, served by the
    continuous-batching loop and by serial plain solves."""
    a = argparse.Namespace(**vars(args))
    a.serve_rate, a.serve_seconds, a.serve_max_sweeps = (args.served_rate, args.served_seconds,
                                                         args.served_max_sweeps)
    return run_served(a)


def main():
    args = parse()
    if args.cpu_worker is not None:
        print(json.dumps(cpu_worker(json.loads(args.cpu_worker))), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding "
              "is a design note, not built", file=sys.stderr)
        return 2
    import torch
    from paper_2401_03555_amd import impact
    from paper_2401_03555_amd.autotune import Autotuner

    assert torch.cuda.is_available(), "no GPU visible"
    impact.lib()
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 20
        src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tuner = Autotuner(path=args.tune_cache)
    head = measure_plain(args, tuner, args.workload, args.steps, args.warmup)
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "(s,u)-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": head["config"],
        "components": {
            "bound_entries_per_s": head["bound_entries_per_s"],
            "build_ms": head["build_ms"],
            "iter_updates_per_s": head["iter_updates_per_s"],
            "iterate_ms": head["iterate_ms"],
            "fixed_pass_launch_ms": head["fixed_pass_launch_ms"],
            "served_p99_ms": None,
            "build_roofline": head["build_roofline"],
        },
        "roofline": head["roofline"],
    }
    for name in [c for c in args.components.split(",") if c and c != args.workload]:
        line["components"][name] = measure_plain(args, tuner, name, max(1, args.steps),
                                                 max(1, args.warmup))
    line["measured_peaks"] = measured_peaks(impact)
    if not args.no_served:
        leg = run_served_leg(args)
        line["components"]["served"] = leg
        line["components"]["served_p99_ms"] = leg["served"]["p99_ms"]
    forms = [f for f in args.forms.split(",") if f]
    if forms:
        line["forms"] = {}
    if "batched" in forms:
        line["forms"]["batched"] = run_batched(args, tuner)
    if "disturbed" in forms:
        line["forms"]["disturbed"] = run_disturbed(args)
    if "served" in forms:
        line["forms"]["served"] = run_served(args)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
