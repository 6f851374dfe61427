"""Autotuner for the schedule choices that do not change results beyond rounding.

Single abstractions: the storage mode (bounds stored once, or per-dimension
factors from which every sweep recomputes the bounds) and, per pass, the
entry order (one sort per row, or one sort per state over its rows' window
box).  Batches: the storage mode of the whole batch and the number of engine
steps captured in one graph launch.

Choices are measured -- a few sweeps of every candidate on the real
abstraction -- and cached under a shape key (device, dimension, input count,
row count, longest and mean row length, rounded to powers of two), in memory
and optionally in a JSON file, so one measurement serves every later system of
that shape.

The first sweeps of a pass cost more than the later ones (the selection
sweep's per-row hints start cold), so each candidate is timed over two probe
lengths: the mean of the short probe prices the first TUNE_SWEEPS sweeps of a
pass, and the extra sweeps of the long probe price every later one.
"""
import json
import math
import os
import time

import numpy as np

from . import impact

TUNE_SWEEPS = 6
TUNE_SWEEPS_LONG = 16
MODES = ("state_box", "per_row")
CHUNKS = (8, 16, 32, 64)


def _b(x):
    return int(round(math.log2(max(1.0, float(x)))))


def _device():
    import torch
    return torch.cuda.get_device_name(0).replace(" ", "_")


def _probe_spec(d, sweeps):
    # every in-domain state is SAFE: the largest amount of work per sweep
    return dict(kind="safety", target=[], avoid=[], eps=1e-300, max_sweeps=sweeps)


def imdp_key(info):
    mean_row = info["n_entries"] / max(1, info["n_rows"])
    return (f"{_device()}/d{info['dim']}/u{info['n_inputs']}/r{_b(info['n_rows'])}"
            f"/m{_b(info['max_row'])}/e{_b(mean_row)}/w{int(info['windowed'])}")


def _bounds_bytes(info):
    # the entry table of the bounds storage: one (lo, hi) pair per entry
    return 16 * info["n_entries"]


class Autotuner:
    def __init__(self, path=None, budget_bytes=None, sweeps=TUNE_SWEEPS, long=TUNE_SWEEPS_LONG):
        self.path = path
        self.sweeps = sweeps
        self.long = long
        self.budget = budget_bytes
        self.table = {}
        self.log = []
        if path and os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    def _save(self):
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)

    def _budget(self):
        if self.budget is not None:
            return self.budget
        import torch
        return int(torch.cuda.mem_get_info()[0] * 0.5)

    def _time_modes(self, imdp, d):
        """Per entry order (rows beyond 512 entries sweep by selection whatever
        the order: one measurement): the mean ms per sweep of each pass over
        its first sweeps, then the ms per sweep of each pass after them."""
        imdp.set_timing(True)
        out = {}
        modes = MODES if imdp.info()["max_row"] <= 512 else MODES[:1]
        for mode in modes:
            imdp.set_sweep_modes(mode, mode)
            imdp.iterate(_probe_spec(d, 1))          # first-use costs out of the timing
            i1 = imdp.iterate(_probe_spec(d, self.sweeps))["info"]
            i2 = imdp.iterate(_probe_spec(d, max(self.long, self.sweeps)))["info"]
            start, later = [], []
            for p in (0, 1):
                t1, n1 = float(i1["sweep_ms"][p]), int(i1["sweeps"][p])
                t2, n2 = float(i2["sweep_ms"][p]), int(i2["sweeps"][p])
                start.append(t1 / max(1, n1))
                # a pass that stopped before the long probe's cap, or timing
                # noise beyond the difference: later sweeps priced as the first
                later.append((t2 - t1) / (n2 - n1) if n2 > n1 and t2 > t1 else start[-1])
            out[mode] = tuple(start + later)
        for mode in MODES:
            out.setdefault(mode, out[modes[0]])
        imdp.set_timing(False)
        return out

    def _pass_ms(self, t, p, w):
        """Predicted ms of ``w`` sweeps of pass ``p`` from a measurement ``t``:
        (first0, first1, later0, later1), or (ms0, ms1) for every sweep."""
        first = t[p]
        later = t[2 + p] if len(t) >= 4 else first
        k = min(w, float(self.sweeps))
        return k * first + (w - k) * later

    def choose(self, system, weights=(1.0, 1.0)):
        """The tuned choice for ``system``: storage and per-pass sweep modes.

        The measured per-sweep times of the two passes are weighted by
        ``weights``, the sweeps each pass is expected to run (e.g. the counts
        of an earlier solve of the same query; equal by default)."""
        probe = impact.build_imdp(system, storage="factors")
        info = probe.info()
        key = imdp_key(info)
        cached = key in self.table
        if cached:
            probe.free()
            measured = self.table[key]["measured"]
        else:
            d = info["dim"]
            cands = {"factors": self._time_modes(probe, d)}
            probe.free()
            if _bounds_bytes(info) <= self._budget():
                im = impact.build_imdp(system, storage="bounds")
                cands["bounds"] = self._time_modes(im, d)
                im.free()
            measured = {s: {m: list(v) for m, v in t.items()} for s, t in cands.items()}
            self.table[key] = {"measured": measured}
            self.log.append((key, measured))
            self._save()
        w0, w1 = (float(x) for x in weights)
        best = None
        for storage, t in measured.items():
            p1 = min(MODES, key=lambda m: self._pass_ms(t[m], 0, w0))
            p2 = min(MODES, key=lambda m: self._pass_ms(t[m], 1, w1))
            c0, c1 = self._pass_ms(t[p1], 0, w0), self._pass_ms(t[p2], 1, w1)
            if best is None or c0 + c1 < best["weighted_ms"]:
                best = dict(storage=storage, policy_pass=p1, fixed_pass=p2, weighted_ms=c0 + c1,
                            ms_per_sweep=[c0 / max(w0, 1e-30), c1 / max(w1, 1e-30)])
        return dict(best, weights=[w0, w1], measured=measured, key=key, cached=cached)

    def build(self, system, **kw):
        """Build ``system`` with its tuned storage and sweep modes."""
        c = self.choose(system)
        im = impact.build_imdp(system, storage=c["storage"], **kw)
        im.set_sweep_modes(c["policy_pass"], c["fixed_pass"])
        return im, c

    # ---- batches ---------------------------------------------------------
    def batch_key(self, infos):
        rows = sum(i["n_rows"] for i in infos)
        mx = max(i["max_row"] for i in infos)
        dims = sorted({i["dim"] for i in infos})
        return (f"{_device()}/batch/n{_b(len(infos))}/r{_b(rows)}/m{_b(mx)}"
                f"/d{'-'.join(map(str, dims))}")

    def _sample(self, systems, sample):
        rows = np.array([np.prod(s["n"]) * len(s["inputs"]) for s in systems], dtype=float)
        order = np.argsort(-rows)
        big = list(order[: sample // 2])
        rest = [int(i) for i in order[sample // 2:]]
        rng = np.random.default_rng(0)
        pick = big + list(rng.choice(rest, size=min(len(rest), sample - len(big)), replace=False))
        return [systems[int(i)] for i in pick]

    def _time_batch(self, systems, storage, chunk, steps):
        import torch
        views = impact.build_imdp_batch(systems, storage=storage)
        eng = impact.Engine(max_queries=len(views))
        for v in views:
            eng.submit(v, _probe_spec(v.info()["dim"], 10 ** 6))
        eng.run(chunk)                                  # capture + first use
        torch.cuda.synchronize()
        t = time.perf_counter()
        done = 0
        while done < steps:
            eng.run(chunk)
            done += chunk
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / done
        eng.free()
        for v in views:
            v.free()
        return ms

    def choose_batch(self, systems, infos=None, sample=16, steps=64):
        """Storage and graph chunk for an engine run over ``systems``.

        ``infos`` (abstraction infos of the whole batch, if already built)
        only feed the key; the measurement runs on a sample: the largest
        instances by row count and seeded random others.
        """
        sub = self._sample(systems, min(sample, len(systems)))
        if infos is None:
            views = impact.build_imdp_batch(sub, storage="factors")
            infos = [v.info() for v in views]
            for v in views:
                v.free()
        key = self.batch_key(infos)
        if key in self.table:
            return dict(self.table[key], key=key, cached=True)
        res = {}
        for storage in ("factors", "bounds"):
            if storage == "bounds":
                est = sum(_bounds_bytes(i) for i in infos)
                if est > self._budget():
                    continue
            res[storage] = {c: self._time_batch(sub, storage, c, steps) for c in CHUNKS}
        storage, chunk = min(((s, c) for s in res for c in res[s]), key=lambda sc: res[sc[0]][sc[1]])
        best = dict(storage=storage, chunk=int(chunk), ms_per_step=res[storage][chunk],
                    measured={s: {str(c): v for c, v in t.items()} for s, t in res.items()})
        self.table[key] = best
        self.log.append((key, best))
        self._save()
        return dict(best, key=key, cached=False)
