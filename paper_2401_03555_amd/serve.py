"""Serving form: a request loop over the multi-query engine.

Requests (system key, specification, eps) arrive over time.  Abstractions stay
resident in HBM in a cache keyed by system and are built on a miss; least
recently used entries that no running query holds are evicted to keep the
cache within its byte budget.  A request is admitted when a query slot is free
and HBM allows it: its abstraction is resident, or the budget left after
evicting idle entries covers its expected size (the exact size once the
system has been built before, else the mean size of those built so far).
Admitted queries run together -- every engine step advances all queries of
one size class by one sweep, classes share the GPU by time -- and new ones
join between steps (continuous batching).  Latency is completion time minus
arrival time.

The serial baseline serves the same trace one request at a time with the
plain single-query call, from a cache with the same budget.
"""
import collections
import time

import numpy as np

from . import impact


def _query_bytes(imdp):
    # value and output vectors the engine allocates per query
    n = imdp.info()["n_states"]
    return n * (8 * 4 + 4 * 3 + 8)


class AbstractionCache:
    """Built abstractions keyed by system, LRU-evicted within a byte budget."""

    def __init__(self, systems, budget_bytes, storage="bounds"):
        self.systems = systems
        self.budget = int(budget_bytes)
        self.storage = storage
        self.entries = collections.OrderedDict()  # key -> (imdp, bytes)
        self.sizes = {}                           # key -> bytes, for every build
        self.entries_of = {}                      # key -> entries per sweep
        self.pins = collections.Counter()
        self.used = 0
        self.hits = self.misses = self.evictions = 0
        self.build_s = 0.0

    def resident(self, key):
        return key in self.entries

    def pinned_bytes(self):
        return sum(b for k, (_, b) in self.entries.items() if self.pins[k] > 0)

    def expected_bytes(self, key):
        if key in self.sizes:
            return self.sizes[key]
        return int(np.mean(list(self.sizes.values()))) if self.sizes else 0

    def fits(self, key, extra=0):
        """True if ``key`` can be made resident beside the pinned entries."""
        if key in self.entries:
            return True
        return self.pinned_bytes() + extra + self.expected_bytes(key) <= self.budget

    def _evict_for(self, need):
        for key in list(self.entries):
            if self.used + need <= self.budget:
                break
            if self.pins[key] > 0:
                continue
            imdp, nbytes = self.entries.pop(key)
            imdp.free()
            self.used -= nbytes
            self.evictions += 1

    def acquire(self, key):
        if key in self.entries:
            self.entries.move_to_end(key)
            self.pins[key] += 1
            self.hits += 1
            return self.entries[key][0]
        self._evict_for(self.expected_bytes(key))
        t = time.perf_counter()
        imdp = impact.build_imdp(self.systems[key], storage=self.storage)
        self.build_s += time.perf_counter() - t
        info = imdp.info()
        nbytes = info["device_bytes"]
        self.sizes[key] = nbytes
        self.entries_of[key] = info["n_entries"]
        self.entries[key] = (imdp, nbytes)
        self.used += nbytes
        self.pins[key] += 1
        self._evict_for(0)
        self.misses += 1
        return imdp

    def release(self, key):
        self.pins[key] -= 1
        if self.used > self.budget:
            self._evict_for(0)

    def clear(self):
        for imdp, _ in self.entries.values():
            imdp.free()
        self.entries.clear()
        self.used = 0

    def stats(self):
        return dict(hits=self.hits, misses=self.misses, evictions=self.evictions,
                    build_s=self.build_s, resident_bytes=self.used, budget_bytes=self.budget)


class _Lane:
    def __init__(self, max_active):
        self.engine = impact.Engine(max_queries=max_active)
        self.max_active = max_active
        self.active = {}       # engine query id -> request
        self.used_s = 0.0      # GPU time given to this lane
        self.step_s = 1e-3     # running estimate of one engine step


class Server:
    """Continuous-batching request loop with size classes.

    Queries are sorted into lanes by the size of their abstraction (entries
    per sweep): small, medium and large, one engine each.  Within a lane,
    every engine step advances all of its queries by one sweep; across lanes,
    GPU time is shared fairly: the lane that has had the least time runs next,
    for about ``slice_ms`` of steps.  So a small query is not slowed to the
    pace of the largest ones beside it (every query of one engine advances one
    sweep per step, whatever its size), and large queries still progress.
    Admission is in arrival order per lane, by free slots and free HBM.
    """

    BOUNDS = (1 << 22, 1 << 26)  # entries: small below the first, large above the second

    def __init__(self, cache, max_active=64, steps=8, slice_ms=25.0, lanes=3):
        self.cache = cache
        self.max_active = max_active
        self.steps = steps
        self.slice_s = slice_ms * 1e-3
        self.lanes = [_Lane(max_active) for _ in range(lanes)]

    def lane_of(self, n_entries):
        k = sum(n_entries > b for b in self.BOUNDS)
        return min(k, len(self.lanes) - 1)

    def _known_entries(self, key):
        return self.cache.entries_of.get(key)

    def run(self, trace, keep_outputs=False, progress=None):
        """Serve ``trace`` (dicts with arrival ``t`` in seconds, ``key``, ``spec``).

        ``progress(n_done, n_total)`` is called whenever requests complete."""
        t0 = time.perf_counter()
        i, queue, done = 0, [], []
        query_bytes = 0
        peak = 0

        def n_active():
            return sum(len(ln.active) for ln in self.lanes)

        while i < len(trace) or queue or n_active():
            now = time.perf_counter() - t0
            while i < len(trace) and trace[i]["t"] <= now:
                queue.append(dict(trace[i], idx=i))
                i += 1
            # admission in arrival order, per lane, by free slots and free HBM
            blocked = set()
            keep = []
            for req in queue:
                n = self._known_entries(req["key"])
                lane = self.lane_of(n) if n is not None else 0
                if lane in blocked or len(self.lanes[lane].active) >= self.max_active:
                    blocked.add(lane)
                    keep.append(req)
                    continue
                if n_active() and not self.cache.fits(req["key"], query_bytes):
                    blocked.add(lane)
                    keep.append(req)
                    continue
                imdp = self.cache.acquire(req["key"])
                actual = self.lane_of(imdp.info()["n_entries"])
                if actual != lane and len(self.lanes[actual].active) >= self.max_active:
                    self.cache.release(req["key"])
                    blocked.add(actual)
                    keep.append(req)
                    continue
                ln = self.lanes[actual]
                if not ln.active:  # a lane that wakes up starts level with the others
                    busy = [x.used_s for x in self.lanes if x.active]
                    ln.used_s = min(busy) if busy else 0.0
                qid = ln.engine.submit(imdp, req["spec"])
                req["t_admit"] = time.perf_counter() - t0
                req["bytes"] = _query_bytes(imdp)
                query_bytes += req["bytes"]
                ln.active[qid] = req
            queue = keep
            peak = max(peak, n_active())
            live = [ln for ln in self.lanes if ln.active]
            if live:
                ln = min(live, key=lambda x: x.used_s)
                steps = int(min(64, max(1, round(self.slice_s / ln.step_s))))
                t = time.perf_counter()
                ln.engine.run(steps)
                dt = time.perf_counter() - t
                ln.used_s += dt
                ln.step_s = 0.5 * ln.step_s + 0.5 * dt / steps
                t_now = time.perf_counter() - t0
                for r in ln.engine.poll():
                    req = ln.active.pop(r["id"])
                    self.cache.release(req["key"])
                    query_bytes -= req["bytes"]
                    rec = dict(idx=req["idx"], key=req["key"], t=req["t"],
                               t_admit=req["t_admit"], t_done=t_now, latency=t_now - req["t"],
                               info=r["info"], status=r["status"])
                    if keep_outputs:
                        rec.update(lo=r["lo"], hi=r["hi"], policy=r["policy"])
                    done.append(rec)
                    if progress:
                        progress(len(done), len(trace))
            elif i < len(trace):
                time.sleep(max(0.0, trace[i]["t"] - (time.perf_counter() - t0)))
        makespan = time.perf_counter() - t0
        done.sort(key=lambda d: d["idx"])
        return done, dict(makespan=makespan, peak_active=peak)

    def free(self):
        for ln in self.lanes:
            ln.engine.free()


def serve_serial(cache, trace, keep_outputs=False, progress=None):
    """Baseline: one request at a time with the plain single-query call."""
    t0 = time.perf_counter()
    done = []
    for idx, req in enumerate(trace):
        now = time.perf_counter() - t0
        if req["t"] > now:
            time.sleep(req["t"] - now)
        t_admit = time.perf_counter() - t0
        imdp = cache.acquire(req["key"])
        r = imdp.iterate(req["spec"])
        t_done = time.perf_counter() - t0
        cache.release(req["key"])
        rec = dict(idx=idx, key=req["key"], t=req["t"], t_admit=t_admit, t_done=t_done,
                   latency=t_done - req["t"], info=r["info"], status=r["status"])
        if keep_outputs:
            rec.update(lo=r["lo"], hi=r["hi"], policy=r["policy"])
        done.append(rec)
        if progress:
            progress(len(done), len(trace))
    return done, dict(makespan=time.perf_counter() - t0)


def latency_stats(done, makespan):
    lat = np.array([d["latency"] for d in done]) * 1e3
    return dict(n=len(done), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
                qps=len(done) / makespan, makespan_s=makespan,
                not_converged=int(sum(d["status"] != 0 for d in done)))
