"""Host logic of the served form: cache eviction, pinning, admission sizing and
the request trace generator (no GPU; construction is replaced by a stub)."""
import numpy as np
import pytest

from paper_2401_03555_amd import serve, workloads as W


class _Stub:
    def __init__(self, nbytes, log):
        self.nbytes, self.log, self.freed = nbytes, log, False

    def info(self):
        return dict(device_bytes=self.nbytes, n_states=10, n_entries=self.nbytes * 4)

    def free(self):
        self.freed = True
        self.log.append(self)


@pytest.fixture
def cache(monkeypatch):
    log = []
    sizes = {"a": 100, "b": 200, "c": 300, "d": 50}
    monkeypatch.setattr(serve.impact, "build_imdp",
                        lambda system, storage="bounds": _Stub(sizes[system], log))
    c = serve.AbstractionCache({k: k for k in sizes}, budget_bytes=450)
    c.log = log
    return c


def test_cache_hits_and_lru_eviction(cache):
    a = cache.acquire("a")
    cache.release("a")
    assert cache.acquire("a") is a and (cache.hits, cache.misses) == (1, 1)
    cache.release("a")
    cache.acquire("b"); cache.release("b")
    cache.acquire("a"); cache.release("a")  # a is now most recent
    cache.acquire("c"); cache.release("c")  # 600 > 450: evict LRU (b)
    assert set(cache.entries) == {"a", "c"} and cache.used == 400
    assert cache.evictions == 1 and cache.log[0].nbytes == 200


def test_pinned_entries_are_not_evicted(cache):
    cache.acquire("b")
    cache.acquire("c")            # 500 > 450 but both pinned
    assert set(cache.entries) == {"b", "c"} and cache.used == 500
    assert not cache.fits("a")    # pinned 500 + expected (mean 250) > 450
    cache.release("b")            # over budget: the idle entry goes now
    assert set(cache.entries) == {"c"} and cache.used == 300
    assert cache.fits("c") and not cache.fits("a")   # 300 + 250 > 450
    cache.release("c")
    assert cache.fits("a") and set(cache.entries) == {"c"}


def test_expected_size_of_unbuilt_systems(cache):
    assert cache.expected_bytes("a") == 0
    cache.acquire("b"); cache.release("b")
    cache.acquire("d"); cache.release("d")
    assert cache.expected_bytes("c") == 125      # mean of the built sizes
    assert cache.expected_bytes("b") == 200
    cache.acquire("b")
    assert not cache.fits("c", extra=200)        # 200 pinned + 200 + 125 > 450
    assert cache.fits("c", extra=100)


def test_cache_records_entries_and_lanes(cache):
    cache.acquire("c")
    cache.release("c")
    assert cache.entries_of == {"c": 1200}
    # lane choice by entries per sweep (no GPU: the class method only)
    lane_of = serve.Server.lane_of
    fake = type("S", (), {"BOUNDS": serve.Server.BOUNDS, "lanes": [0, 1, 2]})()
    assert lane_of(fake, 1000) == 0
    assert lane_of(fake, (1 << 22) + 1) == 1
    assert lane_of(fake, 1 << 30) == 2


def test_served_trace_shape():
    pool = W.served_pool()
    assert len(pool) == 64
    tr = W.served_trace(pool, rate=200.0, duration=5.0, seed=1)
    assert 850 <= len(tr) <= 1150
    ts = np.array([r["t"] for r in tr])
    assert np.all(np.diff(ts) > 0) and ts[-1] < 5.0
    gaps = np.diff(np.concatenate([[0.0], ts]))
    assert abs(gaps.mean() - 1 / 200) < 0.15 / 200
    kinds = [r["spec"]["kind"] for r in tr]
    assert {kinds.count(k) for k in ("safety", "reach", "reach_avoid")} and len(set(kinds)) == 3
    for r in tr:
        s, spec = pool[r["key"]], r["spec"]
        assert spec["eps"] in (1e-6, 1e-8)
        assert bool(spec["target"]) == (spec["kind"] != "safety")
        assert bool(spec["avoid"]) == (spec["kind"] != "reach")
        lb, ub, n = (np.asarray(s[k], float) for k in ("lb", "ub", "n"))
        for box in spec["target"] + spec["avoid"]:
            for edge in box:
                k = (np.asarray(edge) - lb) / ((ub - lb) / n)
                assert np.allclose(k, np.round(k), atol=1e-9)
                assert np.all(k >= -1e-9) and np.all(k <= n + 1e-9)
    assert W.served_trace(pool, duration=1.0) == W.served_trace(pool, duration=1.0)
