"""impact_interval_iterate_noalloc (temporaries in the library's static device
array) against impact_interval_iterate (temporaries from the allocator), both
called through the C ABI: identical outputs, status and sweep counts on two
calls in a row, the second with a smaller input; a call whose temporaries do
not fit the array is rejected."""
import numpy as np
import pytest

from paper_2401_03555_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def I():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_03555_amd import impact
    impact.lib()
    return impact


def _same(a, b, label):
    print(f"{label}: status {a['status']} / {b['status']}, sweeps {a['info']['sweeps']} / "
          f"{b['info']['sweeps']}", flush=True)
    assert a["status"] == b["status"]
    assert a["info"]["sweeps"] == b["info"]["sweeps"]
    assert a["info"]["n_safe"] == b["info"]["n_safe"]
    for k in ("lo", "hi", "policy"):
        assert bool((a[k] == b[k]).all()), f"{label}: {k} differs"


CASES = [
    # long rows (selection sweep, sorted values and row hints in the array),
    # then a smaller system with short rows
    ("room5d_6", lambda: W.room5d(cells=6)[0], dict(kind="safety", target=[], avoid=[]), 12),
    ("affine2", lambda: W.tiny_affine(d=2, n=9, seed=2),
     dict(kind="reach_avoid", target=[[[0.5, 0.5], [1.5, 1.5]]],
          avoid=[[[-1.5, -1.5], [-0.5, -0.5]]]), 3000),
]


def test_noalloc_matches_allocating_entry_point_twice(I):
    sizes = []
    for name, make, spec, K in CASES:
        system = make()
        g = I.build_imdp(system)
        sizes.append(g.info()["n_states"])
        spec = dict(spec, eps=1e-8, max_sweeps=K)
        ref = g.iterate(spec)
        got = g.iterate(spec, noalloc=True)
        _same(got, ref, name)
        # optimistic policy and a finite horizon through the same array
        for extra in (dict(pessimistic=False), dict(horizon=5)):
            _same(g.iterate(dict(spec, **extra), noalloc=True), g.iterate(dict(spec, **extra)),
                  f"{name} {extra}")
        g.free()
    assert sizes[1] < sizes[0]


def test_noalloc_rejects_calls_beyond_the_array(I):
    # about 1.1 M states need ~72 MB of temporaries, more than the 64 MiB array
    system = dict(kind="affine", A=np.eye(2), B=np.zeros((2, 1)), c=np.zeros(2),
                  lb=[0.0, 0.0], ub=[1.0, 1.0], n=[1100, 1000], inputs=[[0.0]],
                  sigma=[1e-4, 1e-4], k_sigma=6.0)
    g = I.build_imdp(system)
    spec = dict(kind="safety", target=[], avoid=[], eps=1e-8, max_sweeps=2)
    with pytest.raises(I.ImpactError) as ei:
        g.iterate(spec, noalloc=True)
    assert ei.value.code == I.E_UNSUPPORTED
    assert "static scratch" in str(ei.value)
    # the allocating entry point runs it
    r = g.iterate(spec)
    assert r["info"]["sweeps"][0] >= 1
    g.free()
