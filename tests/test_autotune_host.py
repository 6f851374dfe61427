"""Host logic of the autotuner: shape keys, result cache, sampling (no GPU)."""
import json

import numpy as np

from paper_2401_03555_amd import autotune as A, workloads as W


def _info(**kw):
    base = dict(dim=3, n_inputs=20, n_rows=1_000_000, max_row=300, n_entries=60_000_000,
                windowed=1, n_states=50_000)
    base.update(kw)
    return base


def test_keys_bucket_by_powers_of_two(monkeypatch):
    monkeypatch.setattr(A, "_device", lambda: "dev")
    k = A.imdp_key(_info())
    assert k == A.imdp_key(_info(n_rows=1_100_000, max_row=290))
    assert k != A.imdp_key(_info(max_row=600))
    assert k != A.imdp_key(_info(dim=2))
    assert k.startswith("dev/")
    t = A.Autotuner()
    b = t.batch_key([_info(), _info(dim=2, max_row=50)])
    assert "d2-3" in b and b.startswith("dev/batch/")


def test_cached_choice_skips_measurement(monkeypatch, tmp_path):
    monkeypatch.setattr(A, "_device", lambda: "dev")

    class Probe:
        def info(self):
            return _info()

        def free(self):
            pass

    monkeypatch.setattr(A.impact, "build_imdp", lambda system, storage="bounds": Probe())
    path = tmp_path / "tune.json"
    key = A.imdp_key(_info())
    # measured per-sweep ms of (policy pass, fixed pass) per storage and entry order
    measured = {"factors": {"state_box": [1.0, 0.5], "per_row": [3.0, 0.2]},
                "bounds": {"state_box": [0.9, 0.6], "per_row": [2.0, 0.3]}}
    path.write_text(json.dumps({key: {"measured": measured}}))
    t = A.Autotuner(path=str(path))
    c = t.choose({"n": [2, 2, 2]})
    assert c["cached"] and c["policy_pass"] == "state_box" and c["fixed_pass"] == "per_row"
    # equal weights: factors 1.0 + 0.2 = 1.2 beats bounds 0.9 + 0.3 = 1.2 only on ties; a
    # policy pass that runs ten times as many sweeps favours bounds (9.3 < 10.2)
    assert t.choose({"n": [2, 2, 2]}, weights=(10, 1))["storage"] == "bounds"
    # a fixed pass that runs ten times as many sweeps favours factors (3.0 < 3.9)
    c = t.choose({"n": [2, 2, 2]}, weights=(1, 10))
    assert c["storage"] == "factors" and abs(c["weighted_ms"] - 3.0) < 1e-12


def test_sample_takes_largest_and_seeded_rest():
    systems = [s for s, _ in W.batched(count=40, seed=3)]
    t = A.Autotuner()
    sub = t._sample(systems, 10)
    rows = [np.prod(s["n"]) * len(s["inputs"]) for s in systems]
    top = sorted(rows, reverse=True)[:5]
    got = [np.prod(s["n"]) * len(s["inputs"]) for s in sub]
    assert len(sub) == 10 and got[:5] == top
    assert [id(s) for s in t._sample(systems, 10)] == [id(s) for s in sub]


def test_first_and_later_sweeps_priced_apart(monkeypatch, tmp_path):
    """A measurement (first0, first1, later0, later1): the first TUNE_SWEEPS
    sweeps of a pass at the first rate, every later one at the later rate."""
    monkeypatch.setattr(A, "_device", lambda: "dev")

    class Probe:
        def info(self):
            return _info()

        def free(self):
            pass

    monkeypatch.setattr(A.impact, "build_imdp", lambda system, storage="bounds": Probe())
    path = tmp_path / "tune.json"
    key = A.imdp_key(_info())
    # factors: dearer first sweeps, cheaper later ones than bounds
    measured = {"factors": {"state_box": [12.4, 4.8, 7.1, 2.4], "per_row": [12.4, 4.8, 7.1, 2.4]},
                "bounds": {"state_box": [12.3, 4.7, 7.5, 2.7], "per_row": [12.3, 4.7, 7.5, 2.7]}}
    path.write_text(json.dumps({key: {"measured": measured}}))
    t = A.Autotuner(path=str(path))
    assert t.choose({"n": [2, 2, 2]})["storage"] == "bounds"       # one sweep of each pass
    c = t.choose({"n": [2, 2, 2]}, weights=(50, 50))
    s = A.TUNE_SWEEPS
    assert c["storage"] == "factors"
    assert abs(c["weighted_ms"] - (s * 12.4 + (50 - s) * 7.1 + s * 4.8 + (50 - s) * 2.4)) < 1e-9
    assert abs(c["ms_per_sweep"][0] - (s * 12.4 + (50 - s) * 7.1) / 50) < 1e-12
    # fewer sweeps than the first-rate span: every one at the first rate
    c = t.choose({"n": [2, 2, 2]}, weights=(3, 0))
    assert c["storage"] == "bounds" and abs(c["weighted_ms"] - 3 * 12.3) < 1e-9
