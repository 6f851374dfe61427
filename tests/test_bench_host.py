"""Host checks of bench.py (no GPU): its helpers exist, every workload it
names resolves, the recorded-counter lookups work, and more than one GPU is
refused with a message."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_helpers_exist(bench):
    for name in ("measure_plain", "build_roofline", "mc_build_roofline", "algorithmic_bytes",
                 "cpu_baseline", "cpu_worker", "run_batched", "run_served", "run_disturbed",
                 "measured_peaks", "sweep_kernel_name"):
        assert callable(getattr(bench, name)), name


@pytest.mark.parametrize("name", ["unicycle3d", "robot2d", "room5d", "robot2d_correlated"])
def test_workloads_resolve(bench, name):
    system, spec, desc, mc = bench.workload(name)
    assert desc and spec["kind"] in ("safety", "reach", "reach_avoid")
    assert (mc is not None) == (name == "robot2d_correlated")


def test_source_digests_and_recorded_lines(bench):
    digests = {k: bench.kernel_source_hash(k) for k in bench.KERNEL_SOURCES}
    assert len(set(digests.values())) == len(digests)
    # a lookup for a kernel build that was never profiled finds nothing
    assert bench.recorded_traffic("k_sweep_sel", "bounds", "no-such-workload") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
