"""GPU test of the FP64 FMA probe (measurement support, not a method step)."""
import ctypes as C

import pytest

pytestmark = pytest.mark.gpu


def test_probe_runs_and_rejects_bad_arguments():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_03555_amd import impact
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    ptr = C.cast(out.data_ptr(), C.POINTER(C.c_double))
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert impact.lib().impact_probe_fp64_fma(64, 16, ptr, st) == 0
    torch.cuda.synchronize()
    assert out.item() == 0.0            # the guarded store is never taken
    assert impact.lib().impact_probe_fp64_fma(0, 16, ptr, st) == -1
    assert impact.lib().impact_probe_fp64_fma(64, 0, ptr, st) == -1
    assert impact.lib().impact_probe_fp64_fma(64, 16, None, st) == -1
    assert impact.probe_fp64_fma(n_blocks=256, iters=64, reps=1) > 0.0
