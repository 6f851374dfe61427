"""GPU tests of the autotuner: its choices are valid and leave results within
the parity tolerance of the library defaults."""
import numpy as np
import pytest

from paper_2401_03555_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_03555_amd import autotune, impact
    impact.lib()
    return autotune, impact


def test_tuned_build_matches_default(T, tmp_path):
    autotune, impact = T
    system = dict(W.unicycle3d(n=(12, 12, 8))[0], sigma=[0.2, 0.2, 0.1])
    spec = W.unicycle3d()[1]
    spec = dict(spec, max_sweeps=400)
    tuner = autotune.Autotuner(path=str(tmp_path / "t.json"))
    im, c = tuner.build(system)
    assert c["storage"] in ("bounds", "factors") and not c["cached"]
    assert c["policy_pass"] in autotune.MODES and c["fixed_pass"] in autotune.MODES
    assert set(c["measured"]) >= {"factors"}
    r = im.iterate(spec)
    ref_im = impact.build_imdp(system)
    ref = ref_im.iterate(spec)
    assert np.abs((r["lo"] - ref["lo"]).cpu().numpy()).max() <= 1e-9
    assert np.abs((r["hi"] - ref["hi"]).cpu().numpy()).max() <= 1e-9
    # the second tuner reads the first one's file
    c2 = autotune.Autotuner(path=str(tmp_path / "t.json")).choose(system)
    assert c2["cached"] and c2["storage"] == c["storage"]


def test_batch_choice(T):
    autotune, impact = T
    systems = [s for s, _ in W.batched(count=12, seed=11)]
    tuner = autotune.Autotuner(budget_bytes=1 << 33)
    c = tuner.choose_batch(systems, sample=6, steps=8)
    assert c["storage"] in ("bounds", "factors") and c["chunk"] in autotune.CHUNKS
    assert tuner.choose_batch(systems, sample=6, steps=8)["cached"]
