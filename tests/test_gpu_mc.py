"""GPU parity of the correlated-noise (Monte Carlo) build, Section 4.1: the HIP
library through its C ABI against the CPU oracle on the same seeded points.

Bounds: windows identical, entries / OUT / TAIL within 1e-12 absolute (the two
sides differ only in the last bits of exp / erf / erfc).  Values of the
iteration over the built rows: within 1e-9, policies equal up to ties.
"""
import numpy as np
import pytest

import oracle
from paper_2401_03555_amd import workloads as W

from test_gpu_parity import compare_iter, compare_rows, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def I():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_03555_amd import impact
    impact.lib()
    return impact


def _corr(sigma, R):
    s = np.asarray(sigma, dtype=np.float64)
    cov = np.asarray(R, dtype=np.float64) * np.outer(s, s)
    P = np.linalg.inv(cov)
    return 0.5 * (P + P.T), float(np.linalg.det(cov))


def _case(name):
    if name == "robot_corr":
        system, _, mc = W.robot2d_correlated(n=(10, 10), samples=64, grid_pts=2, kappa=3.0)
        return system, mc
    if name == "affine3_corr":
        system = W.tiny_affine(d=3, n=5, seed=3)
        P, det = _corr(system["sigma"], [[1.0, 0.3, 0.1], [0.3, 1.0, -0.2], [0.1, -0.2, 1.0]])
        return system, dict(inv_cov=P, det_cov=det, samples=W.mc_points(48, 3, seed=21),
                            grid_pts=2, kappa=2.0)
    if name == "room5d_corr":
        system = W.room5d(cells=3)[0]
        R = np.eye(5)
        for i in range(5):
            R[i, (i + 1) % 5] = R[(i + 1) % 5, i] = 0.2
        P, det = _corr(system["sigma"], R)
        return system, dict(inv_cov=P, det_cov=det, samples=W.mc_points(32, 5, seed=22),
                            grid_pts=1, kappa=1.0)
    if name == "affine6_corr":
        rng = np.random.default_rng(23)
        M = rng.normal(size=(6, 6))
        cov = 0.04 * (M @ M.T / 6 + 0.5 * np.eye(6))
        P = np.linalg.inv(cov)
        system = dict(kind="affine", A=0.5 * np.eye(6), B=0.3 * np.ones((6, 1)), c=np.zeros(6),
                      lb=[-1.0] * 6, ub=[1.0] * 6, n=[2] * 6, inputs=[[-1.0], [1.0]],
                      sigma=[1.0] * 6, k_sigma=6.0)
        return system, dict(inv_cov=0.5 * (P + P.T), det_cov=float(np.linalg.det(cov)),
                            samples=W.mc_points(16, 6, seed=24), grid_pts=1, kappa=0.5)
    if name == "robot_sharp":
        # noise far narrower than a cell: the factored exponents could overflow,
        # so the rows are evaluated directly
        system, _, mc = W.robot2d_correlated(n=(10, 10), samples=32, grid_pts=2, kappa=2.0)
        cov = np.linalg.inv(mc["inv_cov"]) * 1e-4
        P = np.linalg.inv(cov)
        return system, dict(mc, inv_cov=0.5 * (P + P.T), det_cov=float(np.linalg.det(cov)))
    if name == "affine2_G4":
        system = W.tiny_affine(d=2, n=8, seed=5)
        P, det = _corr(system["sigma"], [[1.0, -0.4], [-0.4, 1.0]])
        return system, dict(inv_cov=P, det_cov=det, samples=W.mc_points(100, 2, seed=25),
                            grid_pts=4, kappa=1.5)
    if name == "affine4_corr":
        rng = np.random.default_rng(26)
        M = rng.normal(size=(4, 4))
        A = 0.7 * M / max(abs(np.linalg.eigvals(M)))
        system = dict(kind="affine", A=A, B=0.2 * np.ones((4, 1)), c=np.zeros(4),
                      lb=[-1.0] * 4, ub=[1.0] * 4, n=[4] * 4, inputs=[[-1.0], [0.0], [1.0]],
                      sigma=[1.0] * 4, k_sigma=6.0)
        R = np.eye(4) + 0.25 * (np.ones((4, 4)) - np.eye(4))
        P, det = _corr([0.15] * 4, R)
        return system, dict(inv_cov=P, det_cov=det, samples=W.mc_points(40, 4, seed=27),
                            grid_pts=2, kappa=1.0)
    if name == "robot_dense_N1":
        system, _, mc = W.robot2d_correlated(n=(6, 6), samples=1, grid_pts=1, kappa=0.0)
        return dict(system, k_sigma=0.0), mc
    raise KeyError(name)


CASES = ["robot_corr", "affine3_corr", "room5d_corr", "affine6_corr", "robot_dense_N1",
         "robot_sharp", "affine2_G4", "affine4_corr"]


@pytest.mark.parametrize("name", CASES)
def test_mc_build_parity_all_rows(I, name):
    system, mc = _case(name)
    say(f"mc build parity: {name}")
    g = I.build_imdp_mc(system, mc)
    info = g.info()
    R, d = info["n_rows"], info["dim"]
    o = oracle.build_mc(system, mc, system["k_sigma"])
    assert info["n_entries"] == o["row_ptr"][-1]
    compare_rows(g.export_rows(0, R), o, R, d, name)
    g.free()


SPECS = {
    "robot_corr": dict(kind="reach_avoid", target=[[[5.0, 5.0], [7.0, 7.0]]],
                       avoid=[[[-2.0, -2.0], [2.0, 2.0]]]),
    "affine3_corr": dict(kind="reach", target=[[[0.0, 0.0, 0.0], [1.3, 1.3, 1.3]]], avoid=[]),
    "room5d_corr": dict(kind="safety", target=[], avoid=[]),
}


@pytest.mark.parametrize("name", list(SPECS))
def test_mc_iterate_parity(I, name):
    system, mc = _case(name)
    spec = dict(SPECS[name], eps=1e-8, max_sweeps=400)
    say(f"mc iterate parity: {name} {spec['kind']}")
    g = I.build_imdp_mc(system, mc)
    rg = g.iterate(spec)
    m = oracle.build_mc(system, mc, system["k_sigma"])
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate(m["n_states"], m["n_inputs"], m["row_ptr"], m["target"], m["lo"], m["hi"],
                        cls, spec["kind"], spec["eps"], spec["max_sweeps"], want_q0=True)
    assert rg["status"] == ro["status"]
    compare_iter(rg, ro, cls, spec["kind"] != "safety", name, q0=ro["q0"], model=m, spec=spec)
    g.free()


def test_mc_build_full_size_sampled_rows(I):
    """The 40x40 correlated robot with 256 random points and 2x2 candidates:
    sampled row blocks against the oracle."""
    system, _, mc = W.robot2d_correlated()
    g = I.build_imdp_mc(system, mc)
    info = g.info()
    R, d = info["n_rows"], info["dim"]
    rng = np.random.default_rng(9)
    for s0 in sorted(set([0, R - 16] + list(rng.integers(0, R - 16, size=6)))):
        rows = np.arange(s0, s0 + 16)
        o = oracle.build_mc(system, mc, system["k_sigma"], rows=rows)
        compare_rows(g.export_rows(int(s0), 16), o, 16, d, f"robot2d_correlated[{s0}:{s0 + 16}]")
    g.free()


def test_mc_rejects_bad_noise(I):
    system, _, mc = W.robot2d_correlated(n=(4, 4), samples=8)
    for bad, code in ((dict(det_cov=2 * mc["det_cov"]), I.E_INVAL),
                      (dict(samples=np.full((4, 2), 1.0)), I.E_INVAL),
                      (dict(grid_pts=0), I.E_INVAL),
                      (dict(grid_pts=65), I.E_UNSUPPORTED)):
        with pytest.raises(I.ImpactError) as e:
            I.build_imdp_mc(system, dict(mc, **bad))
        assert e.value.code == code, bad


@pytest.mark.parametrize("horizon", [0, "auto"])
def test_mc_handle_in_the_engine_equals_plain_iterate(I, horizon):
    """A correlated-noise abstraction is an ordinary handle: the multi-query
    engine runs its query exactly as the plain call does (bitwise)."""
    system, mc = _case("robot_corr")
    spec = dict(SPECS["robot_corr"], eps=1e-8, max_sweeps=400, horizon=horizon)
    imdp = I.build_imdp_mc(system, mc)
    imdp.set_sweep_modes("state_box", "per_row")
    plain = imdp.iterate(spec)
    eng = I.Engine(max_queries=2)
    qid = eng.submit(imdp, spec)
    res = eng.run_all()[qid]
    for k in ("lo", "hi", "policy"):
        a, b = res[k].cpu().numpy(), plain[k].cpu().numpy()
        assert np.array_equal(a, b), (k, np.abs(a - b).max())
    assert tuple(res["info"]["sweeps"]) == tuple(plain["info"]["sweeps"])
    eng.free()
    imdp.free()
