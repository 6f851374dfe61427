"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bounds: windows identical, entries / OUT / TAIL within 1e-12 absolute.
Values: within 1e-9; policies identical except at ties (an input whose oracle
LP value is within 1e-12 of the optimum).  Sweep counts identical.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2401_03555_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BOUND_TOL = 1e-12
VALUE_TOL = 1e-9
TIE_TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def I():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_03555_amd import impact
    impact.lib()  # raises if the library is missing
    return impact


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def compare_rows(gpu, orc, nrows, d, label):
    """gpu: export of rows [row0, row0 + nrows); orc: oracle build of the same rows."""
    assert gpu["win"].shape == (nrows, 2 * d)
    win_bad = np.where((gpu["win"] != orc["win"]).any(1))[0]
    assert len(win_bad) == 0, f"{label}: window mismatch in rows {win_bad[:10]}"
    extra = 1 + int(orc["windowed"])
    ncell = np.diff(orc["row_ptr"]) - extra
    assert np.array_equal(gpu["counts"], ncell)
    sel = np.ones(orc["row_ptr"][-1], bool)
    sel[orc["row_ptr"][1:] - 1] = False
    if extra == 2:
        sel[orc["row_ptr"][1:] - 2] = False
    olo, ohi = orc["lo"][sel], orc["hi"][sel]
    glo, ghi = gpu["entries"][:, 0], gpu["entries"][:, 1]
    assert len(glo) == len(olo)
    dlo = np.abs(glo - olo).max(initial=0.0)
    dhi = np.abs(ghi - ohi).max(initial=0.0)
    dot = np.abs(gpu["ot"] - orc["ot"]).max(initial=0.0)
    say(f"{label}: rows {nrows} cells {len(olo)} max|dlo| {dlo:.2e} max|dhi| {dhi:.2e} "
        f"max|d ot| {dot:.2e}")
    assert dlo <= BOUND_TOL and dhi <= BOUND_TOL and dot <= BOUND_TOL


def gpu_build(I, system, storage="bounds"):
    return I.build_imdp(system, storage=storage)


def check_policy(pol_g, pol_o, q0, cls, reach, label):
    safe = np.where(cls == 0)[0]
    diff = safe[pol_g[safe] != pol_o[safe]]
    bad = []
    for s in diff:
        q = q0[s]
        best = q.max() if reach else q.min()
        got = q[pol_g[s]]
        if (reach and got < best - TIE_TOL) or (not reach and got > best + TIE_TOL):
            bad.append(s)
    say(f"{label}: policy differs on {len(diff)} of {len(safe)} SAFE cells, "
        f"{len(bad)} not ties")
    assert not bad, f"{label}: policy mismatch beyond ties at {bad[:10]}"


def fixed_pass_under(m, cls, spec, policy, optimistic, n_dist=1):
    """Oracle run of the interval Markov chain that ``policy`` induces (with
    its disturbance rows, if any).

    The fixed-input pass starts afresh from the policy alone, so its bound and
    sweep count are those of the second pass of this run.
    """
    N = m["n_states"]
    U = m["n_inputs"] // n_dist
    pol = np.maximum(np.asarray(policy), 0)
    rows = ((np.arange(N) * U + pol)[:, None] * n_dist + np.arange(n_dist)[None, :]).ravel()
    rp = m["row_ptr"]
    starts, ends = rp[rows], rp[rows + 1]
    idx = np.concatenate([np.arange(a, b) for a, b in zip(starts, ends)])
    new_rp = np.concatenate([[0], np.cumsum(ends - starts)]).astype(np.int64)
    return oracle.iterate(N, 1, new_rp, m["target"][idx], m["lo"][idx], m["hi"][idx], cls,
                          spec["kind"], spec["eps"], spec["max_sweeps"], optimistic=optimistic,
                          horizon=spec.get("horizon", 0), n_dist=n_dist)


def compare_iter(g, o, cls, reach, label, q0=None, model=None, spec=None, optimistic=False,
                 n_dist=1):
    """Policy-pass bound and sweeps against the oracle; the policy equal up to
    ties.  Where the policies differ at ties (``model`` given), the
    fixed-input pass is checked against the oracle run under the GPU's policy."""
    lo, hi = g["lo"].cpu().numpy(), g["hi"].cpu().numpy()
    pol = g["policy"].cpu().numpy()
    kp, kf = ("hi", "lo") if optimistic else ("lo", "hi")
    got = dict(lo=lo, hi=hi)
    dlo = np.abs(lo - o["lo"]).max()
    dhi = np.abs(hi - o["hi"]).max()
    say(f"{label}: sweeps gpu {g['info']['sweeps']} oracle {tuple(o['sweeps'])} "
        f"max|dlo| {dlo:.2e} max|dhi| {dhi:.2e} status {g['status']}")
    assert g["info"]["sweeps"][0] == o["sweeps"][0]
    assert np.abs(got[kp] - o[kp]).max() <= VALUE_TOL
    if q0 is not None:
        check_policy(pol, np.asarray(o["policy"]), q0, cls, reach, label)
    else:
        assert np.array_equal(pol, o["policy"])
    ref = o
    if model is not None and not np.array_equal(pol, np.asarray(o["policy"])):
        ref = fixed_pass_under(model, cls, spec, pol, optimistic, n_dist)
        d = np.abs(got[kf] - ref[kf]).max()
        say(f"{label}: policies differ at ties; fixed pass under the GPU policy: "
            f"sweeps {ref['sweeps'][1]} max|d{kf}| {d:.2e}")
    assert g["info"]["sweeps"][1] == ref["sweeps"][1]
    assert np.abs(got[kf] - ref[kf]).max() <= VALUE_TOL


SMALL_SYSTEMS = {
    "affine2_window": lambda: W.tiny_affine(d=2, n=9, seed=2),
    "affine3_window": lambda: W.tiny_affine(d=3, n=6, seed=3),
    "affine2_dense": lambda: W.tiny_affine(d=2, n=7, seed=8, k_sigma=0.0),
    "affine1_window": lambda: dict(kind="affine", A=[[0.9]], B=[[0.4]], c=[0.1], lb=[-3.0],
                                   ub=[3.0], n=[61], inputs=[[-1.0], [0.0], [1.0]],
                                   sigma=[0.08], k_sigma=6.0),
    "unicycle_small": lambda: dict(W.unicycle3d(n=(10, 10, 6))[0], sigma=[0.3, 0.3, 0.2]),
    "robot2d": lambda: W.robot2d()[0],
    "room5d_4": lambda: W.room5d(cells=4)[0],
}


# ---------------------------------------------------------------------------
# bound construction
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(SMALL_SYSTEMS))
def test_build_parity_all_rows(I, name):
    system = SMALL_SYSTEMS[name]()
    say(f"build parity: {name}")
    g = gpu_build(I, system)
    info = g.info()
    R, d = info["n_rows"], info["dim"]
    o = oracle.build(system, system["k_sigma"])
    assert info["n_entries"] == o["row_ptr"][-1]
    compare_rows(g.export_rows(0, R), o, R, d, name)


@pytest.mark.parametrize("name", ["unicycle3d", "room5d"])
def test_build_parity_full_size_sampled(I, name):
    system = (W.unicycle3d()[0] if name == "unicycle3d" else W.room5d()[0])
    say(f"build parity (sampled rows, full size): {name}")
    g = gpu_build(I, system)
    info = g.info()
    R, d = info["n_rows"], info["dim"]
    rng = np.random.default_rng(5)
    starts = sorted(set([0, R - 40] + list(rng.integers(0, R - 40, size=24))))
    for s0 in starts:
        rows = np.arange(s0, s0 + 40)
        o = oracle.build(system, system["k_sigma"], rows=rows)
        compare_rows(g.export_rows(int(s0), 40), o, 40, d, f"{name}[{s0}:{s0 + 40}]")
    assert info["max_row"] <= 4096


def test_factor_storage_matches_bound_storage(I):
    system = W.tiny_affine(d=3, n=6, seed=4)
    a = gpu_build(I, system, "bounds")
    b = gpu_build(I, system, "factors")
    R = a.info()["n_rows"]
    ea, eb = a.export_rows(0, R), b.export_rows(0, R)
    for k in ("win", "ot", "counts", "entries"):
        assert np.array_equal(ea[k], eb[k]), k
    spec = dict(kind="reach_avoid", target=[[[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]]],
                avoid=[[[-1.5, -1.5, -1.5], [-0.5, -0.5, -0.5]]], eps=1e-8, max_sweeps=5000)
    ra, rb = a.iterate(spec), b.iterate(spec)
    for k in ("lo", "hi", "policy"):
        assert bool((ra[k] == rb[k]).all()), k


# ---------------------------------------------------------------------------
# interval iteration
# ---------------------------------------------------------------------------

SPECS = {
    "affine2_window": dict(kind="reach_avoid", target=[[[0.5, 0.5], [1.5, 1.5]]],
                           avoid=[[[-1.5, -1.5], [-0.5, -0.5]]]),
    "affine3_window": dict(kind="reach", target=[[[0.0, 0.0, 0.0], [1.3, 1.3, 1.3]]], avoid=[]),
    "affine2_dense": dict(kind="safety", target=[], avoid=[[[-0.5, -0.5], [0.5, 0.5]]]),
    "affine1_window": dict(kind="reach_avoid", target=[[[1.0], [2.0]]], avoid=[[[-0.5], [0.0]]]),
    "unicycle_small": dict(kind="reach_avoid", target=[[[2.0, 2.0, -4.0], [5.0, 5.0, 4.0]]],
                           avoid=[[[-1.0, -1.0, -4.0], [1.0, 1.0, 4.0]]]),
    "room5d_4": dict(kind="safety", target=[], avoid=[]),
}


@pytest.mark.parametrize("name", list(SPECS))
def test_iterate_parity_small(I, name):
    system = SMALL_SYSTEMS[name]()
    spec = dict(SPECS[name], eps=1e-8, max_sweeps=3000 if name != "room5d_4" else 40)
    say(f"iterate parity: {name} {spec['kind']}")
    g = gpu_build(I, system)
    rg = g.iterate(spec)
    m = oracle.build(system, system["k_sigma"])
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate(m["n_states"], m["n_inputs"], m["row_ptr"], m["target"], m["lo"], m["hi"],
                        cls, spec["kind"], spec["eps"], spec["max_sweeps"], want_q0=True)
    assert rg["status"] == ro["status"]
    compare_iter(rg, ro, cls, spec["kind"] != "safety", name, q0=ro["q0"], model=m, spec=spec)


def test_iterate_parity_robot2d_converged(I):
    with open(os.path.join(HERE, "golden", "robot2d_oracle.json")) as f:
        gold = json.load(f)
    system, spec = W.robot2d()
    g = gpu_build(I, system)
    rg = g.iterate(spec)
    cls = oracle.label(system, spec["target"], spec["avoid"])
    q0 = np.array([[np.nan if x is None else x for x in row] for row in gold["q0"]])
    o = dict(lo=np.array(gold["lo"]), hi=np.array(gold["hi"]), policy=np.array(gold["policy"]),
             sweeps=gold["sweeps"])
    compare_iter(rg, o, cls, True, "robot2d (converged)", q0=q0)
    assert rg["status"] == 0


def test_iterate_parity_unicycle_full_size_fixed_sweeps(I):
    system, spec = W.unicycle3d()
    K = 2
    say("unicycle3d full size, 2 sweeps per pass")
    g = gpu_build(I, system)
    rg = g.iterate(spec, max_sweeps=K)
    m = oracle.build(system, system["k_sigma"])
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate(m["n_states"], m["n_inputs"], m["row_ptr"], m["target"], m["lo"], m["hi"],
                        cls, spec["kind"], spec["eps"], K, want_q0=True)
    assert rg["status"] == ro["status"] == 1
    compare_iter(rg, ro, cls, True, "unicycle3d K=2", q0=ro["q0"])


def _golden_npz(name):
    path = os.path.join(HERE, "golden", f"{name}_oracle.npz")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def check_policy_ties(pol_g, gold, cls, label):
    """The GPU policy equals the oracle's, or takes an input the oracle's last
    pass-1 sweep valued within 1e-12 of the optimum (its tie mask)."""
    safe = np.where(cls == 0)[0]
    diff = safe[pol_g[safe] != gold["policy"][safe]]
    ok = (gold["ties"][diff] >> pol_g[diff].astype(np.int64)) & 1
    bad = diff[ok == 0]
    say(f"{label}: policy differs on {len(diff)} of {len(safe)} SAFE cells, {len(bad)} not ties")
    assert len(bad) == 0, f"{label}: policy mismatch beyond ties at {bad[:10]}"
    return len(diff)


@pytest.mark.parametrize("storage", ["bounds", "factors"])
def test_iterate_parity_room5d_full_size_two_sweeps(I, storage):
    # the largest single-GPU workload at full size: 10^5 cells, rows of up to
    # 3,127 entries (the long-row selection sweep), two sweeps of each pass
    # against the oracle's run stored by tests/golden/make_golden.py
    gold = _golden_npz("room5d_k2")
    system, spec = W.room5d()
    say(f"room5d full size [{storage}], 2 sweeps per pass")
    g = gpu_build(I, system, storage=storage)
    assert g.info()["max_row"] == 3127
    r = g.iterate(spec, max_sweeps=2)
    cls = oracle.label(system, spec["target"], spec["avoid"])
    lo, hi = r["lo"].cpu().numpy(), r["hi"].cpu().numpy()
    dlo, dhi = np.abs(lo - gold["lo"]).max(), np.abs(hi - gold["hi"]).max()
    say(f"room5d: sweeps {r['info']['sweeps']} oracle {tuple(gold['sweeps'])} status "
        f"{r['status']} / {int(gold['status'])} max|dlo| {dlo:.2e} max|dhi| {dhi:.2e}")
    assert r["info"]["sweeps"] == tuple(int(x) for x in gold["sweeps"])
    assert r["status"] == int(gold["status"]) == 1
    assert dlo <= VALUE_TOL
    n_tie = check_policy_ties(r["policy"].cpu().numpy(), gold, cls, "room5d K=2")
    if n_tie == 0:
        assert dhi <= VALUE_TOL
    else:
        # the fixed-input pass under the GPU's policy, from the oracle
        m = oracle.build(system, system["k_sigma"])
        ref = fixed_pass_under(m, cls, dict(spec, max_sweeps=2), r["policy"].cpu().numpy(),
                               False)
        assert np.abs(hi - ref["hi"]).max() <= VALUE_TOL


def test_iterate_parity_unicycle_full_size_converged(I):
    # the default workload run to eps (42 + 87 sweeps) against the oracle's
    # converged run stored by tests/golden/make_golden.py
    gold = _golden_npz("unicycle3d_converged")
    system, spec = W.unicycle3d()
    g = gpu_build(I, system, storage="factors")
    r = g.iterate(spec)
    cls = oracle.label(system, spec["target"], spec["avoid"])
    lo, hi = r["lo"].cpu().numpy(), r["hi"].cpu().numpy()
    dlo, dhi = np.abs(lo - gold["lo"]).max(), np.abs(hi - gold["hi"]).max()
    say(f"unicycle3d converged: sweeps {r['info']['sweeps']} oracle {tuple(gold['sweeps'])} "
        f"max|dlo| {dlo:.2e} max|dhi| {dhi:.2e}")
    assert r["status"] == int(gold["status"]) == 0
    assert r["info"]["sweeps"][0] == int(gold["sweeps"][0])
    assert dlo <= VALUE_TOL
    n_tie = check_policy_ties(r["policy"].cpu().numpy(), gold, cls, "unicycle3d converged")
    if n_tie == 0:
        assert r["info"]["sweeps"][1] == int(gold["sweeps"][1])
        assert dhi <= VALUE_TOL
    else:
        m = oracle.build(system, system["k_sigma"])
        ref = fixed_pass_under(m, cls, spec, r["policy"].cpu().numpy(), False)
        assert r["info"]["sweeps"][1] == ref["sweeps"][1]
        assert np.abs(hi - ref["hi"]).max() <= VALUE_TOL


def test_iterate_properties_unicycle_full_size(I):
    system, spec = W.unicycle3d()
    g = gpu_build(I, system)
    r = g.iterate(spec, max_sweeps=20000)
    lo, hi = r["lo"].cpu().numpy(), r["hi"].cpu().numpy()
    pol = r["policy"].cpu().numpy()
    cls = oracle.label(system, spec["target"], spec["avoid"])
    info = r["info"]
    say(f"unicycle3d full: status {r['status']} info {info}")
    assert info["n_safe"] == 53664
    assert (lo >= -1e-15).all() and (hi <= 1 + 1e-12).all()
    assert (lo <= hi + 1e-12).all()
    assert set(np.unique(pol[cls == 0])) <= set(range(20)) and (pol[cls != 0] == -1).all()
    assert (lo[cls == 1] == 1).all() and (lo[cls == 2] == 0).all()
    if r["status"] == 0:
        assert max(info["gap"]) <= spec["eps"]
    # determinism: a second solve is bitwise identical
    r2 = g.iterate(spec, max_sweeps=20000)
    for k in ("lo", "hi", "policy"):
        assert bool((r[k] == r2[k]).all()), k


def test_room5d_full_size_fixed_sweeps_properties(I):
    system, spec = W.room5d()
    g = gpu_build(I, system)
    info = g.info()
    say(f"room5d full build: {info}")
    r = g.iterate(spec, max_sweeps=3)
    lo, hi = r["lo"].cpu().numpy(), r["hi"].cpu().numpy()
    assert r["status"] == 1 and r["info"]["sweeps"] == (3, 3)
    # FP64 rounding can put V a few ulps outside [0, 1] (the oracle does the same)
    assert (lo >= -1e-12).all() and (hi <= 1 + 1e-12).all() and (lo <= hi + 1e-12).all()


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_empty_safe_set_runs_no_sweeps(I):
    system = W.tiny_affine(d=2, n=5, seed=3)
    spec = dict(kind="reach", target=[[[-2.0, -2.0], [2.0, 2.0]]], avoid=[], eps=1e-8,
                max_sweeps=10)
    r = gpu_build(I, system).iterate(spec)
    assert r["status"] == 0 and r["info"]["sweeps"] == (0, 0) and r["info"]["n_safe"] == 0
    assert bool((r["lo"] == 1).all()) and bool((r["policy"] == -1).all())


def test_imc_single_input(I):
    system = W.tiny_affine(d=2, n=8, seed=14, n_inputs=1)
    spec = dict(kind="reach", target=[[[0.0, 0.0], [1.0, 1.0]]], avoid=[], eps=1e-8,
                max_sweeps=5000)
    rg = gpu_build(I, system).iterate(spec)
    ro = oracle.solve(system, system["k_sigma"], "reach", spec["target"], None, 1e-8, 5000)
    compare_iter(rg, ro, ro["cls"], True, "imc")


def test_rows_leaving_the_domain_have_only_out_and_tail(I):
    # the mean of every row sits far outside [lb, ub]: empty windows
    system = dict(kind="affine", A=[[1.0]], B=[[0.0]], c=[50.0], lb=[-1.0], ub=[1.0], n=[8],
                  inputs=[[0.0]], sigma=[0.1], k_sigma=6.0)
    g = gpu_build(I, system)
    e = g.export_rows(0, 8)
    o = oracle.build(system, 6.0)
    assert (e["counts"] == 0).all()
    compare_rows(e, o, 8, 1, "empty windows")
    r = g.iterate(dict(kind="safety", target=[], avoid=[], eps=1e-8, max_sweeps=10))
    assert r["status"] == 0 and bool((r["hi"].abs() < 1e-12).all())


def _dense_rows(n0, n1):
    # dense rows of n0 * n1 cells + OUT (one input): every row is as long as the grid
    return dict(kind="affine", A=np.eye(2) * 0.5, B=np.zeros((2, 1)), c=np.zeros(2),
                lb=[-1.0, -1.0], ub=[1.0, 1.0], n=[n0, n1], inputs=[[0.0]], sigma=[0.4, 0.4],
                k_sigma=0.0)


DENSE_SPEC = dict(kind="reach_avoid", target=[[[0.5, 0.5], [1.0, 1.0]]],
                  avoid=[[[-1.0, -1.0], [-0.5, -0.5]]], eps=1e-8)


# row lengths of each long-row kernel class: 4,033 entries (4 wavefronts,
# 16 cells per thread), 4,097 (8 wavefronts) and 8,282 (16 wavefronts)
@pytest.mark.parametrize("n0,n1,K", [(63, 64, 3), (64, 64, 3), (91, 91, 2)])
def test_long_dense_rows_match_oracle(I, n0, n1, K):
    system = _dense_rows(n0, n1)
    say(f"dense rows {n0}x{n1}: {n0 * n1 + 1} entries, {K} sweeps per pass")
    g = gpu_build(I, system)
    assert g.info()["max_row"] == n0 * n1 + 1
    spec = dict(DENSE_SPEC, max_sweeps=K)
    rg = g.iterate(spec)
    m = oracle.build(system, 0.0)
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate(m["n_states"], 1, m["row_ptr"], m["target"], m["lo"], m["hi"], cls,
                        "reach_avoid", 1e-8, K)
    compare_iter(rg, ro, cls, True, f"{n0 * n1 + 1}-entry rows")


def test_rows_beyond_the_longest_supported_are_rejected(I):
    import paper_2401_03555_amd.impact as imp
    with pytest.raises(imp.ImpactError) as ei:
        gpu_build(I, _dense_rows(128, 128))  # 16,385 entries
    assert ei.value.code == imp.E_UNSUPPORTED


def test_ragged_rows_mix_wave_and_block_paths(I):
    # windows from 1 cell to > 512 entries inside one abstraction
    system = dict(kind="affine", A=np.diag([0.5, 1.0]), B=np.array([[1.0], [0.0]]),
                  c=np.zeros(2), lb=[-4.0, -4.0], ub=[4.0, 4.0], n=[40, 40],
                  inputs=[[-3.0], [0.0], [3.0]], sigma=[0.2, 0.9], k_sigma=6.0)
    g = gpu_build(I, system)
    info = g.info()
    say(f"ragged: max_row {info['max_row']}")
    assert info["max_row"] > 512
    counts = g.export_rows(0, info["n_rows"], entries=False)["counts"] + 2
    assert (counts <= 64).any() and ((counts > 64) & (counts <= 512)).any()
    o = oracle.build(system, 6.0)
    compare_rows(g.export_rows(0, info["n_rows"]), o, info["n_rows"], 2, "ragged")
    spec = dict(kind="reach_avoid", target=[[[2.0, -1.0], [3.0, 1.0]]],
                avoid=[[[-1.0, -4.0], [0.0, 4.0]]], eps=1e-8, max_sweeps=40)
    rg = g.iterate(spec)
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate(o["n_states"], 3, o["row_ptr"], o["target"], o["lo"], o["hi"], cls,
                        "reach_avoid", 1e-8, 40, want_q0=True)
    compare_iter(rg, ro, cls, True, "ragged", q0=ro["q0"])


# ---------------------------------------------------------------------------
# sweep modes: one sort per row vs one sort per state box
# ---------------------------------------------------------------------------

def _wide_box_system():
    # rows of <= 400 entries whose inputs shift the mean by +-5 cells, so most
    # state boxes exceed 512 cells and those states sort per row
    return dict(kind="affine", A=np.eye(2), B=np.array([[1.0], [0.0]]), c=np.zeros(2),
                lb=[-10.0, -10.0], ub=[10.0, 10.0], n=[40, 40], inputs=[[-2.5], [0.0], [2.5]],
                sigma=[0.8, 0.8], k_sigma=6.0)


MODE_CASES = {
    "affine2_window": (SMALL_SYSTEMS["affine2_window"], SPECS["affine2_window"], 3000),
    "unicycle_small": (SMALL_SYSTEMS["unicycle_small"], SPECS["unicycle_small"], 3000),
    "affine1_window": (SMALL_SYSTEMS["affine1_window"], SPECS["affine1_window"], 500),
    "robot2d_K60": (SMALL_SYSTEMS["robot2d"], dict(kind="reach_avoid",
                                                   target=[[[5.0, 5.0], [8.0, 8.0]]],
                                                   avoid=[[[-2.0, -2.0], [2.0, 2.0]]]), 60),
    "wide_box": (_wide_box_system, dict(kind="reach_avoid", target=[[[4.0, 4.0], [8.0, 8.0]]],
                                        avoid=[[[-3.0, -3.0], [0.0, 0.0]]]), 30),
}


@pytest.mark.parametrize("mode", ["per_row", "state_box"])
@pytest.mark.parametrize("case", list(MODE_CASES))
def test_sweep_modes_match_oracle(I, case, mode):
    make, spec, K = MODE_CASES[case]
    system = make()
    spec = dict(spec, eps=1e-8, max_sweeps=K)
    g = I.build_imdp(system, sweep_mode=mode)
    info = g.info()
    say(f"{case} [{mode}]: max_row {info['max_row']} max_box {info['max_box']}")
    if case == "wide_box":
        assert info["max_box"] > 512 >= info["max_row"]
    rg = g.iterate(spec)
    m = oracle.build(system, system["k_sigma"])
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate(m["n_states"], m["n_inputs"], m["row_ptr"], m["target"], m["lo"], m["hi"],
                        cls, spec["kind"], spec["eps"], K, want_q0=True)
    compare_iter(rg, ro, cls, spec["kind"] != "safety", f"{case}[{mode}]", q0=ro["q0"],
                 model=m, spec=spec)


# ---------------------------------------------------------------------------
# batch construction: one launch per kernel over several systems
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("storage", ["bounds", "factors"])
def test_batch_build_equals_separate_builds(I, storage):
    systems = [SMALL_SYSTEMS["affine2_window"](), SMALL_SYSTEMS["affine1_window"](),
               SMALL_SYSTEMS["affine3_window"](), SMALL_SYSTEMS["unicycle_small"](),
               W.tiny_affine(d=2, n=13, seed=21), _wide_box_system()]
    views = I.build_imdp_batch(systems, storage=storage)
    for k, (system, v) in enumerate(zip(systems, views)):
        single = I.build_imdp(system, storage=storage)
        a, b = v.info(), single.info()
        for key in ("n_states", "n_rows", "n_entries", "dim", "n_inputs", "max_row", "max_box"):
            assert a[key] == b[key], (k, key, a[key], b[key])
        R = a["n_rows"]
        ea, eb = v.export_rows(0, R), single.export_rows(0, R)
        for key in ("win", "ot", "counts", "entries"):
            assert np.array_equal(ea[key], eb[key]), (k, key)
    # the views iterate exactly like separately built handles
    spec = dict(SPECS["affine2_window"], eps=1e-8, max_sweeps=200)
    r1 = views[0].iterate(spec)
    r2 = I.build_imdp(systems[0], storage=storage).iterate(spec)
    for key in ("lo", "hi", "policy"):
        assert bool((r1[key] == r2[key]).all()), key
    del views


# ---------------------------------------------------------------------------
# optimistic policy (Sec. 5 with IMDP_lower = false): the policy pass takes
# the favourable bound, the fixed-input pass the adversarial one
# ---------------------------------------------------------------------------

OPT_CASES = ["affine2_window", "affine3_window", "affine2_dense", "affine1_window",
             "unicycle_small"]


@pytest.mark.parametrize("mode", ["per_row", "state_box"])
@pytest.mark.parametrize("name", OPT_CASES)
def test_optimistic_policy_matches_oracle(I, name, mode):
    system = SMALL_SYSTEMS[name]()
    spec = dict(SPECS[name], eps=1e-8, max_sweeps=3000, pessimistic=False)
    say(f"optimistic iterate parity: {name} {spec['kind']} [{mode}]")
    g = I.build_imdp(system, sweep_mode=mode)
    rg = g.iterate(spec)
    m = oracle.build(system, system["k_sigma"])
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate(m["n_states"], m["n_inputs"], m["row_ptr"], m["target"], m["lo"], m["hi"],
                        cls, spec["kind"], spec["eps"], spec["max_sweeps"], want_q0=True,
                        optimistic=True)
    assert rg["status"] == ro["status"]
    compare_iter(rg, ro, cls, spec["kind"] != "safety", f"{name} optimistic", q0=ro["q0"],
                 model=m, spec=spec, optimistic=True)
    lo, hi = rg["lo"].cpu().numpy(), rg["hi"].cpu().numpy()
    assert (lo <= hi + 1e-12).all()


def test_optimistic_and_pessimistic_policies_differ_where_choice_matters(I):
    # each policy is optimal for its own bound: the pessimistic one maximises
    # the guaranteed (lower) reach bound over the policies, the optimistic one
    # the possible (upper) bound; with several inputs some state's choice differs
    system = SMALL_SYSTEMS["unicycle_small"]()
    spec = dict(SPECS["unicycle_small"], eps=1e-8, max_sweeps=3000)
    g = I.build_imdp(system)
    rp = g.iterate(spec)
    ro = g.iterate(dict(spec, pessimistic=False))
    plo, phi = rp["lo"].cpu().numpy(), rp["hi"].cpu().numpy()
    olo, ohi = ro["lo"].cpu().numpy(), ro["hi"].cpu().numpy()
    tol = spec["eps"]
    assert (plo >= olo - tol).all()
    assert (ohi >= phi - tol).all()
    assert (ohi - phi).max() > 1e3 * tol
    assert (rp["policy"] != ro["policy"]).any()


# ---------------------------------------------------------------------------
# finite horizon (Remark 5.1): T sweeps of value iteration per pass
# ---------------------------------------------------------------------------

FH_CASES = ["affine2_window", "affine3_window", "affine2_dense", "unicycle_small"]


@pytest.mark.parametrize("mode", ["per_row", "state_box"])
@pytest.mark.parametrize("pessimistic", [True, False], ids=["pess", "opt"])
@pytest.mark.parametrize("name", FH_CASES)
def test_finite_horizon_matches_oracle(I, name, pessimistic, mode):
    system = SMALL_SYSTEMS[name]()
    T = 7
    spec = dict(SPECS[name], eps=1e-8, max_sweeps=1, horizon=T, pessimistic=pessimistic)
    say(f"finite horizon T={T}: {name} {spec['kind']} pessimistic={pessimistic} [{mode}]")
    g = I.build_imdp(system, sweep_mode=mode)
    rg = g.iterate(spec)
    m = oracle.build(system, system["k_sigma"])
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate(m["n_states"], m["n_inputs"], m["row_ptr"], m["target"], m["lo"], m["hi"],
                        cls, spec["kind"], spec["eps"], 1, want_q0=True,
                        optimistic=not pessimistic, horizon=T)
    assert rg["status"] == ro["status"] == 0
    assert tuple(rg["info"]["sweeps"]) == (T, T)
    compare_iter(rg, ro, cls, spec["kind"] != "safety", f"{name} T={T}", q0=ro["q0"],
                 model=m, spec=spec, optimistic=not pessimistic)


def test_finite_horizon_full_size_unicycle(I):
    system, spec = W.unicycle3d()
    T = 3
    spec = dict(spec, horizon=T)
    say(f"unicycle3d full size, finite horizon T={T}")
    g = gpu_build(I, system, "factors")
    rg = g.iterate(spec)
    m = oracle.build(system, system["k_sigma"])
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate(m["n_states"], m["n_inputs"], m["row_ptr"], m["target"], m["lo"], m["hi"],
                        cls, spec["kind"], spec["eps"], 1, want_q0=True, horizon=T)
    assert rg["status"] == ro["status"] == 0
    compare_iter(rg, ro, cls, True, f"unicycle3d T={T}", q0=ro["q0"], model=m, spec=spec)


def test_finite_horizon_degenerate_cases(I):
    system = SMALL_SYSTEMS["affine2_window"]()
    g = gpu_build(I, system)
    # no SAFE cell: nothing to sweep, whatever the horizon
    everything = [[[-100.0, -100.0], [100.0, 100.0]]]
    r = g.iterate(dict(kind="reach", target=everything, avoid=[], eps=1e-8, max_sweeps=1,
                       horizon=9))
    assert r["status"] == 0 and tuple(r["info"]["sweeps"]) == (0, 0)
    assert bool((r["lo"] == 1).all()) and bool((r["hi"] == 1).all())
    # T = 1: one sweep from zero is the one-step probability; both passes agree
    # with the infinite-horizon call capped at one sweep on the V0 side
    spec = dict(SPECS["affine2_window"], eps=1e-8, max_sweeps=1)
    one = g.iterate(dict(spec, horizon=1))
    capped = g.iterate(spec)
    assert tuple(one["info"]["sweeps"]) == (1, 1) and one["status"] == 0
    assert bool((one["lo"] == capped["lo"]).all())
    with pytest.raises(I.ImpactError, match="horizon"):
        g.iterate(dict(spec, horizon=-2))  # -1 is the automatic horizon


# ---------------------------------------------------------------------------
# Remark 5.2: horizon from the self-convergence of each pass's iterates
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("pessimistic", [True, False], ids=["pess", "opt"])
@pytest.mark.parametrize("name", ["affine2_window", "affine2_dense", "unicycle_small"])
def test_auto_horizon_matches_oracle(I, name, pessimistic):
    system = SMALL_SYSTEMS[name]()
    spec = dict(SPECS[name], eps=1e-8, max_sweeps=3000, horizon="auto", pessimistic=pessimistic)
    say(f"auto horizon: {name} {spec['kind']} pessimistic={pessimistic}")
    g = I.build_imdp(system)
    rg = g.iterate(spec)
    m = oracle.build(system, system["k_sigma"])
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate_auto_horizon(m["n_states"], m["n_inputs"], m["row_ptr"], m["target"],
                                     m["lo"], m["hi"], cls, spec["kind"], spec["eps"],
                                     spec["max_sweeps"], want_q0=True, optimistic=not pessimistic)
    info = rg["info"]
    say(f"  self sweeps gpu {info['self_sweeps']} oracle {ro['self_sweeps']}, K {ro['horizon']}")
    assert tuple(info["self_sweeps"]) == tuple(ro["self_sweeps"])
    assert info["horizon"] == ro["horizon"]
    assert rg["status"] == ro["status"]
    compare_iter(rg, ro, cls, spec["kind"] != "safety", f"{name} auto", q0=ro["q0"], model=m,
                 spec=dict(spec, horizon=ro["horizon"]), optimistic=not pessimistic)


# ---------------------------------------------------------------------------
# disturbance player (eq. (5.1)): rows (s, u, w), worst over w, best over u
# ---------------------------------------------------------------------------

def _disturbed(seed, n_dist=3, d=2, n=7):
    system = W.tiny_affine(d=d, n=n, seed=seed, n_inputs=3)
    rng = np.random.default_rng(seed + 100)
    return dict(system, D=rng.normal(0, 0.3, (d, 2)),
                disturbances=rng.uniform(-0.5, 0.5, (n_dist, 2)))


@pytest.mark.parametrize("storage", ["bounds", "factors"])
def test_disturbance_build_parity(I, storage):
    system = _disturbed(3)
    g = I.build_imdp(system, storage=storage)
    info = g.info()
    assert info["n_dist"] == 3 and info["n_inputs"] == 3
    o = oracle.build(system, system["k_sigma"])
    R = info["n_rows"]
    assert R == o["row_ptr"].size - 1 == 49 * 9
    compare_rows(g.export_rows(0, R), o, R, 2, f"disturbed build [{storage}]")


DIST_SPECS = {
    "reach_avoid": dict(kind="reach_avoid", target=[[[0.5, 0.5], [2.0, 2.0]]],
                        avoid=[[[-2.0, -2.0], [-1.0, -1.0]]]),
    "safety": dict(kind="safety", target=[], avoid=[[[-0.5, -0.5], [0.5, 0.5]]]),
}


@pytest.mark.parametrize("mode", ["state_box", "per_row"])
@pytest.mark.parametrize("horizon", [0, 6])
@pytest.mark.parametrize("pessimistic", [True, False], ids=["pess", "opt"])
@pytest.mark.parametrize("kind", list(DIST_SPECS))
def test_disturbance_iterate_parity(I, kind, pessimistic, horizon, mode):
    system = _disturbed(21 if kind == "safety" else 12)
    spec = dict(DIST_SPECS[kind], eps=1e-8, max_sweeps=1 if horizon else 3000,
                pessimistic=pessimistic, horizon=horizon)
    say(f"disturbed iterate: {kind} pessimistic={pessimistic} horizon={horizon} [{mode}]")
    g = I.build_imdp(system)
    g.set_sweep_modes(mode, mode)
    rg = g.iterate(spec)
    m = oracle.build(system, system["k_sigma"])
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate(m["n_states"], 3, m["row_ptr"], m["target"], m["lo"], m["hi"], cls,
                        spec["kind"], spec["eps"], spec["max_sweeps"], want_q0=True,
                        optimistic=not pessimistic, horizon=horizon, n_dist=3)
    assert rg["status"] == ro["status"]
    compare_iter(rg, ro, cls, kind != "safety", f"disturbed {kind}", q0=ro["q0"], model=m,
                 spec=spec, optimistic=not pessimistic, n_dist=3)


def test_disturbance_with_long_rows_uses_the_workgroup_path(I):
    # dense rows of 26 x 26 + 1 = 677 entries go to the workgroup LP
    system = dict(kind="affine", A=np.eye(2) * 0.8, B=np.eye(2) * 0.5, c=np.zeros(2),
                  lb=[-2.0, -2.0], ub=[2.0, 2.0], n=[26, 26], inputs=[[0.5, 0.0], [0.0, 0.5]],
                  sigma=[0.3, 0.3], k_sigma=0.0, D=np.eye(2) * 0.2,
                  disturbances=[[1.0, 0.0], [0.0, -1.0]])
    spec = dict(kind="reach_avoid", target=[[[1.0, 1.0], [2.0, 2.0]]],
                avoid=[[[-0.5, -0.5], [0.5, 0.5]]], eps=1e-8, max_sweeps=40)
    g = I.build_imdp(system)
    assert g.info()["max_row"] > 512
    rg = g.iterate(spec)
    m = oracle.build(system, 0.0)
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate(m["n_states"], 2, m["row_ptr"], m["target"], m["lo"], m["hi"], cls,
                        spec["kind"], spec["eps"], spec["max_sweeps"], want_q0=True, n_dist=2)
    compare_iter(rg, ro, cls, True, "disturbed long rows", q0=ro["q0"], model=m, spec=spec,
                 n_dist=2)


def test_disturbance_rejections(I):
    system = _disturbed(5)
    with pytest.raises(ValueError):
        I.build_imdp_batch([system])
    uni = dict(W.unicycle3d(n=(6, 6, 4))[0], D=np.eye(3), disturbances=[[0.0, 0.0, 0.0]])
    with pytest.raises(I.ImpactError, match="affine"):
        I.build_imdp(uni)
    bad = dict(system, disturbances=np.array([[0.0, np.nan], [0.1, 0.2]]))
    with pytest.raises(I.ImpactError, match="non-finite"):
        I.build_imdp(bad)
    many = dict(system, disturbances=np.zeros((90, 2)))   # 3 inputs x 90 > 256 rows per state
    with pytest.raises(I.ImpactError, match="256"):
        I.build_imdp(many)


@pytest.mark.parametrize("horizon", [0, "auto"])
@pytest.mark.parametrize("pessimistic", [True, False], ids=["pess", "opt"])
@pytest.mark.parametrize("kind", list(DIST_SPECS))
def test_disturbance_player_in_the_engine_matches_oracle(I, kind, pessimistic, horizon):
    """The multi-query engine runs disturbed abstractions with the selection
    sweep (worst disturbance row per input): against the oracle, both
    policies, the infinite and the automatic horizon, with other queries in
    flight."""
    system = _disturbed(21 if kind == "safety" else 12)
    spec = dict(DIST_SPECS[kind], eps=1e-8, max_sweeps=3000, pessimistic=pessimistic,
                horizon=horizon)
    say(f"disturbed engine: {kind} pessimistic={pessimistic} horizon={horizon}")
    g = I.build_imdp(system)
    other = I.build_imdp(W.tiny_affine(d=2, n=9, seed=2))
    eng = I.Engine(max_queries=4)
    qid = eng.submit(g, spec)
    eng.submit(other, dict(kind="reach", target=[[[0.5, 0.5], [1.5, 1.5]]], avoid=[], eps=1e-6,
                           max_sweeps=200))
    rg = eng.run_all()[qid]
    m = oracle.build(system, system["k_sigma"])
    cls = oracle.label(system, spec["target"], spec["avoid"])
    args = (m["n_states"], 3, m["row_ptr"], m["target"], m["lo"], m["hi"], cls, spec["kind"],
            spec["eps"], spec["max_sweeps"])
    if horizon == "auto":
        ro = oracle.iterate_auto_horizon(*args, want_q0=True, optimistic=not pessimistic,
                                         n_dist=3)
        assert rg["info"]["horizon"] == ro["horizon"]
        assert tuple(rg["info"]["self_sweeps"]) == tuple(ro["self_sweeps"])
        lo, hi = rg["lo"].cpu().numpy(), rg["hi"].cpu().numpy()
        kp = "hi" if not pessimistic else "lo"
        assert np.abs(dict(lo=lo, hi=hi)[kp] - ro[kp]).max() <= VALUE_TOL
    else:
        ro = oracle.iterate(*args, want_q0=True, optimistic=not pessimistic, n_dist=3)
        assert rg["status"] == ro["status"]
        compare_iter(rg, ro, cls, kind != "safety", f"disturbed engine {kind}", q0=ro["q0"],
                     model=m, spec=spec, optimistic=not pessimistic, n_dist=3)
    eng.free()


def test_disturbance_robot2d_state_box_equals_per_row(I):
    # the measured disturbed workload (dense 401-entry rows, 99 rows per state)
    # with a sweep cap: both sweep kernels against the oracle at 25 sweeps
    system, spec = W.robot2d_disturbed()
    spec = dict(spec, max_sweeps=25)
    m = oracle.build(system, 0.0)
    cls = oracle.label(system, spec["target"], spec["avoid"])
    ro = oracle.iterate(m["n_states"], 9, m["row_ptr"], m["target"], m["lo"], m["hi"], cls,
                        spec["kind"], spec["eps"], 25, want_q0=True, n_dist=11)
    for mode in ("state_box", "per_row"):
        g = I.build_imdp(system)
        g.set_sweep_modes(mode, mode)
        rg = g.iterate(spec)
        assert rg["status"] == ro["status"] == 1
        compare_iter(rg, ro, cls, True, f"robot2d disturbed [{mode}]", q0=ro["q0"], model=m,
                     spec=spec, n_dist=11)
