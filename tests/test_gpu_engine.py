"""GPU tests of the multi-query engine (batched and served forms).

A query run by the engine must equal the same query run alone by
impact_interval_iterate with the same sweep kernels (bitwise: the engine runs
the state-box kernel for the policy pass and the per-row kernel for the
fixed-input pass, and the selection sweep for rows beyond 512 entries), must
not depend on which other queries share its launches (bitwise), and must match
the CPU oracle at the parity tolerances.
"""
import numpy as np
import pytest

import oracle
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


def _engine_modes(imdp):
    imdp.set_sweep_modes("state_box", "per_row")
    return imdp


def _np(r):
    return r["lo"].cpu().numpy(), r["hi"].cpu().numpy(), r["policy"].cpu().numpy()


def _same(a, b, label):
    for x, y, k in zip(_np(a), _np(b), ("lo", "hi", "policy")):
        assert np.array_equal(x, y), f"{label}: {k} differs (max {np.abs(x - y).max()})"
    assert tuple(a["info"]["sweeps"]) == tuple(b["info"]["sweeps"]), label


def _affine2():
    return W.tiny_affine(d=2, n=9, seed=2)


def _long_rows():
    # dense 2D rows of 26 x 26 + 1 = 677 entries: the selection-sweep class
    return dict(kind="affine", A=np.eye(2) * 0.8, B=np.eye(2) * 0.5, c=np.zeros(2),
                lb=[-2.0, -2.0], ub=[2.0, 2.0], n=[26, 26], inputs=[[0.5, 0.0], [0.0, 0.5]],
                sigma=[0.3, 0.3], k_sigma=0.0)


CASES = [
    ("affine2_ra", _affine2, dict(kind="reach_avoid", target=[[[0.5, 0.5], [1.5, 1.5]]],
                                  avoid=[[[-1.5, -1.5], [-0.5, -0.5]]], eps=1e-8,
                                  max_sweeps=400)),
    ("affine3_reach", lambda: W.tiny_affine(d=3, n=6, seed=3),
     dict(kind="reach", target=[[[0.0, 0.0, 0.0], [1.3, 1.3, 1.3]]], avoid=[], eps=1e-8,
          max_sweeps=2000)),
    ("affine2_safety", lambda: W.tiny_affine(d=2, n=7, seed=8, k_sigma=0.0),
     dict(kind="safety", target=[], avoid=[[[-0.5, -0.5], [0.5, 0.5]]], eps=1e-8,
          max_sweeps=300)),
    ("unicycle", lambda: dict(W.unicycle3d(n=(10, 10, 6))[0], sigma=[0.3, 0.3, 0.2]),
     dict(kind="reach_avoid", target=[[[2.0, 2.0, -4.0], [5.0, 5.0, 4.0]]],
          avoid=[[[-1.0, -1.0, -4.0], [1.0, 1.0, 4.0]]], eps=1e-8, max_sweeps=3000)),
    ("long_rows", _long_rows, dict(kind="reach_avoid", target=[[[1.0, 1.0], [2.0, 2.0]]],
                                   avoid=[[[-0.5, -0.5], [0.5, 0.5]]], eps=1e-8,
                                   max_sweeps=60)),
]


@pytest.mark.parametrize("pessimistic", [True, False], ids=["pess", "opt"])
@pytest.mark.parametrize("name,make,spec", CASES, ids=[c[0] for c in CASES])
def test_engine_query_equals_plain_iterate(I, name, make, spec, pessimistic):
    system = make()
    spec = dict(spec, pessimistic=pessimistic)
    imdp = _engine_modes(I.build_imdp(system))
    plain = imdp.iterate(spec)
    eng = I.Engine(max_queries=4)
    qid = eng.submit(imdp, spec)
    res = eng.run_all()
    assert set(res) == {qid}
    _same(res[qid], plain, name)
    assert res[qid]["status"] == plain["status"]


def test_engine_alone_equals_in_the_mix(I):
    systems = {name: make() for name, make, _ in CASES}
    imdps = I.build_imdp_batch([systems[n] for n, _, _ in CASES[:4]])
    imdps = dict(zip([n for n, _, _ in CASES[:4]], imdps))
    imdps["long_rows"] = I.build_imdp(systems["long_rows"])
    alone = {}
    for name, _, spec in CASES:
        eng = I.Engine(max_queries=2)
        q = eng.submit(imdps[name], spec)
        alone[name] = eng.run_all()[q]
    # everything at once, plus extra queries on the same abstractions
    eng = I.Engine(max_queries=16)
    ids = {}
    for name, _, spec in CASES:
        ids[eng.submit(imdps[name], spec)] = name
    extra = dict(kind="reach", target=[[[-1.0, -1.0], [0.0, 0.0]]], avoid=[], eps=1e-6,
                 max_sweeps=500)
    eng.submit(imdps["affine2_ra"], extra)
    eng.submit(imdps["long_rows"], dict(extra, max_sweeps=20))
    res = eng.run_all()
    assert len(res) == len(CASES) + 2
    for qid, name in ids.items():
        _same(res[qid], alone[name], f"{name} in the mix")


def test_engine_long_rows_mixed_storage_ragged_segments(I):
    """Selection-sweep queries of both storage modes in one launch (the kernel
    then reads each query's storage), with SAFE sets of 591, 571 and 627
    states: none a multiple of the fixed-input pass's eight-state groups, so
    every later query's segment starts inside a group.  Each result equals
    the same query run alone by the plain call (bitwise)."""
    system = _long_rows()
    specs = [dict(kind="reach_avoid", target=[[[1.0, 1.0], [2.0, 2.0]]],
                  avoid=[[[-0.5, -0.5], [0.5, 0.5]]], eps=1e-8, max_sweeps=60),
             dict(kind="safety", target=[], avoid=[[[-2.0, -2.0], [-1.0, 0.3]]], eps=1e-8,
                  max_sweeps=40),
             dict(kind="reach", target=[[[-1.0, -1.0], [0.0, 0.0]]], avoid=[], eps=1e-6,
                  max_sweeps=50)]
    safe = [int((np.asarray(oracle.label(system, sp["target"], sp["avoid"])) == 0).sum())
            for sp in specs]
    assert safe == [591, 571, 627]
    imdps = {st: _engine_modes(I.build_imdp(system, storage=st)) for st in ("bounds", "factors")}
    assert imdps["bounds"].info()["max_row"] > 512
    plain = {(st, k): imdps[st].iterate(sp) for st in imdps for k, sp in enumerate(specs)}
    for together in (("bounds", "factors"), ("factors",)):
        eng = I.Engine(max_queries=8)
        ids = {eng.submit(imdps[st], sp): (st, k) for k, sp in enumerate(specs) for st in together}
        res = eng.run_all()
        for qid, key in ids.items():
            _same(res[qid], plain[key], f"{key} with {together}")
        eng.free()
    for im in imdps.values():
        im.free()


def test_engine_room5d_long_rows_equal_plain(I):
    """The 5D room at 5 cells per dimension (rows of up to 1,026 entries: the
    5D selection-sweep kernels): safety and reach-avoid queries on stored and
    factored bounds, each storage alone and both in one launch, equal the
    plain call bitwise."""
    system = W.room5d(cells=5)[0]
    specs = [dict(kind="safety", target=[], avoid=[], eps=1e-8, max_sweeps=25),
             dict(kind="reach_avoid", target=[[[20.2] * 5, [21.0] * 5]],
                  avoid=[[[19.0] * 5, [19.8] * 5]], eps=1e-8, max_sweeps=25)]
    imdps = {st: _engine_modes(I.build_imdp(system, storage=st)) for st in ("bounds", "factors")}
    assert imdps["bounds"].info()["max_row"] > 512
    plain = {(st, k): imdps[st].iterate(sp) for st in imdps for k, sp in enumerate(specs)}
    for together in (("bounds",), ("factors",), ("bounds", "factors")):
        eng = I.Engine(max_queries=8)
        ids = {eng.submit(imdps[st], sp): (st, k) for k, sp in enumerate(specs) for st in together}
        res = eng.run_all()
        for qid, key in ids.items():
            _same(res[qid], plain[key], f"room5d {key} with {together}")
        eng.free()
    for im in imdps.values():
        im.free()


def test_engine_matches_oracle_on_batched_instances(I):
    import torch
    rng = np.random.default_rng(7)
    insts = []
    while len(insts) < 6:
        system, spec = W.random_linear(rng, d=2)
        if np.prod(system["n"]) <= 900:
            insts.append((system, spec))
    views = I.build_imdp_batch([s for s, _ in insts], storage="factors")
    eng = I.Engine(max_queries=8)
    ids = [eng.submit(v, dict(spec, max_sweeps=400)) for v, (_, spec) in zip(views, insts)]
    res = eng.run_all()
    for qid, (system, spec) in zip(ids, insts):
        ref = oracle.solve(system, system["k_sigma"], spec["kind"], spec["target"], spec["avoid"],
                           spec["eps"], 400, want_q0=True)
        lo, hi, pol = _np(res[qid])
        assert tuple(res[qid]["info"]["sweeps"]) == tuple(ref["sweeps"])
        assert np.abs(lo - ref["lo"]).max() <= 1e-9 and np.abs(hi - ref["hi"]).max() <= 1e-9
        safe = ref["cls"] == 0
        diff = np.where(safe & (pol != ref["policy"]))[0]
        for s in diff:
            q = ref["q0"][s]
            assert q[pol[s]] >= q.max() - 1e-12
    del torch


def test_engine_reuses_slots_and_handles_degenerate_queries(I):
    system = _affine2()
    imdp = _engine_modes(I.build_imdp(system))
    spec = CASES[0][2]
    ref = imdp.iterate(spec)
    eng = I.Engine(max_queries=2)
    done = {}
    pending = 0
    for k in range(5):  # more queries than slots: poll frees them
        while pending >= 2:
            eng.run(8)
            for r in eng.poll():
                done[r["id"]] = r
                pending -= 1
        eng.submit(imdp, spec)
        pending += 1
    done.update(eng.run_all())
    assert len(done) == 5
    for r in done.values():
        _same(r, ref, "reused slot")
    # every cell a target: nothing to iterate
    q = eng.submit(imdp, dict(kind="reach", target=[[[-2.0, -2.0], [2.0, 2.0]]], avoid=[],
                              eps=1e-8, max_sweeps=10))
    r = eng.run_all()[q]
    assert r["info"]["sweeps"] == (0, 0) and bool((r["lo"] == 1).all())
    assert bool((r["policy"] == -1).all())
    # eps >= 1: no sweeps, outputs from the initial brackets
    q = eng.submit(imdp, dict(spec, eps=2.0))
    r = eng.run_all()[q]
    plain = imdp.iterate(dict(spec, eps=2.0))
    _same(r, plain, "eps >= 1")


@pytest.mark.parametrize("pessimistic", [True, False], ids=["pess", "opt"])
def test_engine_finite_horizon_equals_plain_iterate(I, pessimistic):
    imdps, specs = [], []
    for name, make, spec in CASES:
        imdps.append(_engine_modes(I.build_imdp(make())))
        specs.append(dict(spec, horizon=5 + len(specs), pessimistic=pessimistic))
    plain = [im.iterate(sp) for im, sp in zip(imdps, specs)]
    eng = I.Engine(max_queries=len(CASES))
    ids = [eng.submit(im, sp) for im, sp in zip(imdps, specs)]
    res = eng.run_all()
    for qid, p, (name, _, _), sp in zip(ids, plain, CASES, specs):
        _same(res[qid], p, f"{name} T={sp['horizon']}")
        assert res[qid]["status"] == p["status"] == 0
        assert tuple(res[qid]["info"]["sweeps"]) == (sp["horizon"], sp["horizon"])


@pytest.mark.parametrize("pessimistic", [True, False], ids=["pess", "opt"])
def test_engine_auto_horizon_equals_plain_iterate(I, pessimistic):
    # Remark 5.2 in the engine: a self-convergence stage, then the finite
    # stage of the larger sweep count, the same run as the single-query call
    imdps, specs = [], []
    for name, make, spec in CASES:
        imdps.append(_engine_modes(I.build_imdp(make())))
        specs.append(dict(spec, horizon="auto", pessimistic=pessimistic))
    plain = [im.iterate(sp) for im, sp in zip(imdps, specs)]
    eng = I.Engine(max_queries=len(CASES))
    ids = [eng.submit(im, sp) for im, sp in zip(imdps, specs)]
    res = eng.run_all()
    for qid, p, (name, _, _) in zip(ids, plain, CASES):
        _same(res[qid], p, f"{name} auto")
        assert res[qid]["status"] == p["status"]
        assert res[qid]["info"]["horizon"] == p["info"]["horizon"]
        assert tuple(res[qid]["info"]["self_sweeps"]) == tuple(p["info"]["self_sweeps"])


def test_engine_auto_horizon_matches_oracle(I):
    rng = np.random.default_rng(17)
    insts = []
    while len(insts) < 4:
        system, spec = W.random_linear(rng, d=2)
        if np.prod(system["n"]) <= 900:
            insts.append((system, dict(spec, horizon="auto", max_sweeps=3000)))
    views = I.build_imdp_batch([s for s, _ in insts], storage="factors")
    eng = I.Engine(max_queries=8)
    ids = [eng.submit(v, spec) for v, (_, spec) in zip(views, insts)]
    res = eng.run_all()
    for qid, (system, spec) in zip(ids, insts):
        m = oracle.build(system, system["k_sigma"])
        cls = oracle.label(system, spec["target"], spec["avoid"])
        ref = oracle.iterate_auto_horizon(m["n_states"], m["n_inputs"], m["row_ptr"],
                                          m["target"], m["lo"], m["hi"], cls, spec["kind"],
                                          spec["eps"], spec["max_sweeps"], want_q0=True)
        r = res[qid]
        lo, hi, pol = _np(r)
        assert tuple(r["info"]["self_sweeps"]) == tuple(ref["self_sweeps"])
        assert r["info"]["horizon"] == ref["horizon"]
        assert np.abs(lo - ref["lo"]).max() <= 1e-9
        safe = cls == 0
        diff = np.where(safe & (pol != ref["policy"]))[0]
        for s_ in diff:
            q = ref["q0"][s_]
            assert q[pol[s_]] >= q.max() - 1e-12
        if len(diff) == 0:
            assert np.abs(hi - ref["hi"]).max() <= 1e-9
