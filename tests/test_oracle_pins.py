"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: Gaussian masses are checked
against 50-digit quadrature-grade values from mpmath, min/max bounds against
dense sampling of the source cell, the LP against vertex enumeration and
HiGHS, the iteration against closed-form geometric series, exact-MDP policy
iteration and Monte Carlo simulation of the concrete system.
"""
import itertools
import math

import mpmath
import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.special import ndtr

from paper_2401_03555_amd import workloads as W

mpmath.mp.dps = 50


def mp_mass(a, b, m, s):
    """P(m + w in [a,b]), w ~ N(0, s^2), with 50 significant digits."""
    a, b, m, s = (mpmath.mpf(x) for x in (a, b, m, s))
    return float(mpmath.ncdf((b - m) / s) - mpmath.ncdf((a - m) / s))


def mp_phi(z):
    return float(mpmath.ncdf(mpmath.mpf(z)))


# --------------------------------------------------------------------------
# Per-dimension Gaussian masses (Def. 3.1 with a Gaussian kernel)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("a,b,m,s", [
    (0.0, 1.0, 0.5, 0.25), (1.0, 2.0, 0.5, 0.25), (2.0, 3.0, 0.5, 0.25),
    (-3.0, -2.0, 0.5, 0.25), (5.0, 6.0, 0.0, 0.5), (-1.0, 1.0, 0.0, 1e-3),
    (0.3, 0.5, 0.31, 0.05), (19.0, 19.2, 20.7, 0.05), (-0.2, 0.2, 3.0, 0.4),
    (10.0, 11.0, -1.0, 1.0),
])
def test_gauss_mass_matches_50_digit_values(orc, a, b, m, s):
    got = orc.gauss_cell_mass(a, b, m, s)
    ref = mp_mass(a, b, m, s)
    assert got == pytest.approx(ref, rel=2e-13, abs=1e-300)


def test_gauss_mass_symmetry(orc):
    # cells at +-k around the mean carry equal mass (the tail-aware form keeps this)
    for k in range(0, 8):
        left = orc.gauss_cell_mass(-k - 1.0, -k + 0.0, 0.5 - 0.5, 0.3)
        right = orc.gauss_cell_mass(k + 0.0, k + 1.0, 0.0, 0.3)
        assert left == pytest.approx(right, rel=1e-14, abs=0)


def test_1d_closed_form_bounds(orc):
    # x+ = x + c + w on unit cells, sigma = 1/4 (cell width / sigma = 4), source cell [0,1].
    # Mean interval = source cell shifted by c; min at an end, max at the clamped midpoint.
    s = 0.25
    flo, fhi = orc.factor_bounds(0.0, 1.0, 0.0, 1.0, s)
    assert flo == pytest.approx(mp_phi(4) - 0.5, rel=1e-13)
    assert fhi == pytest.approx(2 * mp_phi(2) - 1, rel=1e-13)  # erf(sqrt 2)
    flo, fhi = orc.factor_bounds(1.0, 2.0, 0.0, 1.0, s)
    assert flo == pytest.approx(mp_phi(8) - mp_phi(4), rel=1e-12)
    assert fhi == pytest.approx(mp_phi(4) - 0.5, rel=1e-13)
    # c = +0.5: mean interval [0.5, 1.5]
    flo, fhi = orc.factor_bounds(0.0, 1.0, 0.5, 1.5, s)
    assert flo == pytest.approx(mp_phi(-2) - mp_phi(-6), rel=1e-13)
    flo, fhi = orc.factor_bounds(-2.0, -1.0, 0.5, 1.5, s)
    assert fhi == pytest.approx(mp_phi(-6) - mp_phi(-10), rel=1e-12)


@pytest.mark.parametrize("mlo,mhi,a,b,s", [
    (0.0, 1.0, 0.0, 1.0, 0.25), (0.2, 0.9, 1.0, 2.0, 0.3), (-0.4, 0.1, 0.0, 0.5, 0.1),
    (3.0, 3.5, 0.0, 1.0, 0.7), (0.45, 0.55, 0.0, 1.0, 0.05),
])
def test_factor_bounds_dense_sampling(orc, mlo, mhi, a, b, s):
    flo, fhi = orc.factor_bounds(a, b, mlo, mhi, s)
    ms = np.linspace(mlo, mhi, 20001)
    vals = np.array([mp_mass(a, b, m, s) for m in ms[::40]] +
                    [mp_mass(a, b, mlo, s), mp_mass(a, b, mhi, s)])
    dense = ndtr((b - ms) / s) - ndtr((a - ms) / s)
    assert vals.min() >= flo - 1e-15 and vals.max() <= fhi + 1e-15
    assert dense.min() >= flo - 1e-14 and dense.max() <= fhi + 1e-14
    # tightness: the extremes are attained (min at an end, max within a sampling step)
    assert abs(min(vals.min(), dense.min()) - flo) < 1e-14
    step = (mhi - mlo) / 20000
    assert fhi - dense.max() < 1e-12 + (step / s) ** 2


# --------------------------------------------------------------------------
# Interval trigonometry and mean boxes (Def. 3.1 min/max over the partition)
# --------------------------------------------------------------------------

def test_interval_cos_sin_dense_sampling(orc):
    rng = np.random.default_rng(7)
    for _ in range(300):
        lo = rng.uniform(-7, 7)
        hi = lo + rng.uniform(0, 3) ** 2
        th = np.linspace(lo, hi, 4001)
        for fn, f in ((orc.interval_cos, np.cos), (orc.interval_sin, np.sin)):
            mn, mx = fn(lo, hi)
            v = f(th)
            assert v.min() >= mn - 1e-15 and v.max() <= mx + 1e-15
            assert v.min() - mn < 2e-6 and mx - v.max() < 2e-6


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_affine_mean_box_contains_and_is_tight(orc, seed):
    system = W.tiny_affine(d=3, n=5, seed=seed)
    rng = np.random.default_rng(seed)
    A, B, c = np.asarray(system["A"]), np.asarray(system["B"]), np.asarray(system["c"])
    n = system["n"]
    for _ in range(20):
        s = int(rng.integers(0, np.prod(n)))
        u = int(rng.integers(0, len(system["inputs"])))
        mlo, mhi = orc.mean_box(system, s, u)
        k = np.unravel_index(s, n)
        lo = np.array([orc.cell_edge(system, i, k[i]) for i in range(3)])
        hi = np.array([orc.cell_edge(system, i, k[i] + 1) for i in range(3)])
        corners = np.array(list(itertools.product(*zip(lo, hi))))
        f = corners @ A.T + B @ system["inputs"][u] + c
        assert (f >= mlo - 1e-15).all() and (f <= mhi + 1e-15).all()
        assert np.abs(f.min(0) - mlo).max() < 1e-12 and np.abs(f.max(0) - mhi).max() < 1e-12


def test_unicycle_mean_box_contains(orc):
    system, _ = W.unicycle3d(n=(6, 6, 7))
    rng = np.random.default_rng(3)
    for _ in range(40):
        s = int(rng.integers(0, 6 * 6 * 7))
        u = int(rng.integers(0, 20))
        mlo, mhi = orc.mean_box(system, s, u)
        k = np.unravel_index(s, (6, 6, 7))
        lo = np.array([orc.cell_edge(system, i, k[i]) for i in range(3)])
        hi = np.array([orc.cell_edge(system, i, k[i] + 1) for i in range(3)])
        x = rng.uniform(lo, hi, size=(4000, 3))
        v, om = system["inputs"][u]
        f = np.stack([x[:, 0] + 0.1 * v * np.cos(x[:, 2]), x[:, 1] + 0.1 * v * np.sin(x[:, 2]),
                      x[:, 2] + 0.1 * om], 1)
        assert (f >= mlo).all() and (f <= mhi).all()
        assert (mhi - mlo).max() < (hi - lo).max() + 0.3


@pytest.mark.parametrize("n", [(6, 6, 7), (10, 10, 24), (4, 4, 3)])
def test_unicycle_mean_box_is_tight(orc, n):
    """Each successor coordinate is a sum of functions of separate state
    coordinates (x0 + dt v cos th, x1 + dt v sin th, th + dt om), so its range
    over the cell is reached: a dense tensor grid of the cell (its corners and
    2,001 headings) attains the box up to the grid's resolution and the
    2^-48 padding.  An over-wide enclosure (a missed extremum test, a
    dropped clamp, cos/sin ranges taken over too wide a heading interval)
    fails the tightness bound."""
    system, _ = W.unicycle3d(n=n)
    N = int(np.prod(n))
    rng = np.random.default_rng(4)
    for _ in range(30):
        s = int(rng.integers(0, N))
        u = int(rng.integers(0, 20))
        mlo, mhi = orc.mean_box(system, s, u)
        k = np.unravel_index(s, n)
        lo = np.array([orc.cell_edge(system, i, k[i]) for i in range(3)])
        hi = np.array([orc.cell_edge(system, i, k[i] + 1) for i in range(3)])
        th = np.linspace(lo[2], hi[2], 2001)
        v, om = system["inputs"][u]
        x0 = np.array([lo[0], hi[0]])[:, None]
        x1 = np.array([lo[1], hi[1]])[:, None]
        f0 = (x0 + 0.1 * v * np.cos(th)[None, :]).ravel()
        f1 = (x1 + 0.1 * v * np.sin(th)[None, :]).ravel()
        f2 = th + 0.1 * om
        smin = np.array([f0.min(), f1.min(), f2.min()])
        smax = np.array([f0.max(), f1.max(), f2.max()])
        # heading spacing h: the sampled extremum of dt v cos/sin is within
        # dt v h^2 / 8 of the true one; padding <= 2^-48 * (|x| + dt v + |th|)
        h = (hi[2] - lo[2]) / 2000
        tol = 0.1 * v * h * h / 8 + 1e-12
        assert (mlo <= smin + 1e-15).all() and (mhi >= smax - 1e-15).all()
        assert (smin - mlo).max() <= tol and (mhi - smax).max() <= tol, (s, u, smin - mlo, mhi - smax)


# --------------------------------------------------------------------------
# Rows of the abstraction: containment, invariants, OUT / TAIL
# --------------------------------------------------------------------------

def _exact_row(system, x, u):
    """Exact one-step masses from the concrete point x (dense over all cells), via scipy ndtr."""
    lb, ub, n = map(np.asarray, (system["lb"], system["ub"], system["n"]))
    sigma = np.asarray(system["sigma"])
    uv = np.asarray(system["inputs"][u])
    if system["kind"] == "affine":
        m = np.asarray(system["A"]) @ x + np.asarray(system["B"]) @ uv + np.asarray(system["c"])
    else:
        m = np.array([x[0] + 0.1 * uv[0] * np.cos(x[2]), x[1] + 0.1 * uv[0] * np.sin(x[2]),
                      x[2] + 0.1 * uv[1]])
    per_dim = []
    for i in range(len(n)):
        e = lb[i] + (ub[i] - lb[i]) / n[i] * np.arange(n[i] + 1)
        e[-1] = ub[i]
        per_dim.append(ndtr((e[1:] - m[i]) / sigma[i]) - ndtr((e[:-1] - m[i]) / sigma[i]))
    T = per_dim[0]
    for p in per_dim[1:]:
        T = np.multiply.outer(T, p)
    out = 1 - np.prod([1 - (ndtr((lb[i] - m[i]) / sigma[i]) + ndtr((m[i] - ub[i]) / sigma[i]))
                       for i in range(len(n))])
    return T.reshape(-1), out


@pytest.mark.parametrize("case", ["affine2", "affine3", "unicycle", "dense2"])
def test_row_containment_by_sampling(orc, case):
    if case == "affine2":
        system = W.tiny_affine(d=2, n=7, seed=4)
    elif case == "affine3":
        system = W.tiny_affine(d=3, n=4, seed=5)
    elif case == "dense2":
        system = W.tiny_affine(d=2, n=6, seed=6, k_sigma=0.0)
    else:
        system, _ = W.unicycle3d(n=(8, 8, 6))
        system["sigma"] = [0.4, 0.4, 0.3]
    m = orc.build(system, system["k_sigma"])
    rng = np.random.default_rng(11)
    n = system["n"]
    n_states = int(np.prod(n))
    nu = m["n_inputs"]
    d = len(n)
    rows = rng.choice(n_states * nu, size=min(25, n_states * nu), replace=False)
    for r in rows:
        s, u = divmod(int(r), nu)
        k = np.unravel_index(s, n)
        lo_e = np.array([orc.cell_edge(system, i, k[i]) for i in range(d)])
        hi_e = np.array([orc.cell_edge(system, i, k[i] + 1) for i in range(d)])
        b, e = m["row_ptr"][r], m["row_ptr"][r + 1]
        tgt, lo, hi = m["target"][b:e], m["lo"][b:e], m["hi"][b:e]
        cells = tgt >= 0
        for x in rng.uniform(lo_e, hi_e, size=(30, d)):
            T, out = _exact_row(system, x, u)
            assert (T[tgt[cells]] >= lo[cells] - 1e-14).all()
            assert (T[tgt[cells]] <= hi[cells] + 1e-14).all()
            io = np.where(tgt == -1)[0][0]
            assert lo[io] - 1e-14 <= out <= hi[io] + 1e-14
            if m["windowed"]:
                it = np.where(tgt == -2)[0][0]
                outside = np.ones(len(T), bool)
                outside[tgt[cells]] = False
                assert T[outside].sum() <= hi[it] + 1e-14


def test_row_invariants_and_low_cost_rule(orc):
    for system in (W.tiny_affine(d=2, n=9, seed=2), W.tiny_affine(d=3, n=5, seed=3),
                   W.tiny_affine(d=2, n=5, seed=8, k_sigma=0.0), W.robot2d()[0]):
        m = orc.build(system, system["k_sigma"])
        rp, lo, hi = m["row_ptr"], m["lo"], m["hi"]
        assert (lo >= 0).all() and (hi <= 1).all() and (lo <= hi).all()
        assert (lo[hi == 0] == 0).all()  # Section 4.4: T_max = 0 implies T_min = 0
        slo = np.add.reduceat(lo, rp[:-1])
        shi = np.add.reduceat(hi, rp[:-1])
        assert slo.max() <= 1 + 1e-14 and shi.min() >= 1 - 1e-14


def test_windowed_entries_equal_dense_entries(orc):
    system = W.tiny_affine(d=2, n=12, seed=9)
    system["sigma"] = [0.05, 0.05]
    mw = orc.build(system, 6.0)
    md = orc.build(system, 0.0)
    for r in range(md["row_ptr"].size - 1):
        bw, ew = mw["row_ptr"][r], mw["row_ptr"][r + 1]
        bd, ed = md["row_ptr"][r], md["row_ptr"][r + 1]
        dense_hi = dict(zip(md["target"][bd:ed], md["hi"][bd:ed]))
        dense_lo = dict(zip(md["target"][bd:ed], md["lo"][bd:ed]))
        tw = mw["target"][bw:ew]
        cells = tw >= 0
        assert np.array_equal(mw["lo"][bw:ew][cells], [dense_lo[t] for t in tw[cells]])
        assert np.array_equal(mw["hi"][bw:ew][cells], [dense_hi[t] for t in tw[cells]])
        assert mw["lo"][bw:ew][-2] == md["lo"][ed - 1] and mw["hi"][bw:ew][-2] == md["hi"][ed - 1]
        tail_hi = mw["hi"][ew - 1]
        outside = [dense_hi[t] for t in dense_hi if t >= 0 and t not in set(tw[cells])]
        assert all(h <= tail_hi + 1e-16 for h in outside)


def test_tail_closed_form_1d(orc):
    # x+ = x + w, unit cells on [-50,50], sigma = 1/4, k = 6: the mean box is the source
    # cell (padded), the window is cells k-2 .. k+2, and the largest escape probability
    # from the window box, attained at an end of the mean interval, is Phi(-8) + Phi(-12).
    system = dict(kind="affine", A=[[1.0]], B=[[0.0]], c=[0.0], lb=[-50.0], ub=[50.0], n=[100],
                  inputs=[[0.0]], sigma=[0.25], k_sigma=6.0)
    m = orc.build(system, 6.0, rows=[50])
    assert list(m["win"][0]) == [48, 5]
    assert m["ot"][0, 3] == pytest.approx(mp_phi(-8) + mp_phi(-12), rel=1e-9)
    # 3D product form 1 - (1 - p)^3 for the same geometry in every dimension
    system3 = dict(kind="affine", A=np.eye(3), B=np.zeros((3, 1)), c=np.zeros(3),
                   lb=[-50.0] * 3, ub=[50.0] * 3, n=[100] * 3, inputs=[[0.0]], sigma=[0.25] * 3,
                   k_sigma=6.0)
    row = 50 * 100 * 100 + 50 * 100 + 50
    m3 = orc.build(system3, 6.0, rows=[row])
    p = mpmath.ncdf(-8) + mpmath.ncdf(-12)
    assert m3["ot"][0, 3] == pytest.approx(float(1 - (1 - p) ** 3), rel=1e-9)


def test_out_entry_closed_form_1d(orc):
    # boundary cell [9,10] of [-10,10], x+ = x + w, sigma = 0.5: exit mass at m is
    # Phi((-10-m)/s) + Phi((m-10)/s); max at m = 10, min at m = 9
    system = dict(kind="affine", A=[[1.0]], B=[[0.0]], c=[0.0], lb=[-10.0], ub=[10.0], n=[20],
                  inputs=[[0.0]], sigma=[0.5], k_sigma=0.0)
    m = orc.build(system, 0.0, rows=[19])
    out_lo, out_hi = m["ot"][0, 0], m["ot"][0, 1]
    assert out_hi == pytest.approx(mp_phi(-40) + mp_phi(0), rel=1e-12)
    assert out_lo == pytest.approx(mp_phi(-38) + mp_phi(-2), rel=1e-12)


# --------------------------------------------------------------------------
# LP of eq. (5.1) by the sorting method
# --------------------------------------------------------------------------

def _vertex_lp(lo, hi, val, maximise):
    """Enumerate vertices of {lo <= p <= hi, sum p = 1}: all but one coordinate at a bound."""
    n = len(lo)
    best = None
    for free in range(n):
        others = [j for j in range(n) if j != free]
        for pick in itertools.product((0, 1), repeat=n - 1):
            p = np.zeros(n)
            for j, b in zip(others, pick):
                p[j] = hi[j] if b else lo[j]
            p[free] = 1 - p.sum()
            if lo[free] - 1e-15 <= p[free] <= hi[free] + 1e-15:
                v = float(p @ val)
                if best is None or (v > best if maximise else v < best):
                    best = v
    return best


def _random_intervals(rng, n):
    while True:
        lo = rng.uniform(0, 1, n) * rng.uniform(0, 2 / n)
        hi = lo + rng.uniform(0, 1, n) * rng.uniform(0, 3 / n)
        if lo.sum() <= 1 <= hi.sum():
            return lo, np.minimum(hi, 1)


def test_lp_matches_vertex_enumeration(orc):
    rng = np.random.default_rng(5)
    for trial in range(300):
        n = int(rng.integers(1, 9))
        lo, hi = _random_intervals(rng, n)
        val = rng.uniform(0, 1, n)
        if trial % 3 == 0:
            val = np.round(val * 3) / 3  # many ties
        for mx in (False, True):
            q, p = orc.lp_sorted(lo, hi, val, mx)
            assert q == pytest.approx(_vertex_lp(lo, hi, val, mx), abs=1e-12)
            assert (p >= lo - 1e-15).all() and (p <= hi + 1e-15).all()
            assert p.sum() == pytest.approx(1.0, abs=1e-14)


def test_lp_matches_highs(orc):
    rng = np.random.default_rng(6)
    for _ in range(40):
        n = int(rng.integers(10, 300))
        lo, hi = _random_intervals(rng, n)
        val = rng.uniform(0, 1, n)
        for mx in (False, True):
            q, _ = orc.lp_sorted(lo, hi, val, mx)
            res = linprog(-val if mx else val, A_eq=np.ones((1, n)), b_eq=[1.0],
                          bounds=list(zip(lo, hi)), method="highs")
            ref = -res.fun if mx else res.fun
            assert q == pytest.approx(ref, abs=1e-9)


# --------------------------------------------------------------------------
# Interval iteration: worked single-state examples (closed forms of eq. (5.2))
# --------------------------------------------------------------------------

def test_worked_reach_avoid_single_state(orc):
    # state 0 SAFE with entries (self, TARGET=state 1, AVOID=state 2):
    # lo = (.3,.1,.2), hi = (.6,.3,.5).  Pass 1 (minimising LP): p = (.4,.1,.5),
    # V' = .1 + .4 V, gap .4^k -> 21 sweeps, V0 = (1 - .4^21)/6.
    # Pass 2 (maximising LP): p = (.5,.3,.2), V' = .3 + .5 V, gap .5^k -> 27 sweeps,
    # V1 = .6 + .4 * .5^27.
    row_ptr = [0, 3, 3, 3]
    r = orc.iterate(3, 1, row_ptr, [0, 1, 2], [.3, .1, .2], [.6, .3, .5],
                    np.array([0, 1, 2], np.int8), "reach_avoid", 1e-8, 1000)
    assert r["sweeps"] == (21, 27) and r["converged"] == (1, 1) and r["status"] == 0
    assert r["lo"][0] == pytest.approx((1 - 0.4 ** 21) / 6, abs=1e-15)
    assert r["hi"][0] == pytest.approx(0.6 + 0.4 * 0.5 ** 27, abs=1e-15)
    assert list(r["lo"][1:]) == [1.0, 0.0] and list(r["hi"][1:]) == [1.0, 0.0]
    assert list(r["policy"]) == [0, -1, -1]


def test_worked_safety_single_state(orc):
    # self [.7,.9], OUT [.1,.25].  Pass 1 (maximising LP): OUT .25, self .75 -> V* = 1,
    # gap .75^k -> 65 sweeps.  Pass 2 (minimising LP): OUT .1, self .9 -> gap .9^k ->
    # 175 sweeps.  Outer outputs: lo = 1 - V1 = 0, hi = 1 - V0 = .9^175.
    r = orc.iterate(1, 1, [0, 2], [0, -1], [.7, .1], [.9, .25], np.array([0], np.int8),
                    "safety", 1e-8, 1000)
    assert r["sweeps"] == (65, 175)
    assert r["gap"][0] == pytest.approx(0.75 ** 65, rel=1e-12)
    assert r["lo"][0] == 0.0
    assert r["hi"][0] == pytest.approx(0.9 ** 175, rel=1e-11)
    assert r["lo"][0] <= r["hi"][0]


def test_non_convergence_hits_cap(orc):
    # self [.9,1], OUT [0,.1] under safety: pass 2 (minimising LP) puts all mass on self,
    # so V0 stays 0 and V1 stays 1 -- the cap must end the pass.
    r = orc.iterate(1, 1, [0, 2], [0, -1], [.9, 0.0], [1.0, .1], np.array([0], np.int8),
                    "safety", 1e-8, 500)
    assert r["status"] == 1 and r["converged"] == (1, 0)
    assert r["sweeps"][1] == 500 and r["gap"][1] == 1.0
    assert r["lo"][0] == 0.0 and r["hi"][0] == 1.0


# --------------------------------------------------------------------------
# Interval iteration against textbook reductions
# --------------------------------------------------------------------------

def _random_exact_mdp(rng, n_safe, n_u, n_cells_extra=2):
    """Rows with lo == hi (a plain MDP); every row leaks >= 5% to TARGET / AVOID."""
    n = n_safe + n_cells_extra
    cls = np.array([0] * n_safe + [1, 2], np.int8)
    row_ptr, tgt, p = [0], [], []
    for s in range(n):
        for u in range(n_u):
            if s >= n_safe:
                row_ptr.append(row_ptr[-1])
                continue
            support = rng.choice(n_safe, size=min(4, n_safe), replace=False)
            w = rng.uniform(0.1, 1, len(support) + 2)
            w[-2:] = np.maximum(w[-2:], 0.05 * w.sum())
            w /= w.sum()
            tgt += list(support) + [n_safe, n_safe + 1]
            p += list(w)
            row_ptr.append(row_ptr[-1] + len(support) + 2)
    return n, cls, np.array(row_ptr), np.array(tgt), np.array(p)


def _policy_iteration(n_safe, n_u, row_ptr, tgt, p, value_of_avoid, maximise):
    pi = np.zeros(n_safe, int)
    for _ in range(100):
        P = np.zeros((n_safe, n_safe))
        b = np.zeros(n_safe)
        for s in range(n_safe):
            r = s * n_u + pi[s]
            for t, w in zip(tgt[row_ptr[r]:row_ptr[r + 1]], p[row_ptr[r]:row_ptr[r + 1]]):
                if t < n_safe:
                    P[s, t] += w
                elif t == n_safe:
                    b[s] += w * (1.0 - value_of_avoid)  # TARGET
                else:
                    b[s] += w * value_of_avoid  # AVOID
        V = np.linalg.solve(np.eye(n_safe) - P, b)
        Q = np.zeros((n_safe, n_u))
        for s in range(n_safe):
            for u in range(n_u):
                r = s * n_u + u
                ts, ws = tgt[row_ptr[r]:row_ptr[r + 1]], p[row_ptr[r]:row_ptr[r + 1]]
                Q[s, u] = sum(w * (V[t] if t < n_safe else (1.0 - value_of_avoid if t == n_safe
                                                             else value_of_avoid))
                              for t, w in zip(ts, ws))
        new = Q.argmax(1) if maximise else Q.argmin(1)
        better = Q[np.arange(n_safe), new] > Q[np.arange(n_safe), pi] + 1e-13 if maximise else \
            Q[np.arange(n_safe), new] < Q[np.arange(n_safe), pi] - 1e-13
        if not better.any():
            return V
        pi = np.where(better, new, pi)
    raise AssertionError("policy iteration did not settle")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_mdp_reach_avoid_equals_policy_iteration(orc, seed):
    rng = np.random.default_rng(seed)
    n, cls, rp, tgt, p = _random_exact_mdp(rng, 12, 3)
    r = orc.iterate(n, 3, rp, tgt, p, p, cls, "reach_avoid", 1e-10, 100000)
    V = _policy_iteration(12, 3, rp, tgt, p, 0.0, True)  # AVOID value 0, TARGET value 1
    assert np.allclose(r["lo"][:12], V, atol=1e-9) and np.allclose(r["hi"][:12], V, atol=1e-9)


@pytest.mark.parametrize("seed", [3, 4])
def test_exact_mdp_safety_equals_policy_iteration(orc, seed):
    rng = np.random.default_rng(seed)
    n, cls, rp, tgt, p = _random_exact_mdp(rng, 10, 2)
    cls = cls.copy()
    cls[-2] = 2  # safety has no TARGET set: both absorbing cells are unsafe
    r = orc.iterate(n, 2, rp, tgt, p, p, cls, "safety", 1e-10, 100000)
    # probability of reaching the unsafe set, minimised over inputs; both sinks have value 1
    pi = np.zeros(10, int)
    for _ in range(100):
        P = np.zeros((10, 10))
        b = np.zeros(10)
        for s in range(10):
            rr = s * 2 + pi[s]
            for t, w in zip(tgt[rp[rr]:rp[rr + 1]], p[rp[rr]:rp[rr + 1]]):
                if t < 10:
                    P[s, t] += w
                else:
                    b[s] += w
        V = np.linalg.solve(np.eye(10) - P, b)
        Q = np.array([[sum(w * (V[t] if t < 10 else 1.0)
                           for t, w in zip(tgt[rp[s * 2 + u]:rp[s * 2 + u + 1]],
                                           p[rp[s * 2 + u]:rp[s * 2 + u + 1]]))
                       for u in range(2)] for s in range(10)])
        new = Q.argmin(1)
        better = Q[np.arange(10), new] < Q[np.arange(10), pi] - 1e-13
        if not better.any():
            break
        pi = np.where(better, new, pi)
    assert np.allclose(r["lo"][:10], 1 - V, atol=1e-9) and np.allclose(r["hi"][:10], 1 - V, atol=1e-9)


def test_sweeps_are_monotone_and_ordered(orc):
    system = W.tiny_affine(d=2, n=8, seed=12)
    m = orc.build(system, system["k_sigma"])
    cls = orc.label(system, [[[0.5, 0.5], [1.5, 1.5]]], [[[-1.5, -1.5], [-0.5, -0.5]]])
    r = orc.iterate(m["n_states"], m["n_inputs"], m["row_ptr"], m["target"], m["lo"], m["hi"],
                    cls, "reach_avoid", 1e-8, 60, hist_cap=60)
    h0, h1 = r["hist_v0"][:r["sweeps"][0]], r["hist_v1"][:r["sweeps"][0]]
    safe = cls == 0
    assert (np.diff(h0[:, safe], axis=0) >= -1e-15).all()
    assert (np.diff(h1[:, safe], axis=0) <= 1e-15).all()
    assert (h0[:, safe] <= h1[:, safe] + 1e-15).all()
    assert (r["lo"] <= r["hi"] + 1e-12).all()


def test_reach_is_reach_avoid_without_avoid(orc):
    system = W.tiny_affine(d=2, n=7, seed=13)
    m = orc.build(system, system["k_sigma"])
    cls = orc.label(system, [[[0.0, 0.0], [1.0, 1.0]]], None)
    a = orc.iterate(m["n_states"], m["n_inputs"], m["row_ptr"], m["target"], m["lo"], m["hi"],
                    cls, "reach", 1e-8, 5000)
    b = orc.iterate(m["n_states"], m["n_inputs"], m["row_ptr"], m["target"], m["lo"], m["hi"],
                    cls, "reach_avoid", 1e-8, 5000)
    for k in ("lo", "hi", "policy"):
        assert np.array_equal(a[k], b[k])


def test_aggregated_target_avoid_rows_give_the_same_lp(orc):
    # Section 3.1: target / avoid transitions may be summed into R and A entries.
    # With equal values inside each class the per-entry LP has the same optimum.
    rng = np.random.default_rng(21)
    for _ in range(200):
        n = int(rng.integers(3, 12))
        lo, hi = _random_intervals(rng, n)
        cls = rng.integers(0, 3, n)
        v = np.where(cls == 0, rng.uniform(0, 1, n), np.where(cls == 1, 1.0, 0.0))
        keep = cls == 0
        lo_a = np.concatenate([lo[keep], [lo[cls == 1].sum(), lo[cls == 2].sum()]])
        hi_a = np.concatenate([hi[keep], [hi[cls == 1].sum(), hi[cls == 2].sum()]])
        v_a = np.concatenate([v[keep], [1.0, 0.0]])
        for mx in (False, True):
            assert orc.lp_sorted(lo, hi, v, mx)[0] == pytest.approx(
                orc.lp_sorted(lo_a, hi_a, v_a, mx)[0], abs=1e-14)


def test_imc_has_trivial_policy(orc):
    system = W.tiny_affine(d=2, n=6, seed=14, n_inputs=1)
    m = orc.build(system, system["k_sigma"])
    cls = orc.label(system, [[[0.0, 0.0], [1.0, 1.0]]], None)
    r = orc.iterate(m["n_states"], 1, m["row_ptr"], m["target"], m["lo"], m["hi"], cls, "reach",
                    1e-8, 5000)
    assert set(r["policy"][cls == 0]) == {0}


# --------------------------------------------------------------------------
# Optimistic policy (IMDP_lower = false, Sec. 5): the policy is optimised on
# the favourable LP and fixed for the adversarial one
# --------------------------------------------------------------------------

def _two_input_choice():
    # state 0 SAFE, 1 TARGET, 2 AVOID; input 0: target and avoid in [.4, .6];
    # input 1: target and avoid in [.1, .9].  Rows of the non-SAFE states are empty.
    row_ptr = [0, 2, 4, 4, 4, 4, 4]
    target = [1, 2, 1, 2]
    lo = [.4, .4, .1, .1]
    hi = [.6, .6, .9, .9]
    return row_ptr, target, lo, hi, np.array([0, 1, 2], np.int8)


def test_worked_pessimistic_and_optimistic_policies(orc):
    # Pessimistic: the adversary puts the free mass on AVOID, so input 0 is
    # worth .4 and input 1 only .1 -> pi = 0, lo = .4; with pi fixed the
    # favourable LP gives hi = .6.  Optimistic: the favourable LP gives .6 vs
    # .9 -> pi = 1, hi = .9; fixed, the adversarial LP gives lo = .1.
    # Every LP here is exact after one sweep (no self loop).
    row_ptr, target, lo, hi, cls = _two_input_choice()
    p = orc.iterate(3, 2, row_ptr, target, lo, hi, cls, "reach_avoid", 1e-8, 100)
    o = orc.iterate(3, 2, row_ptr, target, lo, hi, cls, "reach_avoid", 1e-8, 100,
                    optimistic=True)
    assert p["policy"][0] == 0 and o["policy"][0] == 1
    assert (p["lo"][0], p["hi"][0]) == (pytest.approx(0.4, abs=1e-15), pytest.approx(0.6, abs=1e-15))
    assert (o["lo"][0], o["hi"][0]) == (pytest.approx(0.1, abs=1e-15), pytest.approx(0.9, abs=1e-15))
    assert p["status"] == 0 and o["status"] == 0


def test_optimistic_equals_pessimistic_without_choice(orc):
    # one input: no policy to choose, the two passes swap places only
    system = W.tiny_affine(d=2, n=6, seed=14, n_inputs=1)
    m = orc.build(system, system["k_sigma"])
    cls = orc.label(system, [[[0.0, 0.0], [1.0, 1.0]]], [[[-1.0, -1.0], [-0.4, -0.4]]])
    for kind in ("reach_avoid", "safety"):
        c = cls.copy()
        if kind == "safety":
            c[c == 1] = 0
        args = (m["n_states"], 1, m["row_ptr"], m["target"], m["lo"], m["hi"], c, kind, 1e-8, 5000)
        p = orc.iterate(*args)
        o = orc.iterate(*args, optimistic=True)
        assert np.array_equal(p["lo"], o["lo"]) and np.array_equal(p["hi"], o["hi"])
        assert p["sweeps"] == o["sweeps"][::-1]


@pytest.mark.parametrize("seed", [12, 21, 24])
def test_optimistic_policy_orders_the_bounds(orc, seed):
    # hi_opt bounds max over policies of P_max from above; lo_opt is a lower
    # bound of P_min under one policy, at most max over policies of P_min,
    # which lo_pess approximates from below within eps (and vice versa).
    system = W.tiny_affine(d=2, n=7, seed=seed, n_inputs=4)
    m = orc.build(system, system["k_sigma"])
    cls = orc.label(system, [[[0.5, 0.5], [2.0, 2.0]]], [[[-2.0, -2.0], [-1.0, -1.0]]])
    eps = 1e-9
    args = (m["n_states"], 4, m["row_ptr"], m["target"], m["lo"], m["hi"], cls, "reach_avoid",
            eps, 20000)
    p = orc.iterate(*args)
    o = orc.iterate(*args, optimistic=True)
    assert p["status"] == 0 and o["status"] == 0
    assert np.all(p["hi"] <= o["hi"] + eps)
    assert np.all(o["lo"] <= p["lo"] + eps)
    assert np.all(o["lo"] <= o["hi"] + eps)
    assert (o["hi"] - p["hi"]).max() > 1e-3  # the optimistic policy does raise the upper bound


# --------------------------------------------------------------------------
# Soundness against the concrete system (Monte Carlo under the synthesized policy)
# --------------------------------------------------------------------------

def test_monte_carlo_reach_avoid_within_bounds(orc):
    system = dict(kind="affine", A=np.eye(2) * 0.9, B=np.eye(2) * 0.6, c=np.zeros(2),
                  lb=[-3.0, -3.0], ub=[3.0, 3.0], n=[6, 6],
                  inputs=np.array(list(itertools.product([-1.0, 0.0, 1.0], repeat=2))),
                  sigma=[0.35, 0.35], k_sigma=0.0)
    target = [[[1.0, 1.0], [3.0, 3.0]]]
    avoid = [[[-1.0, -1.0], [0.0, 0.0]]]
    res = orc.solve(system, 0.0, "reach_avoid", target, avoid, 1e-9, 100000)
    cls, pol = res["cls"], res["policy"]
    rng = np.random.default_rng(99)
    A, B = system["A"], system["B"]
    n_paths, H = 4000, 200
    for s in rng.choice(np.where(cls == 0)[0], size=6, replace=False):
        k = np.unravel_index(s, (6, 6))
        x = np.stack([rng.uniform(-3 + k[0], -2 + k[0], n_paths),
                      rng.uniform(-3 + k[1], -2 + k[1], n_paths)], 1)
        alive = np.ones(n_paths, bool)
        hit = np.zeros(n_paths, bool)
        for _ in range(H):
            idx = np.clip(np.floor(x + 3).astype(int), 0, 5)
            cell = idx[:, 0] * 6 + idx[:, 1]
            u = system["inputs"][np.maximum(pol[cell], 0)]
            x = x @ A.T + u @ B.T + rng.normal(scale=0.35, size=x.shape)
            inside = (np.abs(x) <= 3).all(1)
            idx = np.clip(np.floor(x + 3).astype(int), 0, 5)
            c2 = cls[idx[:, 0] * 6 + idx[:, 1]]
            newly_hit = alive & inside & (c2 == 1)
            dead = alive & (~inside | (c2 == 2))
            hit |= newly_hit
            alive &= ~(newly_hit | dead)
        p = hit.mean()
        sd = max(np.sqrt(p * (1 - p) / n_paths), 1e-3)
        assert p <= res["hi"][s] + 4 * sd
        assert p + alive.mean() >= res["lo"][s] - 4 * sd


# --------------------------------------------------------------------------
# Labels (centre rule) against counts fixed by the workload geometry
# --------------------------------------------------------------------------

def test_label_counts(orc):
    sysd, spec = W.robot2d()
    cls = orc.label(sysd, spec["target"], spec["avoid"])
    assert list(np.bincount(cls, minlength=3)) == [375, 9, 16]
    sysd, spec = W.unicycle3d()
    cls = orc.label(sysd, spec["target"], spec["avoid"])
    assert list(np.bincount(cls, minlength=3)) == [53664, 1536, 4800]


@pytest.mark.parametrize("optimistic", [False, True])
def test_fixed_input_pass_depends_on_the_policy_alone(orc, optimistic):
    # Alg. 3/4: the second pass restarts from the initial vectors with u fixed
    # by the first pass's policy, so it equals the run of the induced IMC
    system = W.tiny_affine(d=2, n=7, seed=12, n_inputs=4)
    m = orc.build(system, system["k_sigma"])
    cls = orc.label(system, [[[0.5, 0.5], [2.0, 2.0]]], [[[-2.0, -2.0], [-1.0, -1.0]]])
    full = orc.iterate(m["n_states"], 4, m["row_ptr"], m["target"], m["lo"], m["hi"], cls,
                       "reach_avoid", 1e-9, 20000, optimistic=optimistic)
    rows = np.arange(m["n_states"]) * 4 + np.maximum(full["policy"], 0)
    starts, ends = m["row_ptr"][rows], m["row_ptr"][rows + 1]
    idx = np.concatenate([np.arange(a, b) for a, b in zip(starts, ends)])
    rp = np.concatenate([[0], np.cumsum(ends - starts)]).astype(np.int64)
    imc = orc.iterate(m["n_states"], 1, rp, m["target"][idx], m["lo"][idx], m["hi"][idx], cls,
                      "reach_avoid", 1e-9, 20000, optimistic=optimistic)
    k = "lo" if optimistic else "hi"
    assert imc["sweeps"][1] == full["sweeps"][1]
    assert np.array_equal(imc[k], full[k])


# --------------------------------------------------------------------------
# Finite horizon (Remark 5.1): each pass is T sweeps of value iteration
# --------------------------------------------------------------------------

def _self_loop_choice(kind):
    # state 0 SAFE, state 1 TARGET (reach) or AVOID (safety).  Each input keeps
    # the chain in state 0 or moves it to state 1; the move's probability is
    # in [.3, .4] under input 0 and in [.2, .6] under input 1.
    row_ptr = [0, 2, 4, 4, 4]
    target = [0, 1, 0, 1]
    lo = [.6, .3, .4, .2]
    hi = [.7, .4, .8, .6]
    return row_ptr, target, lo, hi, np.array([0, 1 if kind != "safety" else 2], np.int8)


@pytest.mark.parametrize("T", [1, 3, 10])
def test_finite_horizon_geometric_closed_forms(orc, T):
    # reach within T steps with a per-step move probability q: 1 - (1 - q)^T;
    # staying safe for T steps: (1 - q)^T.  The adversary's q is an end of the
    # interval at every step.  Pessimistic: reach takes u maximising the worst
    # q (input 0, .3), safety u minimising the worst q (input 0, .4); the
    # optimistic policy takes the best q (input 1: .6 to reach, .2 to fail).
    cases = {
        ("reach", False): (0, 1 - .7 ** T, 1 - .6 ** T),
        ("reach", True): (1, 1 - .8 ** T, 1 - .4 ** T),
        ("safety", False): (0, .6 ** T, .7 ** T),
        ("safety", True): (1, .4 ** T, .8 ** T),
    }
    for (kind, opt), (pi, lo, hi) in cases.items():
        row_ptr, target, l, h, cls = _self_loop_choice(kind)
        r = orc.iterate(2, 2, row_ptr, target, l, h, cls, kind, 1e-8, 1, optimistic=opt,
                        horizon=T)
        assert r["status"] == 0 and r["sweeps"] == (T, T), (kind, opt)
        assert r["policy"][0] == pi, (kind, opt)
        assert r["lo"][0] == pytest.approx(lo, abs=1e-15), (kind, opt)
        assert r["hi"][0] == pytest.approx(hi, abs=1e-15), (kind, opt)


def _random_interval_imdp(rng, n_safe, n_u):
    # dense rows over n_safe SAFE states + TARGET + AVOID; each interval holds
    # a probability vector, so every row is feasible
    n = n_safe + 2
    row_ptr, target, lo, hi = [0], [], [], []
    for s in range(n):
        for u in range(n_u):
            if s < n_safe:
                p = rng.dirichlet(np.ones(n))
                lo += list(np.maximum(0.0, p - rng.uniform(0, .15, n)))
                hi += list(np.minimum(1.0, p + rng.uniform(0, .15, n)))
                target += list(range(n))
            row_ptr.append(len(target))
    cls = np.array([0] * n_safe + [1, 2], np.int8)
    return n, row_ptr, np.array(target), np.array(lo), np.array(hi), cls


def _highs_lp(lo, hi, val, maximise):
    res = linprog(-val if maximise else val, A_eq=np.ones((1, len(val))), b_eq=[1.0],
                  bounds=list(zip(lo, hi)), method="highs")
    return -res.fun if maximise else res.fun


@pytest.mark.parametrize("kind,opt,seed", [("reach_avoid", False, 1), ("reach_avoid", True, 2),
                                           ("safety", False, 3), ("safety", True, 4)])
def test_finite_horizon_equals_backward_induction(orc, kind, opt, seed):
    # T-step game by backward induction with HiGHS LPs: the first pass's
    # bound is the T-step optimum over inputs (a decision per step), the
    # policy is an optimal first decision, the second pass holds it for T steps
    rng = np.random.default_rng(seed)
    n_safe, n_u, T = 4, 3, 6
    n, row_ptr, tgt, lo, hi, cls = _random_interval_imdp(rng, n_safe, n_u)
    if kind == "safety":
        cls = cls.copy()
        cls[n_safe] = 2  # no TARGET under safety: both extra states are unsafe
    safety = kind == "safety"
    r = orc.iterate(n, n_u, row_ptr, tgt, lo, hi, cls, kind, 1e-8, 1, optimistic=opt,
                    horizon=T, want_q0=True)
    safe = np.where(cls == 0)[0]

    def value(V, t):
        if cls[t] == 0:
            return V[t]
        if cls[t] == 1:
            return 1.0
        return 1.0 if safety else 0.0

    adverse_max = safety            # the adversary's LP direction
    first_max = adverse_max if not opt else not adverse_max
    better = min if safety else max  # over inputs
    W = np.zeros(n)
    last_q = None
    for _ in range(T):
        Wn = W.copy()
        last_q = {}
        for s in safe:
            qs = []
            for u in range(n_u):
                a, b = row_ptr[s * n_u + u], row_ptr[s * n_u + u + 1]
                val = np.array([value(W, t) for t in tgt[a:b]])
                qs.append(_highs_lp(lo[a:b], hi[a:b], val, first_max))
            Wn[s] = better(qs)
            last_q[s] = qs
        W = Wn
    pol = r["policy"]
    H = np.zeros(n)
    for _ in range(T):
        Hn = H.copy()
        for s in safe:
            a, b = row_ptr[s * n_u + pol[s]], row_ptr[s * n_u + pol[s] + 1]
            val = np.array([value(H, t) for t in tgt[a:b]])
            Hn[s] = _highs_lp(lo[a:b], hi[a:b], val, not first_max)
        H = Hn
    for s in safe:
        assert last_q[s][pol[s]] == pytest.approx(better(last_q[s]), abs=1e-9)
    first = 1 - W[safe] if safety else W[safe]
    second = 1 - H[safe] if safety else H[safe]
    lo_ref, hi_ref = (second, first) if opt else (first, second)
    assert np.abs(r["lo"][safe] - lo_ref).max() < 1e-9
    assert np.abs(r["hi"][safe] - hi_ref).max() < 1e-9
    assert r["sweeps"] == (T, T) and r["status"] == 0


def test_finite_horizon_rises_to_the_infinite_horizon_bound(orc):
    # reach within T steps grows with T and stays below the infinite-horizon
    # lower bound's limit (V0 of interval iteration approaches it from below)
    system = W.tiny_affine(d=2, n=7, seed=12, n_inputs=4)
    m = orc.build(system, system["k_sigma"])
    cls = orc.label(system, [[[0.5, 0.5], [2.0, 2.0]]], [[[-2.0, -2.0], [-1.0, -1.0]]])
    args = (m["n_states"], 4, m["row_ptr"], m["target"], m["lo"], m["hi"], cls, "reach_avoid")
    inf = orc.iterate(*args, 1e-12, 100000)
    prev = np.zeros(m["n_states"])
    for T in (1, 2, 4, 8, 16, 64, 256):
        r = orc.iterate(*args, 1e-8, 1, horizon=T)
        assert (r["lo"] >= prev - 1e-15).all()
        assert (r["lo"] <= inf["lo"] + 1e-12).all()
        prev = r["lo"]
    assert np.abs(prev - inf["lo"]).max() < 1e-6


def test_finite_horizon_without_safe_states_runs_no_sweep(orc):
    row_ptr, target, lo, hi, cls = _self_loop_choice("reach")
    cls = np.array([1, 1], np.int8)
    r = orc.iterate(2, 2, row_ptr, target, lo, hi, cls, "reach", 1e-8, 1, horizon=5)
    assert r["sweeps"] == (0, 0) and r["status"] == 0
    assert (r["lo"] == 1).all() and (r["hi"] == 1).all()


# --------------------------------------------------------------------------
# Remark 5.2: horizon from the self-convergence of each iterate
# --------------------------------------------------------------------------

def _first_k(move, eps=1e-8):
    # first sweep k >= 1 whose move (a closed form in k) is at most eps
    return next(k for k in range(1, 100000) if move(k) <= eps)


def test_self_stop_worked_reach_avoid(orc):
    # the single-state chain of the worked reach-avoid example: pass 1
    # V' = .1 + .4 V moves V0 by .1 * .4^(k-1) and V1 (from 1) by .5 * .4^(k-1);
    # pass 2 V' = .3 + .5 V moves V0 by .3 * .5^(k-1), V1 by .2 * .5^(k-1)
    row_ptr, cls = [0, 3, 3, 3], np.array([0, 1, 2], np.int8)
    args = (3, 1, row_ptr, [0, 1, 2], [.3, .1, .2], [.6, .3, .5], cls, "reach_avoid", 1e-8, 1000)
    k1 = _first_k(lambda k: .5 * .4 ** (k - 1))
    k2 = _first_k(lambda k: .3 * .5 ** (k - 1))
    r = orc.iterate(*args, self_stop=True)
    assert r["sweeps"] == (k1, k2) and r["converged"] == (1, 1)
    assert r["gap"][0] == pytest.approx(.5 * .4 ** (k1 - 1), rel=1e-9)
    a = orc.iterate_auto_horizon(*args)
    K = max(k1, k2)
    assert a["horizon"] == K and a["sweeps"] == (K, K) and a["self_sweeps"] == (k1, k2)
    assert a["status"] == 0
    assert a["lo"][0] == pytest.approx((1 - .4 ** K) / 6, abs=1e-15)
    assert a["hi"][0] == pytest.approx(.6 * (1 - .5 ** K), abs=1e-15)


def test_auto_horizon_where_the_bounds_never_meet(orc):
    # the non-converging safety chain: self in [.9, 1], OUT in [0, .1].  Pass 1
    # (bad mass maximised): V' = .1 + .9 V moves V0 by .1 * .9^(k-1) while V1
    # stays at 1; pass 2 (minimised): nothing moves, so one sweep.  The horizon
    # is pass 1's count K, and the K-step bounds are .9^K (the adversary leaves
    # with .1 each step) and 1 (it never leaves).
    args = (1, 1, [0, 2], [0, -1], [.9, 0.0], [1.0, .1], np.array([0], np.int8), "safety",
            1e-8, 500)
    K = _first_k(lambda k: .1 * .9 ** (k - 1))
    a = orc.iterate_auto_horizon(*args)
    assert a["self_sweeps"] == (K, 1) and a["horizon"] == K and a["status"] == 0
    assert a["lo"][0] == pytest.approx(.9 ** K, rel=1e-12)
    assert a["hi"][0] == 1.0
    # the plain interval iteration hits its cap on the same chain
    assert orc.iterate(*args)["status"] == 1


def test_self_stop_cap_and_empty_safe_set(orc):
    args = (1, 1, [0, 2], [0, -1], [.9, 0.0], [1.0, .1], np.array([0], np.int8), "safety", 1e-8)
    r = orc.iterate(*args, 50, self_stop=True)
    assert r["sweeps"] == (50, 1) and r["converged"] == (0, 1) and r["status"] == 1
    r = orc.iterate(1, 1, [0, 2], [0, -1], [.9, 0.0], [1.0, .1], np.array([2], np.int8), "safety",
                    1e-8, 50, self_stop=True)
    assert r["sweeps"] == (0, 0) and r["status"] == 0


# --------------------------------------------------------------------------
# Disturbance player (eq. (5.1): max over u of min over w-hat)
# --------------------------------------------------------------------------

def _two_by_two():
    # state 0 SAFE, 1 TARGET, 2 AVOID; rows (u, w) of state 0 are exact
    # (lo = hi): (0,0) target .5; (0,1) .1; (1,0) .3; (1,1) .3, the rest to AVOID
    row_ptr = [0, 2, 4, 6, 8] + [8] * 8
    target = [1, 2] * 4
    p = [.5, .5, .1, .9, .3, .7, .3, .7]
    return row_ptr, target, p, p, np.array([0, 1, 2], np.int8)


def test_disturbance_worked_example(orc):
    # the disturbance answers each input with its worst row: input 0 is worth
    # .1, input 1 .3, so pi = 1 and both bounds are .3; with the disturbances
    # read as four more inputs the controller would claim .5
    row_ptr, target, lo, hi, cls = _two_by_two()
    for opt in (False, True):
        r = orc.iterate(3, 2, row_ptr, target, lo, hi, cls, "reach_avoid", 1e-9, 100,
                        optimistic=opt, n_dist=2, want_q0=True)
        assert r["policy"][0] == 1 and r["status"] == 0
        assert r["lo"][0] == pytest.approx(.3, abs=1e-15) and r["hi"][0] == pytest.approx(.3, abs=1e-15)
        assert r["q0"][0] == pytest.approx([.1, .3], abs=1e-15)
    r = orc.iterate(3, 4, row_ptr, target, lo, hi, cls, "reach_avoid", 1e-9, 100)
    assert r["policy"][0] == 0 and r["lo"][0] == pytest.approx(.5, abs=1e-15)


def test_disturbance_safety_finite_horizon(orc):
    # state 0 SAFE with a self loop, state 1 AVOID.  Bad mass per step:
    # (u0,w0) .1, (u0,w1) .4, (u1,w0) .2, (u1,w1) .25.  The disturbance takes
    # the larger bad mass (.4 and .25), the controller the smaller: pi = 1 and
    # staying safe for T steps has probability .75^T
    row_ptr = [0, 2, 4, 6, 8] + [8] * 4
    target = [0, 1] * 4
    p = [.9, .1, .6, .4, .8, .2, .75, .25]
    for T in (1, 4, 9):
        r = orc.iterate(2, 2, row_ptr, target, p, p, np.array([0, 2], np.int8), "safety", 1e-9, 1,
                        horizon=T, n_dist=2)
        assert r["policy"][0] == 1
        assert r["lo"][0] == pytest.approx(.75 ** T, rel=1e-14)
        assert r["hi"][0] == pytest.approx(.75 ** T, rel=1e-14)


def _disturbed_system(seed, n_dist=3):
    sys_ = W.tiny_affine(d=2, n=7, seed=seed, n_inputs=3)
    rng = np.random.default_rng(seed + 100)
    sys_ = dict(sys_, D=rng.normal(0, 0.3, (2, 2)),
                disturbances=rng.uniform(-0.5, 0.5, (n_dist, 2)))
    return sys_


def test_disturbed_mean_box_contains_and_is_tight(orc):
    # the build row (u, w) has the mean box of A x + B u + D w + c over the cell
    system = _disturbed_system(3)
    A, B, c = (np.asarray(system[k]) for k in ("A", "B", "c"))
    Dm, Wd, U = np.asarray(system["D"]), np.asarray(system["disturbances"]), np.asarray(system["inputs"])
    rng = np.random.default_rng(4)
    for _ in range(20):
        s = int(rng.integers(0, 49))
        u, w = int(rng.integers(0, len(U))), int(rng.integers(0, len(Wd)))
        mlo, mhi = orc.mean_box(system, s, u * len(Wd) + w)
        k = np.unravel_index(s, system["n"])
        lo = np.array([orc.cell_edge(system, i, k[i]) for i in range(2)])
        hi = np.array([orc.cell_edge(system, i, k[i] + 1) for i in range(2)])
        corners = np.array(list(itertools.product(*zip(lo, hi))))
        f = corners @ A.T + B @ U[u] + Dm @ Wd[w] + c
        assert (f >= mlo - 1e-15).all() and (f <= mhi + 1e-15).all()
        assert np.abs(f.min(0) - mlo).max() < 1e-12 and np.abs(f.max(0) - mhi).max() < 1e-12


def test_single_disturbance_is_a_shift_of_c(orc):
    # one disturbance w0: rows are those of the system with c + D w0
    system = _disturbed_system(5, n_dist=1)
    shifted = {k: v for k, v in system.items() if k not in ("D", "disturbances")}
    shifted["c"] = np.asarray(system["c"]) + np.asarray(system["D"]) @ np.asarray(system["disturbances"][0])
    a, b = orc.build(system, system["k_sigma"]), orc.build(shifted, shifted["k_sigma"])
    assert np.array_equal(a["row_ptr"], b["row_ptr"]) and np.array_equal(a["target"], b["target"])
    assert np.abs(a["lo"] - b["lo"]).max() < 1e-12 and np.abs(a["hi"] - b["hi"]).max() < 1e-12


@pytest.mark.parametrize("seed", [12, 21])
def test_disturbance_player_lowers_the_guarantee(orc, seed):
    # a stronger adversary cannot raise the pessimistic lower bound: with all
    # disturbances the bound is at most that of every single-disturbance system
    system = _disturbed_system(seed)
    tgt, avd = [[[0.5, 0.5], [2.0, 2.0]]], [[[-2.0, -2.0], [-1.0, -1.0]]]
    full = orc.solve(system, system["k_sigma"], "reach_avoid", tgt, avd, 1e-10, 100000)
    assert full["status"] == 0
    for k in range(len(system["disturbances"])):
        one = dict(system, disturbances=np.asarray(system["disturbances"])[k:k + 1])
        r = orc.solve(one, one["k_sigma"], "reach_avoid", tgt, avd, 1e-10, 100000)
        assert (full["lo"] <= r["lo"] + 1e-9).all()
    assert (full["lo"] <= full["hi"] + 1e-9).all()
