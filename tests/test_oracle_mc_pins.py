"""Pins of the oracle's correlated-noise (Monte Carlo) abstraction, Section 4.1.

Nothing here re-types the oracle's arithmetic.  The pins are:
  - marginal standard deviations against numpy's matrix inverse;
  - the lattice covering radius against its closed form (diagonal) and a
    dense brute-force search (correlated);
  - the total-variation distance of two shifted Gaussians against numerical
    integration, and the mass-shift bound against exact cell masses from
    scipy's multivariate normal CDF over the whole half-spacing box;
  - the Monte Carlo estimate against the closed-form 1D mass (midpoint
    lattice), scipy's bivariate normal CDF (correlated, midpoint lattice),
    and scipy's density and standard error of the mean (random points);
  - the built rows against the closed-form abstraction of the same system
    with a diagonal covariance (same windows, bracketing bounds), and against
    exact masses at random means of the source cell (correlated, soundness).
"""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate, stats
from scipy.special import ndtr

import oracle
from paper_2401_03555_amd import workloads as W


def _spd(rng, d):
    M = rng.normal(size=(d, d))
    return M @ M.T + d * 0.1 * np.eye(d)


def _rect_mass(mean, cov, a, b):
    """Exact N(mean, cov) mass of the box [a, b] (scipy's multivariate CDF)."""
    return float(stats.multivariate_normal(mean=mean, cov=cov).cdf(b, lower_limit=a))


# --------------------------------------------------------------------------
# Marginals, covering radius, shift bound
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,seed", [(1, 0), (2, 1), (3, 2), (5, 3), (8, 4)])
def test_marginal_sigma_matches_numpy_inverse(d, seed):
    cov = _spd(np.random.default_rng(seed), d)
    P = np.linalg.inv(cov)
    P = 0.5 * (P + P.T)
    s = oracle.marginal_sigma(P)
    np.testing.assert_allclose(s, np.sqrt(np.diag(np.linalg.inv(P))), rtol=1e-12)


def test_marginal_sigma_rejects_singular():
    with pytest.raises(ValueError):
        oracle.marginal_sigma(np.array([[1.0, 1.0], [1.0, 1.0]]))


def test_cover_radius_diagonal_closed_form():
    P = np.diag([4.0, 0.25, 9.0])
    mlo, mhi = np.array([0.0, -1.0, 2.0]), np.array([0.6, 1.0, 2.3])
    for G in (1, 2, 5):
        half = 0.5 * (mhi - mlo) / G
        want = math.sqrt(float(np.sum(np.diag(P) * half ** 2)))
        assert abs(oracle.mc_cover_radius(P, mlo, mhi, G) - want) <= 1e-14 * want


def test_cover_radius_correlated_brute_force():
    rng = np.random.default_rng(5)
    for d in (2, 3):
        P = np.linalg.inv(_spd(rng, d))
        P = 0.5 * (P + P.T)
        mlo = rng.normal(size=d)
        mhi = mlo + rng.uniform(0.1, 1.0, size=d)
        G = 3
        half = 0.5 * (mhi - mlo) / G
        # every point of the half-spacing box, on a dense grid (corners included)
        ax = [np.linspace(-h, h, 41) for h in half]
        E = np.array(list(itertools.product(*ax)))
        brute = math.sqrt(float(np.max(np.einsum("ki,ij,kj->k", E, P, E))))
        r = oracle.mc_cover_radius(P, mlo, mhi, G)
        assert abs(r - brute) <= 1e-12 * brute


def test_total_variation_of_shifted_gaussians():
    """The TV leg of the shift bound is 2 Phi(rho/2) - 1: integrate
    |phi(x) - phi(x - rho)| / 2 numerically and compare (1D standard normal,
    a far-away box so that the derivative leg does not bind)."""
    for rho in (0.05, 0.4, 1.3, 3.0):
        tv, _ = integrate.quad(lambda x: 0.5 * abs(stats.norm.pdf(x) - stats.norm.pdf(x - rho)),
                               -30, 30, points=[rho / 2], limit=200)
        # huge volume: the derivative leg exceeds the TV leg, which is returned
        got = oracle.mc_shift_bound([1.0], 1.0, rho, 1e6, [-1.0], [1.0])
        assert abs(got - tv) <= 1e-10


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_shift_bound_covers_exact_mass_changes(seed):
    """For a cell and a candidate mean, the exact mass at every mean of the
    candidate's half-spacing box differs from the mass at the candidate by at
    most the bound (scipy CDF on a dense grid of means)."""
    rng = np.random.default_rng(seed)
    cov = np.array([[0.5, 0.3], [0.3, 0.8]]) * rng.uniform(0.5, 2.0)
    P = np.linalg.inv(cov)
    P = 0.5 * (P + P.T)
    sigma = np.sqrt(np.diag(cov))
    c = rng.normal(size=2)
    half = rng.uniform(0.05, 0.4, size=2)
    rho = oracle.mc_cover_radius(P, c - half, c + half, 1)
    for off in ([0.0, 0.0], [1.0, -0.5], [2.5, 1.5], [-0.3, 3.0]):
        a = c + np.array(off) - 0.25
        b = a + 0.5
        zlo, zhi = a - (c + half), b - (c - half)
        bound = oracle.mc_shift_bound(sigma, float(np.linalg.det(cov)), rho, 0.25, zlo, zhi)
        p0 = _rect_mass(c, cov, a, b)
        worst = max(abs(_rect_mass(c + np.array([u, v]), cov, a, b) - p0)
                    for u in np.linspace(-half[0], half[0], 9)
                    for v in np.linspace(-half[1], half[1], 9))
        assert worst <= bound + 1e-9, (off, worst, bound)


# --------------------------------------------------------------------------
# The Monte Carlo estimate
# --------------------------------------------------------------------------

@pytest.mark.parametrize("a,b,m,s", [(0.0, 1.0, 0.4, 0.5), (1.0, 1.5, 0.0, 0.8),
                                     (-2.0, -1.0, 0.3, 1.1)])
def test_estimate_1d_midpoint_rule_matches_closed_form(a, b, m, s):
    X = W.mc_points(4096, 1, kind="lattice")
    p, _ = oracle.mc_cell_estimate([[1.0 / s ** 2]], s ** 2, [a], [b], [m], X)
    exact = ndtr((b - m) / s) - ndtr((a - m) / s)
    # midpoint rule error <= (b - a)^3 max|f''| / (24 N^2)
    assert abs(p - exact) <= 1e-8


def test_estimate_correlated_2d_matches_bivariate_cdf():
    cov = np.array([[0.5, 0.3], [0.3, 0.8]])
    P = np.linalg.inv(cov)
    X = W.mc_points(250 ** 2, 2, kind="lattice")
    for a, b, m in (([0.0, 0.0], [0.5, 0.7], [0.2, 0.1]), ([-1.0, 0.5], [-0.5, 1.5], [0.0, 0.0]),
                    ([0.3, -0.8], [1.3, 0.2], [-0.2, 0.4])):
        p, _ = oracle.mc_cell_estimate(P, float(np.linalg.det(cov)), a, b, m, X)
        assert abs(p - _rect_mass(m, cov, a, b)) <= 2e-6


def test_estimate_and_standard_error_match_scipy_density():
    cov = np.array([[0.7, -0.2, 0.1], [-0.2, 0.4, 0.05], [0.1, 0.05, 0.9]])
    P = np.linalg.inv(cov)
    X = W.mc_points(500, 3, seed=11)
    a, b, m = np.array([0.0, -0.2, 0.1]), np.array([0.4, 0.3, 0.6]), np.array([0.1, 0.0, 0.2])
    y = a + (b - a) * X
    z = stats.multivariate_normal(mean=m, cov=cov).pdf(y)
    vol = float(np.prod(b - a))
    p, se = oracle.mc_cell_estimate(P, float(np.linalg.det(cov)), a, b, m, X)
    assert abs(p - vol * z.mean()) <= 1e-12 * p
    assert abs(se - vol * stats.sem(z)) <= 1e-10 * se


# --------------------------------------------------------------------------
# Built rows
# --------------------------------------------------------------------------

def test_build_diagonal_brackets_closed_form_abstraction():
    """Uncorrelated noise: windows and row shapes equal the closed-form
    build's; every Monte Carlo bound brackets the exact one (product midpoint
    rule, kappa = 0) and stays within the shift bound of it; the union OUT /
    TAIL bounds contain the product ones."""
    system, _, mc = W.robot2d_correlated(n=(12, 12), corr=0.0)
    mc = dict(mc, samples=W.mc_points(48 ** 2, 2, kind="lattice"), kappa=0.0, grid_pts=3)
    rows = np.arange(0, 144 * 9, 7)
    m = oracle.build_mc(system, mc, system["k_sigma"], rows=rows)
    c = oracle.build(system, system["k_sigma"], rows=rows)
    np.testing.assert_array_equal(m["win"], c["win"])
    np.testing.assert_array_equal(m["row_ptr"], c["row_ptr"])
    np.testing.assert_array_equal(m["target"], c["target"])
    cell = c["target"] >= 0
    sigma = np.sqrt(0.75)
    w = 20.0 / 12
    norm = 1.0 / (2 * math.pi * 0.75)
    # product midpoint rule: error <= vol sum_i h_i^2 max|f_ii| / 24, |f_ii| <= norm / sigma^2
    quad = w * w * 2 * (w / 48) ** 2 * norm / sigma ** 2 / 24
    assert np.all(m["lo"][cell] <= c["lo"][cell] + quad)
    assert np.all(m["hi"][cell] >= c["hi"][cell] - quad)
    # the largest shift bound of these rows: the derivative leg at its peak
    rho = math.sqrt(2 * (0.5 * w / 3) ** 2) / sigma
    lip = w * w * norm * rho * math.exp(-0.5)
    assert np.all(m["lo"][cell] >= c["lo"][cell] - lip - quad)
    assert np.all(m["hi"][cell] <= c["hi"][cell] + lip + quad)
    assert np.all(m["ot"][:, 0] <= c["ot"][:, 0] + 1e-15)
    assert np.all(m["ot"][:, 1] >= c["ot"][:, 1] - 1e-15)
    assert np.all(m["ot"][:, 3] >= c["ot"][:, 3] - 1e-15)


def test_build_correlated_is_sound_at_random_source_points():
    """Correlated noise, random points, kappa = 4: the exact mass of every
    window cell, of leaving the domain and of the in-domain tail, at random
    points of the source cell, lies within the row's bounds."""
    system, _, mc = W.robot2d_correlated(n=(10, 10), samples=2048, grid_pts=2, kappa=4.0)
    cov = np.linalg.inv(mc["inv_cov"])
    rng = np.random.default_rng(3)
    nu = len(system["inputs"])
    rows = rng.choice(100 * nu, size=6, replace=False)
    m = oracle.build_mc(system, mc, system["k_sigma"], rows=rows)
    lb, ub = np.array(system["lb"]), np.array(system["ub"])
    w = (ub - lb) / np.array(system["n"])
    for q, row in enumerate(rows):
        s, u = divmod(int(row), nu)
        k = np.array(divmod(s, system["n"][1]))
        b0, e0 = m["row_ptr"][q], m["row_ptr"][q + 1]
        for _ in range(3):
            x = lb + (k + rng.random(2)) * w
            mean = x + 0.5 * system["inputs"][u]
            inside = _rect_mass(mean, cov, lb, ub)
            out = 1.0 - inside
            assert m["ot"][q, 0] - 1e-9 <= out <= m["ot"][q, 1] + 1e-9
            win_mass = 0.0
            for e in range(b0, e0):
                t = m["target"][e]
                if t < 0:
                    continue
                kt = np.array(divmod(int(t), system["n"][1]))
                p = _rect_mass(mean, cov, lb + kt * w, lb + (kt + 1) * w)
                win_mass += p
                assert m["lo"][e] - 1e-9 <= p <= m["hi"][e] + 1e-9, (row, t, p, m["lo"][e], m["hi"][e])
            assert inside - win_mass <= m["ot"][q, 3] + 1e-7


def test_build_rejects_bad_noise():
    system, _, mc = W.robot2d_correlated(n=(4, 4), samples=16)
    for bad in (dict(det_cov=2 * mc["det_cov"]), dict(inv_cov=np.array([[1.0, 2.0], [2.0, 1.0]])),
                dict(samples=np.full((4, 2), 1.0)), dict(grid_pts=0), dict(kappa=-1.0)):
        with pytest.raises(ValueError):
            oracle.build_mc(system, dict(mc, **bad), system["k_sigma"])
