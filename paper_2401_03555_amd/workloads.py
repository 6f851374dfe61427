"""Seeded synthetic workloads shaped like the paper's case studies.

This module only *describes* inputs: systems, grids, input sets, noise levels
and specifications as plain dicts of numbers.  It holds none of the method's
arithmetic, so both the GPU library and the CPU oracle can be fed from it.

System dict keys: ``kind`` ("affine" | "unicycle"), ``A``, ``B``, ``c`` (affine),
``dt`` (unicycle), ``lb``, ``ub``, ``n`` (cells per dimension; cells tile
[lb, ub]), ``inputs`` (count x dim_u array, first component slowest),
``sigma`` (diagonal noise standard deviations), ``k_sigma`` (window half-width in
standard deviations; 0 means dense rows).
Spec dict keys: ``kind`` ("safety" | "reach" | "reach_avoid"), ``target``,
``avoid`` (lists of [lo, hi] boxes), ``eps``, ``max_sweeps``, optionally
``pessimistic`` (default true; false: optimistic policy) and ``horizon``
(default 0: infinite horizon; T > 0: T sweeps of value iteration per pass;
"auto": the horizon at which each pass's iterates converge to themselves).
"""
import itertools
import math

import numpy as np

SEED = 240103555


def _grid_inputs(*axes):
    return np.array(list(itertools.product(*axes)), dtype=np.float64)


def robot2d(sigma=0.25):
    """2D robot, reach-avoid, dense rows (stand-in for the paper's 2D robot study).

    x+ = x + 0.5 u + w on [-10,10]^2, 20x20 cells of width 1, u in {-1,0,1}^2,
    sigma = 0.25; target [5,8]^2, avoid [-2,2]^2, eps 1e-8.
    """
    system = dict(kind="affine", A=np.eye(2), B=0.5 * np.eye(2), c=np.zeros(2),
                  lb=[-10.0, -10.0], ub=[10.0, 10.0], n=[20, 20],
                  inputs=_grid_inputs([-1.0, 0.0, 1.0], [-1.0, 0.0, 1.0]),
                  sigma=[sigma, sigma], k_sigma=0.0)
    spec = dict(kind="reach_avoid", target=[[[5.0, 5.0], [8.0, 8.0]]],
                avoid=[[[-2.0, -2.0], [2.0, 2.0]]], eps=1e-8, max_sweeps=100000)
    return system, spec


def robot2d_disturbed(n_dist=11):
    """The 2D robot with a disturbance player (stand-in for the paper's 2D robot
    rows with |W| = 11): x+ = x + 0.5 u + D w + noise, D = (1, 0)^T, w in 11
    evenly spaced values of [-0.5, 0.5] (an uncertain drift along x); grid,
    inputs, noise and specification as robot2d."""
    system, spec = robot2d()
    system = dict(system, D=np.array([[1.0], [0.0]]),
                  disturbances=np.linspace(-0.5, 0.5, n_dist).reshape(-1, 1))
    return system, spec


def unicycle3d(n=(50, 50, 24)):
    """3D unicycle vehicle, reach-avoid, +-6 sigma windows (stand-in for the 3D vehicle study).

    x0+ = x0 + 0.1 v cos th, x1+ = x1 + 0.1 v sin th, th+ = th + 0.1 om on
    [-5,5]^2 x [-pi,pi] (no wrap), v in {0.5,1,1.5,2}, om in {-1,-.5,0,.5,1}
    (v-major), sigma = (0.05, 0.05, 0.02); target [3,4.5]^2 x all th,
    avoid [-1,1] x [-3,1] x all th, eps 1e-8.
    """
    pi = math.pi
    system = dict(kind="unicycle", dt=0.1, lb=[-5.0, -5.0, -pi], ub=[5.0, 5.0, pi], n=list(n),
                  inputs=_grid_inputs([0.5, 1.0, 1.5, 2.0], [-1.0, -0.5, 0.0, 0.5, 1.0]),
                  sigma=[0.05, 0.05, 0.02], k_sigma=6.0)
    spec = dict(kind="reach_avoid", target=[[[3.0, 3.0, -pi], [4.5, 4.5, pi]]],
                avoid=[[[-1.0, -3.0, -pi], [1.0, 1.0, pi]]], eps=1e-8, max_sweeps=100000)
    return system, spec


def room5d(cells=10):
    """5D ring of rooms, stay-in-domain safety, +-6 sigma windows (stand-in for the 5D room study).

    x_i+ = 0.85 x_i + 0.05 (x_{i-1} + x_{i+1}) + 0.75 + 0.25 u + w_i, indices
    mod 5, u in {0,1,2,3}; [19,21]^5 with ``cells`` per dimension (10 -> width
    0.2, 100,000 states); sigma 0.05; avoid = leaving the domain only.
    """
    d = 5
    A = np.zeros((d, d))
    for i in range(d):
        A[i, i] = 0.85
        A[i, (i - 1) % d] = 0.05
        A[i, (i + 1) % d] = 0.05
    system = dict(kind="affine", A=A, B=np.full((d, 1), 0.25), c=np.full(d, 0.75),
                  lb=[19.0] * d, ub=[21.0] * d, n=[cells] * d,
                  inputs=np.array([[0.0], [1.0], [2.0], [3.0]]),
                  sigma=[0.05] * d, k_sigma=6.0)
    spec = dict(kind="safety", target=[], avoid=[], eps=1e-8, max_sweeps=50)
    return system, spec


def random_linear(rng, d=None):
    """One instance of the batched generator: 2D or 3D x+ = A x + B u + w.

    A = rho M / specrad(M), M ~ N(0,1), rho ~ U(0.6, 0.95); B ~ N(0, 0.3^2);
    10-60 cells per dimension on [-10,10]^d; inputs on a uniform grid in
    [-1,1]^d with 2-5 points per axis and 4-25 points in total; sigma_i =
    U(0.1, 0.5) cell widths; disjoint grid-aligned target and avoid boxes.
    """
    if d is None:
        d = int(rng.integers(2, 4))
    M = rng.normal(size=(d, d))
    rho = rng.uniform(0.6, 0.95)
    A = rho * M / max(abs(np.linalg.eigvals(M)))
    B = rng.normal(scale=0.3, size=(d, d))
    n = [int(x) for x in rng.integers(10, 61, size=d)]
    while True:
        k = [int(x) for x in rng.integers(2, 6, size=d)]
        if 4 <= int(np.prod(k)) <= 25:
            break
    inputs = _grid_inputs(*[np.linspace(-1.0, 1.0, kk) for kk in k])
    lb, ub = [-10.0] * d, [10.0] * d
    w = [20.0 / ni for ni in n]
    sigma = [rng.uniform(0.1, 0.5) * wi for wi in w]
    boxes = []
    for _ in range(2):
        while True:
            span = [int(rng.integers(1, max(2, ni // 4) + 1)) for ni in n]
            start = [int(rng.integers(0, ni - sp + 1)) for ni, sp in zip(n, span)]
            box = [[lb[i] + start[i] * w[i] for i in range(d)],
                   [lb[i] + (start[i] + span[i]) * w[i] for i in range(d)]]
            cells = [(start[i], start[i] + span[i]) for i in range(d)]
            if not boxes or any(c[1] <= o[0] or o[1] <= c[0]
                                for c, o in zip(cells, boxes[0][1])):
                boxes.append((box, cells))
                break
    system = dict(kind="affine", A=A, B=B, c=np.zeros(d), lb=lb, ub=ub, n=n, inputs=inputs,
                  sigma=sigma, k_sigma=6.0)
    spec = dict(kind="reach_avoid", target=[boxes[0][0]], avoid=[boxes[1][0]], eps=1e-8,
                max_sweeps=100000)
    return system, spec


def mc_points(n, d, seed=SEED + 7, kind="random"):
    """Points of [0, 1)^d for the Monte Carlo cell integrals of correlated noise.

    "random": n seeded uniform points.  "lattice": the midpoints of a tensor
    grid with m = round(n^(1/d)) points per dimension (m^d points, first
    coordinate slowest), a deterministic product midpoint rule.
    """
    if kind == "lattice":
        m = max(1, int(round(n ** (1.0 / d))))
        ax = (np.arange(m, dtype=np.float64) + 0.5) / m
        return np.array(list(itertools.product(*([ax] * d))), dtype=np.float64).reshape(-1, d)
    rng = np.random.default_rng(seed)
    return rng.random((n, d))


def robot2d_correlated(n=(40, 40), samples=256, grid_pts=2, kappa=3.0, corr=0.5, seed=SEED + 7):
    """The paper's 2D robot with correlated noise (stand-in for a full-covariance
    run, Section 4.1): x+ = x + 0.5 u + w on [-10,10]^2, 40x40 cells of width 0.5,
    u in {-1,0,1}^2, Cov = 0.75 [[1, corr], [corr, 1]] (the study's variance,
    with correlation ``corr``), +-6 marginal sigma windows; target [5,7]^2,
    avoid [-2,2]^2, eps 1e-8.  Returns (system, spec, mc) with mc the inverse
    covariance, its determinant and ``samples`` seeded uniform points,
    ``grid_pts`` candidate means per dimension and ``kappa`` standard errors.
    """
    cov = 0.75 * np.array([[1.0, corr], [corr, 1.0]])
    system = dict(kind="affine", A=np.eye(2), B=0.5 * np.eye(2), c=np.zeros(2),
                  lb=[-10.0, -10.0], ub=[10.0, 10.0], n=list(n),
                  inputs=_grid_inputs([-1.0, 0.0, 1.0], [-1.0, 0.0, 1.0]),
                  sigma=[math.sqrt(0.75)] * 2, k_sigma=6.0)
    spec = dict(kind="reach_avoid", target=[[[5.0, 5.0], [7.0, 7.0]]],
                avoid=[[[-2.0, -2.0], [2.0, 2.0]]], eps=1e-8, max_sweeps=100000)
    mc = dict(inv_cov=np.linalg.inv(cov), det_cov=float(np.linalg.det(cov)),
              samples=mc_points(samples, 2, seed=seed), grid_pts=grid_pts, kappa=kappa)
    return system, spec, mc


def batched(count=384, seed=SEED):
    rng = np.random.default_rng(seed)
    return [random_linear(rng) for _ in range(count)]


def tiny_affine(d=2, n=6, seed=1, k_sigma=6.0, n_inputs=3):
    """A small random affine system for property and parity tests."""
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(d, d))
    A = 0.8 * M / max(abs(np.linalg.eigvals(M)))
    B = rng.normal(scale=0.5, size=(d, 1))
    system = dict(kind="affine", A=A, B=B, c=rng.normal(scale=0.2, size=d),
                  lb=[-2.0] * d, ub=[2.0] * d, n=[n] * d,
                  inputs=np.linspace(-1.0, 1.0, n_inputs).reshape(-1, 1),
                  sigma=[0.3 * 4.0 / n] * d, k_sigma=k_sigma)
    return system


def served_pool(seed=SEED + 1):
    """The 64 systems a served trace draws from, keyed "<generator>/<k>".

    Every case-study generator contributes its own configuration and seeded
    variants of it (noise level, grid resolution), and the batched generator
    the rest: robot2d with sigma U(0.15, 0.5) (4), unicycle3d at 50x50x24 and
    three coarser grids (4), room5d at 5-8 cells per dimension (4) and 52
    random linear 2D/3D systems.
    """
    rng = np.random.default_rng(seed)
    pool = {"robot2d/0": robot2d()[0]}
    for k in range(1, 4):
        pool[f"robot2d/{k}"] = robot2d(sigma=float(rng.uniform(0.15, 0.5)))[0]
    pool["unicycle3d/0"] = unicycle3d()[0]
    for k in range(1, 4):
        n = (int(rng.integers(16, 41)), int(rng.integers(16, 41)), int(rng.integers(8, 17)))
        pool[f"unicycle3d/{k}"] = unicycle3d(n=n)[0]
    for k, cells in enumerate((5, 6, 7, 8)):
        pool[f"room5d/{k}"] = room5d(cells=cells)[0]
    for k in range(52):
        pool[f"linear/{k}"] = random_linear(rng)[0]
    return pool


def _aligned_box(rng, system):
    lb, ub, n = (np.asarray(system[k], dtype=np.float64) for k in ("lb", "ub", "n"))
    w = (ub - lb) / n
    span = [int(rng.integers(1, max(2, int(ni) // 4) + 1)) for ni in n]
    start = [int(rng.integers(0, int(ni) - sp + 1)) for ni, sp in zip(n, span)]
    return [[float(lb[i] + start[i] * w[i]) for i in range(len(n))],
            [float(lb[i] + (start[i] + span[i]) * w[i]) for i in range(len(n))]]


def served_trace(pool, rate=200.0, duration=2.0, seed=SEED + 2, max_sweeps=2000,
                 horizon="auto"):
    """Poisson arrivals at ``rate`` per second over ``duration`` seconds.

    Each request names a pool system (uniformly), a specification kind in
    {safety, reach, reach_avoid} (uniformly), grid-aligned random boxes (up to
    a quarter of the cells per dimension) and eps in {1e-6, 1e-8}; ``horizon``
    is the specification's horizon field ("auto" by default: the horizon at
    which each pass's iterates converge to themselves, the paper's remedy for
    queries whose two bounds need not meet; 0 for the plain infinite horizon).
    """
    rng = np.random.default_rng(seed)
    keys = sorted(pool)
    t, trace = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            return trace
        key = keys[int(rng.integers(len(keys)))]
        kind = ("safety", "reach", "reach_avoid")[int(rng.integers(3))]
        target = [_aligned_box(rng, pool[key])] if kind != "safety" else []
        avoid = [_aligned_box(rng, pool[key])] if kind != "reach" else []
        eps = (1e-6, 1e-8)[int(rng.integers(2))]
        trace.append(dict(t=t, key=key, spec=dict(kind=kind, target=target, avoid=avoid,
                                                   eps=eps, max_sweeps=max_sweeps,
                                                   horizon=horizon)))


CONFIGS = {
    "robot2d": robot2d,
    "unicycle3d": unicycle3d,
    "room5d": room5d,
}
