"""CPU oracle for the IMDP abstraction and interval iteration (arXiv 2401.03555).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  This wrapper loads ``liboracle.so``
(built from ``impact_oracle.c`` by ``build_oracle.py``) with ctypes and shares
nothing with the GPU library or its Python binding.

A system is passed as a plain mapping with keys
``kind`` ("affine" | "unicycle"), ``A``, ``B``, ``c`` (affine), ``dt``
(unicycle), ``lb``, ``ub``, ``n`` (grid), ``inputs`` (count x dim_u array) and
``sigma`` (per-dimension noise standard deviation).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

T_OUT = -1
T_TAIL = -2
SAFE, TARGET, AVOID = 0, 1, 2
SAFETY, REACH, REACH_AVOID = 0, 1, 2
SPEC_KINDS = {"safety": SAFETY, "reach": REACH, "reach_avoid": REACH_AVOID}


class _System(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim_x", C.c_int32), ("dim_u", C.c_int32),
                ("A", C.POINTER(C.c_double)), ("B", C.POINTER(C.c_double)),
                ("c", C.POINTER(C.c_double)), ("dt", C.c_double)]


class _Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("lb", C.POINTER(C.c_double)),
                ("ub", C.POINTER(C.c_double)), ("n", C.POINTER(C.c_int32))]


class _Inputs(C.Structure):
    _fields_ = [("count", C.c_int32), ("dim_u", C.c_int32),
                ("values", C.POINTER(C.c_double))]


class _Imdp(C.Structure):
    _fields_ = [("n_states", C.c_int64), ("n_rows", C.c_int64), ("n_entries", C.c_int64),
                ("n_inputs", C.c_int32), ("dim", C.c_int32), ("windowed", C.c_int32),
                ("win", C.POINTER(C.c_int32)), ("ot", C.POINTER(C.c_double)),
                ("row_ptr", C.POINTER(C.c_int64)), ("target", C.POINTER(C.c_int32)),
                ("lo", C.POINTER(C.c_double)), ("hi", C.POINTER(C.c_double))]


class _McNoise(C.Structure):
    _fields_ = [("inv_cov", C.POINTER(C.c_double)), ("det_cov", C.c_double),
                ("n_samples", C.c_int64), ("samples", C.POINTER(C.c_double)),
                ("grid_pts", C.c_int32), ("kappa", C.c_double)]


class _IterInfo(C.Structure):
    _fields_ = [("sweeps", C.c_int64 * 2), ("gap", C.c_double * 2),
                ("converged", C.c_int32 * 2), ("n_safe", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build_oracle
            build_oracle.build()
        L = C.CDLL(LIB_PATH)
        d, i32, i64, pd = C.c_double, C.c_int32, C.c_int64, C.POINTER(C.c_double)
        L.orc_cell_edge.restype = d
        L.orc_cell_edge.argtypes = [C.POINTER(_Grid), C.c_int, i64]
        L.orc_interval_cos.argtypes = [d, d, pd, pd]
        L.orc_interval_sin.argtypes = [d, d, pd, pd]
        L.orc_mean_box.restype = C.c_int
        L.orc_mean_box.argtypes = [C.POINTER(_System), C.POINTER(_Grid), C.POINTER(_Inputs),
                                   i64, i32, pd, pd]
        L.orc_gauss_cell_mass.restype = d
        L.orc_gauss_cell_mass.argtypes = [d, d, d, d]
        L.orc_factor_bounds.argtypes = [d, d, d, d, d, pd, pd]
        L.orc_exit_prob.restype = d
        L.orc_exit_prob.argtypes = [d, d, d, d]
        L.orc_build.restype = C.c_int
        L.orc_build.argtypes = [C.POINTER(_System), C.POINTER(_Grid), C.POINTER(_Inputs), pd, d,
                                C.POINTER(C.c_int64), i64, C.POINTER(_Imdp)]
        L.orc_imdp_free.argtypes = [C.POINTER(_Imdp)]
        L.orc_marginal_sigma.restype = C.c_int
        L.orc_marginal_sigma.argtypes = [C.c_int, pd, pd]
        L.orc_mc_cover_radius.restype = d
        L.orc_mc_cover_radius.argtypes = [C.c_int, pd, pd, pd, C.c_int]
        L.orc_mc_shift_bound.restype = d
        L.orc_mc_shift_bound.argtypes = [C.c_int, pd, d, d, d, pd, pd]
        L.orc_mc_cell_estimate.argtypes = [C.c_int, pd, d, pd, pd, pd, i64, pd, pd, pd]
        L.orc_build_mc.restype = C.c_int
        L.orc_build_mc.argtypes = [C.POINTER(_System), C.POINTER(_Grid), C.POINTER(_Inputs),
                                   C.POINTER(_McNoise), d, C.POINTER(C.c_int64), i64,
                                   C.POINTER(_Imdp)]
        L.orc_label.restype = C.c_int
        L.orc_label.argtypes = [C.POINTER(_Grid), i32, pd, i32, pd, C.POINTER(C.c_int8)]
        L.orc_lp_sorted.restype = d
        L.orc_lp_sorted.argtypes = [i64, pd, pd, pd, i32, pd]
        L.orc_iterate.restype = C.c_int
        L.orc_iterate.argtypes = [i64, i32, C.POINTER(C.c_int64), C.POINTER(C.c_int32), pd, pd,
                                  C.POINTER(C.c_int8), i32, d, i64, pd, pd,
                                  C.POINTER(C.c_int32), C.POINTER(_IterInfo), pd, i64, pd, pd, i32, i64, i32, i32]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def with_disturbances(system):
    """The system whose input list is every (u, w) pair, u-major, and whose
    input matrix is [B | D], so that its mean A x + [B | D] (u, w) + c is the
    disturbed mean A x + B u + D w + c of eq. (5.1)'s rows (x, u, w).  Returns
    (system, number of control inputs, number of disturbances)."""
    U = np.asarray(system["inputs"], dtype=np.float64)
    if U.ndim == 1:
        U = U.reshape(-1, 1) if U.size else np.zeros((1, 0))
    if "disturbances" not in system:
        return system, U.shape[0], 1
    if system["kind"] != "affine":
        raise ValueError("disturbances are supported for affine systems")
    Wd = np.asarray(system["disturbances"], dtype=np.float64)
    d = len(system["lb"])
    Dm = np.asarray(system["D"], dtype=np.float64).reshape(d, Wd.shape[1])
    B = np.asarray(system.get("B", np.zeros((d, U.shape[1]))), dtype=np.float64).reshape(d, U.shape[1])
    pairs = np.array([np.concatenate([u, w]) for u in U for w in Wd])
    out = {k: v for k, v in system.items() if k not in ("disturbances", "D")}
    out.update(inputs=pairs, B=np.hstack([B, Dm]))
    return out, U.shape[0], Wd.shape[0]


class _Marshal:
    """Holds the numpy buffers behind the ctypes structs for one call."""

    def __init__(self, system):
        system = with_disturbances(system)[0]
        kind = system["kind"]
        self.lb, self.ub = _f64(system["lb"]), _f64(system["ub"])
        self.n = np.ascontiguousarray(np.asarray(system["n"], dtype=np.int32))
        d = len(self.lb)
        inputs = np.asarray(system["inputs"], dtype=np.float64)
        if inputs.ndim == 1:
            inputs = inputs.reshape(-1, 1) if inputs.size else np.zeros((1, 0))
        self.inputs = np.ascontiguousarray(inputs)
        self.sigma = _f64(system["sigma"])
        du = self.inputs.shape[1]
        self.grid = _Grid(d, _dptr(self.lb), _dptr(self.ub),
                          self.n.ctypes.data_as(C.POINTER(C.c_int32)))
        self.inp = _Inputs(self.inputs.shape[0], du, _dptr(self.inputs))
        if kind == "affine":
            self.A = _f64(system["A"]).reshape(d, d)
            self.B = _f64(system.get("B", np.zeros((d, du)))).reshape(d, du) if du else np.zeros((d, 1))
            self.c = _f64(system.get("c", np.zeros(d)))
            self.sys = _System(0, d, du, _dptr(self.A), _dptr(self.B), _dptr(self.c), 0.0)
        elif kind == "unicycle":
            self.sys = _System(1, d, du, None, None, None, float(system["dt"]))
        else:
            raise ValueError(f"unknown system kind {kind!r}")


def n_states(system):
    return int(np.prod(np.asarray(system["n"], dtype=np.int64)))


def cell_edge(system, i, k):
    m = _Marshal(system)
    return lib().orc_cell_edge(C.byref(m.grid), i, k)


def interval_cos(lo, hi):
    a, b = C.c_double(), C.c_double()
    lib().orc_interval_cos(lo, hi, C.byref(a), C.byref(b))
    return a.value, b.value


def interval_sin(lo, hi):
    a, b = C.c_double(), C.c_double()
    lib().orc_interval_sin(lo, hi, C.byref(a), C.byref(b))
    return a.value, b.value


def mean_box(system, state, u):
    m = _Marshal(system)
    d = len(m.lb)
    lo, hi = np.zeros(d), np.zeros(d)
    rc = lib().orc_mean_box(C.byref(m.sys), C.byref(m.grid), C.byref(m.inp), state, u,
                            _dptr(lo), _dptr(hi))
    if rc != 0:
        raise ValueError("mean box: unsupported system")
    return lo, hi


def gauss_cell_mass(a, b, m, sigma):
    return lib().orc_gauss_cell_mass(a, b, m, sigma)


def factor_bounds(a, b, mlo, mhi, sigma):
    lo, hi = C.c_double(), C.c_double()
    lib().orc_factor_bounds(a, b, mlo, mhi, sigma, C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def exit_prob(lb, ub, m, sigma):
    return lib().orc_exit_prob(lb, ub, m, sigma)


def marginal_sigma(inv_cov):
    """sqrt of the diagonal of the covariance whose inverse is ``inv_cov``."""
    P = _f64(inv_cov)
    d = int(round(np.sqrt(P.size)))
    s = np.zeros(d)
    if lib().orc_marginal_sigma(d, _dptr(P), _dptr(s)) != 0:
        raise ValueError("inverse covariance is singular or not positive")
    return s


def mc_cover_radius(inv_cov, mlo, mhi, G):
    """Mahalanobis covering radius of a G-per-dimension lattice over [mlo, mhi]."""
    P, mlo, mhi = _f64(inv_cov), _f64(mlo), _f64(mhi)
    return lib().orc_mc_cover_radius(len(mlo), _dptr(P), _dptr(mlo), _dptr(mhi), int(G))


def mc_shift_bound(sigma, det_cov, rho, vol, zlo, zhi):
    """Bound on the change of a cell's mass under a mean shift of Mahalanobis
    length <= rho, with every y - m in the box [zlo, zhi]."""
    sigma, zlo, zhi = _f64(sigma), _f64(zlo), _f64(zhi)
    d = len(sigma)
    norm = 1.0 / np.sqrt((2.0 * np.pi) ** d * det_cov)
    return lib().orc_mc_shift_bound(d, _dptr(sigma), norm, float(rho), float(vol),
                                    _dptr(zlo), _dptr(zhi))


def mc_cell_estimate(inv_cov, det_cov, a, b, m, samples):
    """Plain Monte Carlo N(m, Cov) mass of the box [a, b] and its standard error."""
    P, a, b, m = _f64(inv_cov), _f64(a), _f64(b), _f64(m)
    X = _f64(samples)
    d = len(a)
    norm = 1.0 / np.sqrt((2.0 * np.pi) ** d * det_cov)
    p, se = C.c_double(), C.c_double()
    lib().orc_mc_cell_estimate(d, _dptr(P), norm, _dptr(a), _dptr(b), _dptr(m),
                               X.size // d, _dptr(X), C.byref(p), C.byref(se))
    return p.value, se.value


def _collect(out):
    d, R, E = out.dim, out.n_rows, out.n_entries
    return dict(
        n_states=out.n_states, n_inputs=out.n_inputs, dim=d, windowed=bool(out.windowed),
        win=np.ctypeslib.as_array(out.win, (R, 2 * d)).copy(),
        ot=np.ctypeslib.as_array(out.ot, (R, 4)).copy(),
        row_ptr=np.ctypeslib.as_array(out.row_ptr, (R + 1,)).copy(),
        target=np.ctypeslib.as_array(out.target, (max(E, 1),))[:E].copy(),
        lo=np.ctypeslib.as_array(out.lo, (max(E, 1),))[:E].copy(),
        hi=np.ctypeslib.as_array(out.hi, (max(E, 1),))[:E].copy(),
    )


def _rows_arg(rows):
    if rows is None:
        return None, 0, None
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    return rows.ctypes.data_as(C.POINTER(C.c_int64)), len(rows), rows


def build_mc(system, mc, k_sigma, rows=None):
    """Rows of the abstraction under correlated noise (Section 4.1 full
    covariance, Monte Carlo cell masses); same layout as ``build``.

    ``mc``: dict with ``inv_cov`` (d x d), ``det_cov``, ``samples`` (N x d in
    [0, 1)), ``grid_pts`` (G) and ``kappa``.  ``system["sigma"]`` is unused.
    """
    m = _Marshal(dict(system, sigma=np.ones(len(system["lb"]))))
    P, X = _f64(mc["inv_cov"]), _f64(mc["samples"])
    d = len(m.lb)
    nz = _McNoise(_dptr(P), float(mc["det_cov"]), X.size // d, _dptr(X),
                  int(mc["grid_pts"]), float(mc["kappa"]))
    out = _Imdp()
    rp, nr, keep = _rows_arg(rows)
    rc = lib().orc_build_mc(C.byref(m.sys), C.byref(m.grid), C.byref(m.inp), C.byref(nz),
                            float(k_sigma), rp, nr, C.byref(out))
    try:
        if rc != 0:
            raise ValueError(f"oracle Monte Carlo build failed ({rc})")
        return _collect(out)
    finally:
        lib().orc_imdp_free(C.byref(out))


def build(system, k_sigma, rows=None):
    """Rows of the abstraction as numpy arrays (Alg. 2 with closed-form bounds).

    Returns a dict: n_states, n_inputs, dim, windowed, win (rows x 2*dim),
    ot (rows x 4), row_ptr, target, lo, hi.
    """
    m = _Marshal(system)
    out = _Imdp()
    if rows is not None:
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        rp, nr = rows.ctypes.data_as(C.POINTER(C.c_int64)), len(rows)
    else:
        rp, nr = None, 0
    rc = lib().orc_build(C.byref(m.sys), C.byref(m.grid), C.byref(m.inp), _dptr(m.sigma),
                         float(k_sigma), rp, nr, C.byref(out))
    try:
        if rc != 0:
            raise ValueError(f"oracle build failed ({rc})")
        d, R, E = out.dim, out.n_rows, out.n_entries
        res = dict(
            n_states=out.n_states, n_inputs=out.n_inputs, dim=d, windowed=bool(out.windowed),
            win=np.ctypeslib.as_array(out.win, (R, 2 * d)).copy(),
            ot=np.ctypeslib.as_array(out.ot, (R, 4)).copy(),
            row_ptr=np.ctypeslib.as_array(out.row_ptr, (R + 1,)).copy(),
            target=np.ctypeslib.as_array(out.target, (max(E, 1),))[:E].copy(),
            lo=np.ctypeslib.as_array(out.lo, (max(E, 1),))[:E].copy(),
            hi=np.ctypeslib.as_array(out.hi, (max(E, 1),))[:E].copy(),
        )
    finally:
        lib().orc_imdp_free(C.byref(out))
    return res


def _boxes(boxes, d):
    b = np.asarray(boxes if boxes is not None else np.zeros((0, 2, d)), dtype=np.float64)
    b = np.ascontiguousarray(b.reshape(-1, 2, d))
    return b, b.shape[0]


def label(system, target_boxes=None, avoid_boxes=None):
    """Per-cell class SAFE / TARGET / AVOID from closed boxes on the cell centre."""
    m = _Marshal(system)
    d = len(m.lb)
    tb, nt = _boxes(target_boxes, d)
    ab, na = _boxes(avoid_boxes, d)
    cls = np.zeros(n_states(system), dtype=np.int8)
    lib().orc_label(C.byref(m.grid), nt, _dptr(tb), na, _dptr(ab),
                    cls.ctypes.data_as(C.POINTER(C.c_int8)))
    return cls


def lp_sorted(lo, hi, val, maximise):
    lo, hi, val = _f64(lo), _f64(hi), _f64(val)
    p = np.zeros(len(lo))
    q = lib().orc_lp_sorted(len(lo), _dptr(lo), _dptr(hi), _dptr(val), int(bool(maximise)),
                            _dptr(p))
    return q, p


def iterate(n_states_, n_inputs, row_ptr, target, lo, hi, cls, spec_kind, eps, max_sweeps,
            want_q0=False, hist_cap=0, optimistic=False, horizon=0, self_stop=False,
            n_dist=1):
    """Interval iteration (Alg. 3 / Alg. 4 with the sorting method); the
    policy is pessimistic (IMDP_lower = true, Sec. 5) unless ``optimistic``.
    ``horizon`` T > 0: finite horizon, T sweeps per pass (Remark 5.1).
    ``self_stop``: each pass stops when both its iterates converge to
    themselves (the first step of Remark 5.2).
    ``n_dist``: disturbances per (state, input); ``n_inputs`` then counts the
    control inputs only and the rows are (s * n_inputs + u) * n_dist + w.

    Returns dict(lo, hi, policy, status, sweeps, gap, converged, n_safe[, q0][, hist_v0, hist_v1]).
    """
    if isinstance(spec_kind, str):
        spec_kind = SPEC_KINDS[spec_kind]
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    target = np.ascontiguousarray(target, dtype=np.int32)
    lo, hi = _f64(lo), _f64(hi)
    cls = np.ascontiguousarray(cls, dtype=np.int8)
    out_lo, out_hi = np.zeros(n_states_), np.zeros(n_states_)
    pol = np.zeros(n_states_, dtype=np.int32)
    info = _IterInfo()
    q0 = np.full(n_states_ * n_inputs, np.nan) if want_q0 else None
    h0 = np.zeros((hist_cap, n_states_)) if hist_cap else None
    h1 = np.zeros((hist_cap, n_states_)) if hist_cap else None
    rc = lib().orc_iterate(
        n_states_, n_inputs, row_ptr.ctypes.data_as(C.POINTER(C.c_int64)),
        target.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(lo), _dptr(hi),
        cls.ctypes.data_as(C.POINTER(C.c_int8)), spec_kind, float(eps), int(max_sweeps),
        _dptr(out_lo), _dptr(out_hi), pol.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(info),
        _dptr(q0) if want_q0 else None, hist_cap, _dptr(h0) if hist_cap else None,
        _dptr(h1) if hist_cap else None, int(bool(optimistic)), int(horizon),
        int(bool(self_stop)), int(n_dist))
    if rc < 0:
        raise ValueError(f"oracle iterate rejected its input ({rc})")
    res = dict(lo=out_lo, hi=out_hi, policy=pol, status=rc, sweeps=tuple(info.sweeps),
               gap=tuple(info.gap), converged=tuple(info.converged), n_safe=info.n_safe)
    if want_q0:
        res["q0"] = q0.reshape(n_states_, n_inputs)
    if hist_cap:
        res["hist_v0"], res["hist_v1"] = h0, h1
    return res


def iterate_auto_horizon(n_states_, n_inputs, row_ptr, target, lo, hi, cls, spec_kind, eps,
                         max_sweeps, **kw):
    """Remark 5.2 for runs whose two bounds need not meet: the sweeps each pass
    needs for both of its iterates to converge to themselves; the larger count
    K is the horizon of a finite-horizon (value iteration) run, returned with
    ``horizon`` = K, ``self_sweeps`` and the self runs' ``converged``/``status``.
    """
    args = (n_states_, n_inputs, row_ptr, target, lo, hi, cls, spec_kind, eps, max_sweeps)
    first = iterate(*args, self_stop=True, **kw)
    K = max(1, max(first["sweeps"]))
    r = iterate(*args, horizon=K, **kw)
    r.update(horizon=K, self_sweeps=first["sweeps"], converged=first["converged"],
             status=first["status"])
    return r


def solve(system, k_sigma, spec_kind, target_boxes, avoid_boxes, eps, max_sweeps, **kw):
    """Build + label + iterate, the whole path on the CPU."""
    m = build(system, k_sigma)
    cls = label(system, target_boxes, avoid_boxes)
    _, nu, nw = with_disturbances(system)
    r = iterate(m["n_states"], nu, m["row_ptr"], m["target"], m["lo"], m["hi"], cls,
                spec_kind, eps, max_sweeps, n_dist=nw, **kw)
    r["cls"] = cls
    r["imdp"] = m
    return r
