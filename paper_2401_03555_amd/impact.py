"""Python binding of the gfx950 IMDP library (``libimpact.so``, C ABI in
``include/impact.h``).

Argument marshalling only: every step of construction and iteration runs in
the library's HIP kernels.  PyTorch supplies device memory (through its
caching allocator, passed to the library as alloc/free callbacks) and the
stream.  There is no fallback: if the library is not built, importing
``lib()`` raises.
"""
import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libimpact.so")

OK, NOT_CONVERGED = 0, 1
E_INVAL, E_NOMEM, E_HIP, E_UNSUPPORTED = -1, -2, -3, -4
SYS_KINDS = {"affine": 0, "unicycle": 1}
SPEC_KINDS = {"safety": 0, "reach": 1, "reach_avoid": 2}
STORAGE = {"auto": 0, "bounds": 1, "factors": 2}

# Every function the header declares (checked by the test suite).
EXPORTS = ["impact_build_imdp", "impact_interval_iterate", "impact_last_iter_info",
           "impact_imdp_get_info", "impact_imdp_export_rows", "impact_set_timing",
           "impact_imdp_free", "impact_last_error", "impact_version", "impact_set_sweep_mode",
           "impact_set_sweep_modes",
           "impact_build_imdp_batch", "impact_mq_create", "impact_mq_submit", "impact_mq_run",
           "impact_mq_poll", "impact_mq_query_info", "impact_mq_last_error", "impact_mq_free",
           "impact_probe_fp64_fma", "impact_build_imdp_dist", "impact_interval_iterate_noalloc",
           "impact_build_imdp_mc"]
SWEEP_MODES = {"auto": 0, "per_row": 1, "state_box": 2}

_pd = C.POINTER(C.c_double)
_pi32 = C.POINTER(C.c_int32)
_pi64 = C.POINTER(C.c_int64)


class System(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim_x", C.c_int32), ("dim_u", C.c_int32),
                ("A", _pd), ("B", _pd), ("c", _pd), ("dt", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("lb", _pd), ("ub", _pd), ("n", _pi32)]


class Inputs(C.Structure):
    _fields_ = [("count", C.c_int32), ("dim_u", C.c_int32), ("values", _pd)]


class Noise(C.Structure):
    _fields_ = [("sigma", _pd)]


class McNoise(C.Structure):
    _fields_ = [("inv_cov", _pd), ("det_cov", C.c_double), ("n_samples", C.c_int64),
                ("samples", _pd), ("grid_pts", C.c_int32), ("kappa", C.c_double)]


class Disturbances(C.Structure):
    _fields_ = [("count", C.c_int32), ("dim_w", C.c_int32), ("values", _pd), ("D", _pd)]


class Window(C.Structure):
    _fields_ = [("k_sigma", C.c_double), ("storage", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Device(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p),
                ("stream", C.c_void_p)]


class Spec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_target", C.c_int32), ("n_avoid", C.c_int32),
                ("target_boxes", _pd), ("avoid_boxes", _pd), ("pessimistic", C.c_int32),
                ("max_sweeps", C.c_int64), ("horizon", C.c_int64)]


class IterInfo(C.Structure):
    _fields_ = [("sweeps", C.c_int64 * 2), ("gap", C.c_double * 2),
                ("converged", C.c_int32 * 2), ("n_safe", C.c_int64),
                ("updates", C.c_int64 * 2), ("launches", C.c_int64 * 2),
                ("sweep_ms", C.c_double * 2), ("launch_ms", C.c_double * 2),
                ("iterate_ms", C.c_double), ("horizon", C.c_int64),
                ("self_sweeps", C.c_int64 * 2), ("self_sweep_ms", C.c_double)]


class ImdpInfo(C.Structure):
    _fields_ = [("n_states", C.c_int64), ("n_rows", C.c_int64), ("n_entries", C.c_int64),
                ("dim", C.c_int32), ("n_inputs", C.c_int32), ("windowed", C.c_int32),
                ("storage", C.c_int32), ("max_row", C.c_int32), ("max_box", C.c_int64),
                ("device_bytes", C.c_int64), ("build_ms", C.c_double), ("n_dist", C.c_int32)]


class ImpactError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"impact error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python paper_2401_03555_amd/build_lib.py`")
        L = C.CDLL(LIB_PATH)
        L.impact_build_imdp.restype = C.c_int
        L.impact_build_imdp.argtypes = [C.POINTER(System), C.POINTER(Grid), C.POINTER(Inputs),
                                        C.POINTER(Noise), C.POINTER(Window), C.POINTER(Device),
                                        C.POINTER(C.c_void_p)]
        L.impact_build_imdp_batch.restype = C.c_int
        L.impact_build_imdp_batch.argtypes = [C.c_int32, C.POINTER(System), C.POINTER(Grid),
                                              C.POINTER(Inputs), C.POINTER(Noise),
                                              C.POINTER(Window), C.POINTER(Device),
                                              C.POINTER(C.c_void_p)]
        L.impact_interval_iterate.restype = C.c_int
        L.impact_interval_iterate.argtypes = [C.c_void_p, C.POINTER(Spec), C.c_double, _pd, _pd,
                                              _pi32]
        L.impact_interval_iterate_noalloc.restype = C.c_int
        L.impact_interval_iterate_noalloc.argtypes = [C.c_void_p, C.POINTER(Spec), C.c_double,
                                                      _pd, _pd, _pi32]
        L.impact_last_iter_info.restype = C.c_int
        L.impact_last_iter_info.argtypes = [C.c_void_p, C.POINTER(IterInfo)]
        L.impact_imdp_get_info.restype = C.c_int
        L.impact_imdp_get_info.argtypes = [C.c_void_p, C.POINTER(ImdpInfo)]
        L.impact_imdp_export_rows.restype = C.c_int
        L.impact_imdp_export_rows.argtypes = [C.c_void_p, C.c_int64, C.c_int64, _pi32, _pd,
                                              _pi64, _pd]
        L.impact_set_sweep_mode.restype = C.c_int
        L.impact_set_sweep_mode.argtypes = [C.c_void_p, C.c_int32]
        L.impact_set_sweep_modes.restype = C.c_int
        L.impact_set_sweep_modes.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.impact_set_timing.restype = C.c_int
        L.impact_set_timing.argtypes = [C.c_void_p, C.c_int32]
        L.impact_imdp_free.restype = None
        L.impact_imdp_free.argtypes = [C.c_void_p]
        L.impact_last_error.restype = C.c_char_p
        L.impact_last_error.argtypes = []
        L.impact_version.restype = C.c_char_p
        L.impact_version.argtypes = []
        L.impact_mq_create.restype = C.c_int
        L.impact_mq_create.argtypes = [C.POINTER(Device), C.c_int32, C.POINTER(C.c_void_p)]
        L.impact_mq_submit.restype = C.c_int
        L.impact_mq_submit.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(Spec), C.c_double, _pd,
                                       _pd, _pi32, C.POINTER(C.c_int32)]
        L.impact_mq_run.restype = C.c_int
        L.impact_mq_run.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
        L.impact_mq_poll.restype = C.c_int
        L.impact_mq_poll.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.c_int32,
                                     C.POINTER(C.c_int32)]
        L.impact_mq_query_info.restype = C.c_int
        L.impact_mq_query_info.argtypes = [C.c_void_p, C.c_int32, C.POINTER(IterInfo)]
        L.impact_mq_last_error.restype = C.c_char_p
        L.impact_mq_last_error.argtypes = []
        L.impact_mq_free.restype = None
        L.impact_mq_free.argtypes = [C.c_void_p]
        L.impact_build_imdp_dist.restype = C.c_int
        L.impact_build_imdp_dist.argtypes = [C.POINTER(System), C.POINTER(Grid), C.POINTER(Inputs),
                                             C.POINTER(Disturbances), C.POINTER(Noise),
                                             C.POINTER(Window), C.POINTER(Device),
                                             C.POINTER(C.c_void_p)]
        L.impact_build_imdp_mc.restype = C.c_int
        L.impact_build_imdp_mc.argtypes = [C.POINTER(System), C.POINTER(Grid), C.POINTER(Inputs),
                                           C.POINTER(McNoise), C.POINTER(Window),
                                           C.POINTER(Device), C.POINTER(C.c_void_p)]
        L.impact_probe_fp64_fma.restype = C.c_int
        L.impact_probe_fp64_fma.argtypes = [C.c_int64, C.c_int32, _pd, C.c_void_p]
        _lib = L
    return _lib


HORIZON_AUTO = -1  # the two-step procedure for bounds that need not meet (Remark 5.2)


def _horizon(spec):
    h = spec.get("horizon", 0)
    return HORIZON_AUTO if h == "auto" else int(h)


def _check(rc):
    if rc < 0:
        raise ImpactError(rc, lib().impact_last_error().decode())
    return rc


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _dptr(a):
    return a.ctypes.data_as(_pd)


def _torch_ptr(t, ctype):
    return C.cast(C.c_void_p(t.data_ptr()), C.POINTER(ctype))


class _TorchDevice:
    """alloc/free callbacks backed by torch's caching allocator, plus the stream."""

    def __init__(self, stream=None):
        import torch
        self.torch = torch
        self.device = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream()

        def _alloc(nbytes, _ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:  # out of memory -> NULL -> IMPACT_E_NOMEM
                return None

        def _free(ptr, _ctx):
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.struct = Device(self._alloc, self._free, None, C.c_void_p(self.stream.cuda_stream))


class _Marshal:
    def __init__(self, system):
        self.lb, self.ub = _f64(system["lb"]), _f64(system["ub"])
        self.n = np.ascontiguousarray(np.asarray(system["n"], dtype=np.int32))
        d = len(self.lb)
        inputs = np.asarray(system["inputs"], dtype=np.float64)
        if inputs.ndim == 1:
            inputs = inputs.reshape(-1, 1) if inputs.size else np.zeros((1, 0))
        self.inputs = np.ascontiguousarray(inputs)
        du = self.inputs.shape[1]
        self.sigma = _f64(system["sigma"])
        self.grid = Grid(d, _dptr(self.lb), _dptr(self.ub), self.n.ctypes.data_as(_pi32))
        self.inp = Inputs(self.inputs.shape[0], du, _dptr(self.inputs) if du else None)
        self.noise = Noise(_dptr(self.sigma))
        self.dist = None
        if "disturbances" in system:
            wv = np.asarray(system["disturbances"], dtype=np.float64)
            self.wv = _f64(wv.reshape(wv.shape[0], -1))
            self.D = _f64(np.asarray(system["D"], dtype=np.float64).reshape(d, self.wv.shape[1]))
            self.dist = Disturbances(self.wv.shape[0], self.wv.shape[1], _dptr(self.wv),
                                     _dptr(self.D))
        kind = system["kind"]
        if kind == "affine":
            self.A = _f64(system["A"]).reshape(d, d)
            self.B = _f64(system["B"]).reshape(d, du) if du else _f64(np.zeros(1))
            self.c = _f64(system.get("c", np.zeros(d)))
            self.sys = System(0, d, du, _dptr(self.A), _dptr(self.B), _dptr(self.c), 0.0)
        elif kind == "unicycle":
            self.sys = System(1, d, du, None, None, None, float(system["dt"]))
        else:
            raise ValueError(f"unknown system kind {kind!r}")


class Imdp:
    """A built abstraction resident in HBM (owns a library handle)."""

    def __init__(self, handle, dev):
        self._h = handle
        self._dev = dev  # keeps the allocator callbacks alive as long as the handle

    @property
    def handle(self):
        return self._h

    def info(self):
        i = ImdpInfo()
        _check(lib().impact_imdp_get_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in ImdpInfo._fields_}

    def set_sweep_mode(self, mode):
        _check(lib().impact_set_sweep_mode(self._h, SWEEP_MODES[mode]))

    def set_sweep_modes(self, policy_pass, fixed_pass):
        _check(lib().impact_set_sweep_modes(self._h, SWEEP_MODES[policy_pass],
                                            SWEEP_MODES[fixed_pass]))

    def set_timing(self, enable=True):
        _check(lib().impact_set_timing(self._h, int(bool(enable))))

    def export_rows(self, row0, nrows, entries=True):
        """Rows [row0, row0 + nrows) as numpy: window, ot, counts (window cells), entries."""
        torch = self._dev.torch
        info = self.info()
        d = info["dim"]
        dev = f"cuda:{self._dev.device}"
        win = torch.empty((nrows, 2 * d), dtype=torch.int32, device=dev)
        ot = torch.empty((nrows, 4), dtype=torch.float64, device=dev)
        cnt = torch.empty(nrows, dtype=torch.int64, device=dev)
        _check(lib().impact_imdp_export_rows(self._h, row0, nrows, _torch_ptr(win, C.c_int32),
                                             _torch_ptr(ot, C.c_double),
                                             _torch_ptr(cnt, C.c_int64), None))
        out = dict(win=win.cpu().numpy(), ot=ot.cpu().numpy(), counts=cnt.cpu().numpy())
        if entries:
            total = int(out["counts"].sum())
            ent = torch.empty((max(total, 1), 2), dtype=torch.float64, device=dev)
            _check(lib().impact_imdp_export_rows(self._h, row0, nrows, _torch_ptr(win, C.c_int32),
                                                 _torch_ptr(ot, C.c_double),
                                                 _torch_ptr(cnt, C.c_int64),
                                                 _torch_ptr(ent, C.c_double)))
            out["entries"] = ent.cpu().numpy()[:total]
        return out

    def iterate(self, spec, eps=None, max_sweeps=None, out=None, noalloc=False):
        """Interval iteration; returns dict(lo, hi, policy (torch cuda), status, info).

        noalloc: run impact_interval_iterate_noalloc (temporaries in the
        library's static device array instead of the allocator)."""
        torch = self._dev.torch
        d = self.info()["dim"]
        n = self.info()["n_states"]
        tb = _f64(np.asarray(spec.get("target") or np.zeros((0, 2, d))).reshape(-1, 2, d))
        ab = _f64(np.asarray(spec.get("avoid") or np.zeros((0, 2, d))).reshape(-1, 2, d))
        s = Spec(SPEC_KINDS[spec["kind"]], tb.shape[0], ab.shape[0],
                 _dptr(tb) if tb.size else None, _dptr(ab) if ab.size else None,
                 int(bool(spec.get("pessimistic", True))),
                 int(max_sweeps if max_sweeps is not None else spec.get("max_sweeps", 100000)),
                 _horizon(spec))
        dev = f"cuda:{self._dev.device}"
        if out is None:
            lo = torch.empty(n, dtype=torch.float64, device=dev)
            hi = torch.empty(n, dtype=torch.float64, device=dev)
            pol = torch.empty(n, dtype=torch.int32, device=dev)
        else:
            lo, hi, pol = out
        fn = lib().impact_interval_iterate_noalloc if noalloc else lib().impact_interval_iterate
        rc = _check(fn(
            self._h, C.byref(s), float(eps if eps is not None else spec["eps"]),
            _torch_ptr(lo, C.c_double), _torch_ptr(hi, C.c_double), _torch_ptr(pol, C.c_int32)))
        return dict(lo=lo, hi=hi, policy=pol, status=rc, info=self.last_iter_info())

    def last_iter_info(self):
        i = IterInfo()
        _check(lib().impact_last_iter_info(self._h, C.byref(i)))
        return dict(sweeps=tuple(i.sweeps), gap=tuple(i.gap), converged=tuple(i.converged),
                    n_safe=i.n_safe, updates=tuple(i.updates), launches=tuple(i.launches),
                    sweep_ms=tuple(i.sweep_ms), launch_ms=tuple(i.launch_ms),
                    iterate_ms=i.iterate_ms, horizon=i.horizon,
                    self_sweeps=tuple(i.self_sweeps), self_sweep_ms=i.self_sweep_ms)

    def free(self):
        if self._h:
            lib().impact_imdp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_imdp(system, k_sigma=None, storage="bounds", stream=None, timing=False,
               sweep_mode="auto"):
    """Build the abstraction of ``system`` on the current CUDA(HIP) device."""
    m = _Marshal(system)
    dev = _TorchDevice(stream)
    w = Window(float(system.get("k_sigma", 0.0) if k_sigma is None else k_sigma),
               STORAGE[storage])
    h = C.c_void_p()
    if m.dist is not None:
        _check(lib().impact_build_imdp_dist(C.byref(m.sys), C.byref(m.grid), C.byref(m.inp),
                                            C.byref(m.dist), C.byref(m.noise), C.byref(w),
                                            C.byref(dev.struct), C.byref(h)))
    else:
        _check(lib().impact_build_imdp(C.byref(m.sys), C.byref(m.grid), C.byref(m.inp),
                                       C.byref(m.noise), C.byref(w), C.byref(dev.struct),
                                       C.byref(h)))
    imdp = Imdp(h.value, dev)
    if timing:
        imdp.set_timing(True)
    if sweep_mode != "auto":
        imdp.set_sweep_mode(sweep_mode)
    return imdp


def build_imdp_mc(system, mc, k_sigma=None, stream=None, timing=False, sweep_mode="auto"):
    """Build the abstraction of ``system`` under correlated noise (Monte Carlo
    cell masses).  ``mc``: dict with ``inv_cov`` (d x d), ``det_cov``,
    ``samples`` (N x d points of [0, 1)), ``grid_pts`` and ``kappa``;
    ``system["sigma"]`` is not used."""
    m = _Marshal(dict(system, sigma=np.ones(len(system["lb"]))))
    P, X = _f64(mc["inv_cov"]), _f64(mc["samples"])
    d = len(m.lb)
    nz = McNoise(_dptr(P), float(mc["det_cov"]), X.size // d, _dptr(X), int(mc["grid_pts"]),
                 float(mc["kappa"]))
    dev = _TorchDevice(stream)
    w = Window(float(system.get("k_sigma", 0.0) if k_sigma is None else k_sigma),
               STORAGE["bounds"])
    h = C.c_void_p()
    _check(lib().impact_build_imdp_mc(C.byref(m.sys), C.byref(m.grid), C.byref(m.inp),
                                      C.byref(nz), C.byref(w), C.byref(dev.struct), C.byref(h)))
    imdp = Imdp(h.value, dev)
    if timing:
        imdp.set_timing(True)
    if sweep_mode != "auto":
        imdp.set_sweep_mode(sweep_mode)
    return imdp


def _mq_check(rc):
    if rc < 0:
        raise ImpactError(rc, lib().impact_mq_last_error().decode())
    return rc


def _spec_struct(spec, d, max_sweeps=None):
    tb = _f64(np.asarray(spec.get("target") or np.zeros((0, 2, d))).reshape(-1, 2, d))
    ab = _f64(np.asarray(spec.get("avoid") or np.zeros((0, 2, d))).reshape(-1, 2, d))
    s = Spec(SPEC_KINDS[spec["kind"]], tb.shape[0], ab.shape[0],
             _dptr(tb) if tb.size else None, _dptr(ab) if ab.size else None,
             int(bool(spec.get("pessimistic", True))),
             int(max_sweeps if max_sweeps is not None else spec.get("max_sweeps", 100000)),
             _horizon(spec))
    return s, (tb, ab)


class Engine:
    """Multi-query engine: interval-iteration queries in flight together."""

    def __init__(self, max_queries=1024, stream=None):
        self._dev = _TorchDevice(stream)
        h = C.c_void_p()
        _mq_check(lib().impact_mq_create(C.byref(self._dev.struct), int(max_queries), C.byref(h)))
        self._h = h.value
        self._out = {}    # id -> (lo, hi, policy) tensors
        self._keep = {}   # id -> abstraction (python side)

    def submit(self, imdp, spec, eps=None, max_sweeps=None, out=None):
        torch = self._dev.torch
        info = imdp.info()
        d, n = info["dim"], info["n_states"]
        s, keep = _spec_struct(spec, d, max_sweeps)
        dev = f"cuda:{self._dev.device}"
        if out is None:
            out = (torch.empty(n, dtype=torch.float64, device=dev),
                   torch.empty(n, dtype=torch.float64, device=dev),
                   torch.empty(n, dtype=torch.int32, device=dev))
        lo, hi, pol = out
        qid = C.c_int32()
        _mq_check(lib().impact_mq_submit(
            self._h, imdp.handle, C.byref(s), float(eps if eps is not None else spec["eps"]),
            _torch_ptr(lo, C.c_double), _torch_ptr(hi, C.c_double), _torch_ptr(pol, C.c_int32),
            C.byref(qid)))
        self._out[qid.value] = out
        self._keep[qid.value] = imdp
        return qid.value

    def run(self, steps=16):
        n = C.c_int32()
        _mq_check(lib().impact_mq_run(self._h, int(steps), C.byref(n)))
        return n.value

    def poll(self, cap=4096):
        ids = (C.c_int32 * cap)()
        n = C.c_int32()
        _mq_check(lib().impact_mq_poll(self._h, ids, cap, C.byref(n)))
        done = []
        for k in range(n.value):
            qid = ids[k]
            i = IterInfo()
            _mq_check(lib().impact_mq_query_info(self._h, qid, C.byref(i)))
            lo, hi, pol = self._out.pop(qid)
            self._keep.pop(qid, None)
            done.append(dict(id=qid, lo=lo, hi=hi, policy=pol,
                             status=0 if (i.converged[0] and i.converged[1]) else 1,
                             info=dict(sweeps=tuple(i.sweeps), gap=tuple(i.gap),
                                       converged=tuple(i.converged), n_safe=i.n_safe,
                                       updates=tuple(i.updates), horizon=i.horizon,
                                       self_sweeps=tuple(i.self_sweeps))))
        return done

    def run_all(self, chunk=64):
        results = {}
        while True:
            active = self.run(chunk)
            for r in self.poll():
                results[r["id"]] = r
            if active == 0 and not self._out:
                break
        return results

    def free(self):
        if self._h:
            lib().impact_mq_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_imdp_batch(systems, storage="bounds", stream=None, sweep_mode="auto"):
    """Build several abstractions with one launch of each construction kernel."""
    if any("disturbances" in s for s in systems):
        raise ValueError("the batch build takes no disturbance player; use build_imdp")
    n = len(systems)
    ms = [_Marshal(s) for s in systems]
    dev = _TorchDevice(stream)
    SysA, GridA, InA, NoiseA, WinA = (System * n), (Grid * n), (Inputs * n), (Noise * n), (Window * n)
    sa = SysA(*[m.sys for m in ms])
    ga = GridA(*[m.grid for m in ms])
    ia = InA(*[m.inp for m in ms])
    na = NoiseA(*[m.noise for m in ms])
    wa = WinA(*[Window(float(s.get("k_sigma", 0.0)), STORAGE[storage]) for s in systems])
    hs = (C.c_void_p * n)()
    _check(lib().impact_build_imdp_batch(n, sa, ga, ia, na, wa, C.byref(dev.struct), hs))
    out = [Imdp(h, dev) for h in hs]
    if sweep_mode != "auto":
        for m in out:
            m.set_sweep_mode(sweep_mode)
    return out


def version():
    return lib().impact_version().decode()


def probe_fp64_fma(n_blocks=2048, iters=1024, reps=3):
    """FP64 FMA rate (TFLOP/s) of the library's probe kernel on torch's
    current stream, best of ``reps`` launches (measurement support)."""
    import torch
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    best = None
    for _ in range(reps + 1):                   # the first launch is a warmup
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        _check(lib().impact_probe_fp64_fma(n_blocks, iters, C.cast(out.data_ptr(), _pd),
                                           C.c_void_p(st.cuda_stream)))
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return 2.0 * 16 * iters * 256 * n_blocks / (best * 1e-3) / 1e12
