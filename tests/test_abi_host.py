"""Host-only checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments / failed allocations before touching
the GPU (no GPU is needed for any of these)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2401_03555_amd import impact as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(impact_\w+)\s*\(", text))
    return names


def test_library_exports_every_declared_function():
    L = I.lib()
    decl = declared_functions()
    assert decl, "no declarations found"
    assert decl == set(I.EXPORTS)
    for name in decl:
        assert hasattr(L, name), name
    assert I.version().startswith("impact-gfx950")


def _args(system):
    m = I._Marshal(system)
    w = I.Window(float(system["k_sigma"]), 1)
    return m, w


def _build(m, w, dev=None):
    h = C.c_void_p()
    rc = I.lib().impact_build_imdp(C.byref(m.sys), C.byref(m.grid), C.byref(m.inp),
                                   C.byref(m.noise), C.byref(w),
                                   C.byref(dev) if dev is not None else None, C.byref(h))
    return rc, h


def _system():
    return dict(kind="affine", A=np.eye(2), B=0.5 * np.eye(2), c=np.zeros(2), lb=[-1.0, -1.0],
                ub=[1.0, 1.0], n=[4, 4], inputs=np.zeros((1, 2)), sigma=[0.1, 0.1], k_sigma=6.0)


@pytest.mark.parametrize("mutate,code", [
    (lambda s: s.update(sigma=[0.1, 0.0]), I.E_INVAL),
    (lambda s: s.update(sigma=[0.1, float("nan")]), I.E_INVAL),
    (lambda s: s.update(n=[4, 0]), I.E_INVAL),
    (lambda s: s.update(lb=[-1.0, 1.0]), I.E_INVAL),
    (lambda s: s.update(k_sigma=-1.0), I.E_INVAL),
    (lambda s: s.update(A=np.array([[1.0, float("inf")], [0.0, 1.0]])), I.E_INVAL),
])
def test_build_rejects_bad_arguments(mutate, code):
    s = _system()
    mutate(s)
    m, w = _args(s)
    rc, h = _build(m, w)
    assert rc == code and not h.value
    assert I.lib().impact_last_error().decode()


def test_build_rejects_unicycle_shape():
    s = _system()
    s["kind"] = "unicycle"
    s["dt"] = 0.1
    m, w = _args(s)
    rc, _ = _build(m, w)
    assert rc == I.E_INVAL and b"unicycle" in I.lib().impact_last_error()


def test_build_rejects_unknown_storage():
    m, _ = _args(_system())
    rc, _ = _build(m, I.Window(6.0, 7))
    assert rc == I.E_INVAL


def test_failed_allocation_reports_nomem_without_gpu_work():
    calls = []

    def alloc(n, ctx):
        calls.append(n)
        return None

    def free(p, ctx):
        raise AssertionError("nothing was allocated")

    fa, ff = I.ALLOC_FN(alloc), I.FREE_FN(free)
    dev = I.Device(fa, ff, None, None)
    m, w = _args(_system())
    rc, h = _build(m, w, dev)
    assert rc == I.E_NOMEM and not h.value and calls
    assert b"allocation" in I.lib().impact_last_error()


def test_null_handles_are_rejected():
    L = I.lib()
    assert L.impact_interval_iterate(None, None, 1e-8, None, None, None) == I.E_INVAL
    assert L.impact_imdp_get_info(None, None) == I.E_INVAL
    assert L.impact_last_iter_info(None, None) == I.E_INVAL
    assert L.impact_set_timing(None, 1) == I.E_INVAL
    assert L.impact_imdp_export_rows(None, 0, 1, None, None, None, None) == I.E_INVAL
    L.impact_imdp_free(None)
