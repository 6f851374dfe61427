"""Compile the gfx950 HIP library ``libimpact.so`` in-tree with hipcc.

Flags: FP64 everywhere with no FMA contraction (-ffp-contract=off) so that
window edges are reproducible; packed-FP32 instructions disabled.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libimpact.so")
SOURCES = ["sweep_sb_d3.hip", "sweep_sb_d2.hip", "sweep_sb_d5.hip", "sweep_sb_d0.hip",
           "sweep.hip", "sweep_sel.hip", "abi.hip", "build.hip", "build_mc.hip", "sweep_sb.hip", "mq.hip", "probe.hip"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def _stale(src: str, obj: str, headers) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in (src, *headers))


def build(verbose: bool = False, extra=(), incremental: bool = False) -> str:
    """Compile every source to an object (in parallel), then link the library.

    incremental: recompile only sources whose object is older than the source
    or any header of the library (a development convenience; the default
    rebuilds everything)."""
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-parameter",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, *extra]
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]

    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    headers.append(os.path.join(ROOT, "include", "impact.h"))

    def compile_one(k):
        src = os.path.join(CSRC, SOURCES[k])
        if incremental and not _stale(src, objs[k], headers):
            return subprocess.CompletedProcess([], 0, "", "")
        cmd = [hipcc(), *flags, "-c", src, "-o", objs[k]]
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, capture_output=True, text=True)

    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(compile_one, range(len(SOURCES))))
    for src, r in zip(SOURCES, results):
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
    link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=[a for a in sys.argv[1:] if a not in ("-v", "-i")],
          incremental="-i" in sys.argv)
