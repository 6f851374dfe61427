"""Write oracle results that take too long to recompute inside a test.

Calls only the CPU oracle (``oracle/``) on the seeded workloads and stores the
results next to this script (JSON text, or compressed numpy arrays for the
full-size workloads).  Run from the repository root:

    python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2401_03555_amd import workloads as W  # noqa: E402


def robot2d():
    system, spec = W.robot2d()
    t = time.time()
    r = oracle.solve(system, system["k_sigma"], spec["kind"], spec["target"], spec["avoid"],
                     spec["eps"], spec["max_sweeps"], want_q0=True)
    return dict(
        workload="2D robot reach-avoid, 20x20 cells, 9 inputs, dense rows, eps 1e-8",
        generator="oracle.solve (tests/golden/make_golden.py)",
        seconds=time.time() - t,
        sweeps=list(r["sweeps"]), gap=list(r["gap"]), converged=list(r["converged"]),
        lo=[float(x) for x in r["lo"]], hi=[float(x) for x in r["hi"]],
        policy=[int(x) for x in r["policy"]],
        q0=[[None if np.isnan(x) else float(x) for x in row] for row in r["q0"]],
    )


TIE_TOL = 1e-12


def tie_mask(q0, reach):
    """Per state, a bit per input whose pass-1 V0 LP value (the last sweep's)
    is within TIE_TOL of the optimum: the inputs a policy may take at ties."""
    q = np.where(np.isnan(q0), -np.inf if reach else np.inf, q0)
    best = q.max(axis=1) if reach else q.min(axis=1)
    ok = (q >= best[:, None] - TIE_TOL) if reach else (q <= best[:, None] + TIE_TOL)
    bits = (ok.astype(np.int64) << np.arange(q.shape[1], dtype=np.int64)[None, :]).sum(axis=1)
    return bits.astype(np.int64)


def _npz_result(r, reach, workload, t, **extra):
    return dict(workload=np.array(workload), generator=np.array(
        "oracle.solve (tests/golden/make_golden.py)"), seconds=np.array(time.time() - t),
        sweeps=np.array(r["sweeps"], dtype=np.int64), status=np.array(r["status"]),
        lo=r["lo"], hi=r["hi"], policy=r["policy"].astype(np.int32),
        ties=tie_mask(r["q0"], reach), **extra)


def room5d_k2():
    """The full 5D room (10^5 cells, 4 inputs, rows of up to 3,127 entries), safety,
    two sweeps of each pass."""
    system, spec = W.room5d()
    t = time.time()
    r = oracle.solve(system, system["k_sigma"], spec["kind"], spec["target"], spec["avoid"],
                     spec["eps"], 2, want_q0=True)
    return _npz_result(r, False, "5D room safety, 10^5 cells, 4 inputs, +-6 sigma windows, "
                       "2 sweeps per pass", t)


def unicycle3d_converged():
    """The full 3D unicycle (50x50x24 cells, 20 inputs), reach-avoid to eps 1e-8."""
    system, spec = W.unicycle3d()
    t = time.time()
    r = oracle.solve(system, system["k_sigma"], spec["kind"], spec["target"], spec["avoid"],
                     spec["eps"], spec["max_sweeps"], want_q0=True)
    return _npz_result(r, True, "3D unicycle reach-avoid, 50x50x24 cells, 20 inputs, +-6 sigma "
                       "windows, eps 1e-8, run to convergence", t)


GENERATORS = {"robot2d": robot2d, "room5d_k2": room5d_k2,
              "unicycle3d_converged": unicycle3d_converged}
NPZ = {"room5d_k2", "unicycle3d_converged"}


def main(names):
    for name in names or GENERATORS:
        res = GENERATORS[name]()
        if name in NPZ:
            # arrays of 10^5 doubles: compressed numpy arrays (no pickled objects)
            path = os.path.join(HERE, f"{name}_oracle.npz")
            np.savez_compressed(path, **res)
        else:
            path = os.path.join(HERE, f"{name}_oracle.json")
            with open(path, "w") as f:
                json.dump(res, f, indent=0, allow_nan=False)
        print(f"wrote {path} ({float(res['seconds']):.1f} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
