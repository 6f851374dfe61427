"""Write oracle results that take too long to recompute inside a test.

Calls only the CPU oracle (``oracle/``) on the seeded workloads and stores the
results as JSON text next to this script.  Run from the repository root:

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


GENERATORS = {"robot2d": robot2d}


def main(names):
    for name in names or GENERATORS:
        res = GENERATORS[name]()
        path = os.path.join(HERE, f"{name}_oracle.json")
        with open(path, "w") as f:
            json.dump(res, f, indent=0, allow_nan=False)
        print(f"wrote {path} ({res['seconds']:.1f} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
