"""Write oracle reference values for the larger workloads into tests/golden/.

Calls only the CPU oracle and the seeded input generators.  Usage:
    python tests/golden/make_golden.py cfg2
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2601_16169_amd import inputs as I  # noqa: E402
from oracle import core, davidson  # noqa: E402


def run(name: str, tol: float) -> dict:
    prob = I.WORKLOADS[name]()
    sp = core.Space.from_problem(prob)
    t0 = time.time()
    diag = sp.diag()
    if sp.dim > 100000:
        # evaluate H once (same elements as the matrix-free oracle), then iterate
        H = core.MemoisedH(sp)
        apply_h = H.matvec
    else:
        apply_h = sp.sigma
    res = davidson.davidson(apply_h, diag, I.guess_noise(sp.dim), tol=tol, max_iter=400)
    x = res.vector
    top = np.argsort(-np.abs(x))[:256]
    return {
        "workload": prob.name,
        "source": "oracle/davidson.py over oracle/sqd_oracle.c (plain Davidson-Liu, FP64)",
        "tol": tol,
        "energy": res.energy,
        "iterations": res.iterations,
        "residual": res.residual,
        "converged": res.converged,
        "dim": sp.dim,
        "top_index": [int(k) for k in top],
        "top_value": [float(x[k]) for k in top],
        "seconds": time.time() - t0,
        "threads": core.num_threads(),
    }


if __name__ == "__main__":
    name = sys.argv[1]
    tol = float(sys.argv[2]) if len(sys.argv) > 2 else 1e-8
    out = run(name, tol)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("energy", "iterations", "residual", "seconds")}))
