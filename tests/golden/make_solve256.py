"""Write solve256.json: the oracle's solution of the 256^3 mixed-precision
workload, for the error of the GPU solutions against the FP64 oracle.

Calls only `oracle` and `workloads`.  Grid 256^3 cells (h = 1/256), x,y
periodic, zero-velocity walls, E = 1, nu = 0.35; b = D_h sigma with sigma the
smoothed N(0,1) stress of seed 2 (3 Jacobi passes); x0 = 0; V(2,2) cycles on
6 levels until the relative residual is <= 1e-12 (tighter than the 1e-10 the
GPU solves stop at, so that the stored values are the discrete solution to
about 1e-12).  Stored: the solution's L2 norm over all nodes, 4096 sampled
interior nodes (seeded) with their three components, the residual history.
Runs about 30 minutes on one core.

    python tests/golden/make_solve256.py [n]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.multigrid import MGOracle  # noqa: E402
from oracle.operators import div_node  # noqa: E402
from workloads import lame, stress_field  # noqa: E402

RTOL = 1e-12


def sample_nodes(n, count=4096, seed=11):
    """(k, j, i) of `count` interior nodes of an n^3-cell grid."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, n, count)
    j = rng.integers(0, n, count)
    i = rng.integers(0, n, count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(k, j, i)]


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 256
    lam, mu = lame()
    h = 1.0 / n
    b = div_node(stress_field(n, n, n, 2), h)
    mg = MGOracle(n, n, n, h, lam, mu)
    t0 = time.time()
    x, info = mg.solve(b, np.zeros_like(b), rtol=RTOL, max_cycles=60)
    idx = sample_nodes(n)
    out = {
        "_source": "oracle.multigrid.MGOracle.solve via tests/golden/make_solve256.py",
        "n": n, "rhs": "D_h sigma, sigma = workloads.stress_field(n, n, n, 2)",
        "rtol": RTOL, "cycles": int(info["cycles"]),
        "rel_res_hist": [float(r) for r in info["hist"]],
        "x_norm": float(np.linalg.norm(x)),
        "sample_index": idx,
        "sample_x": [[float(x[c][t]) for c in range(3)] for t in idx],
        "seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "solve%d.json" % n)
    with open(path, "w") as f:
        json.dump(out, f)
    print(path, out["cycles"], out["x_norm"], out["seconds"])


if __name__ == "__main__":
    main()
