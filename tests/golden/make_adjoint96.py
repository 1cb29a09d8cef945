"""Write adjoint96.json: oracle reference for the 96^3 x 10-step adjoint.

Calls only `oracle` and `workloads`.  Simple shear, dt = 10 t_s, U = 1e-5
L/t_s, sigma^0 = 0.99 s_Y in xz, chi^0 = Gaussian random field (mean 0.05,
std 0.003, correlation length 8 cells, seed 4); loss = mean sigma_xz^2 on the
two cell layers next to z = 1/2 after 10 steps; every solve (forward and
adjoint) runs exactly 40 V-cycles, which converges it to rounding.
Stored: the loss, d loss/d chi^0 projected on 16 unit-RMS directions
(seeds 100..115) and 256 sampled gradient entries.  Runs ~1 h on 8 cores.

    python tests/golden/make_adjoint96.py [n] [steps]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint as adj  # noqa: E402
from oracle.multigrid import MGOracle  # noqa: E402
from workloads import lame, shear_state, stz_constants  # noqa: E402


def directions(shape, seeds=range(100, 116)):
    out = []
    for s in seeds:
        d = np.random.default_rng(s).standard_normal(shape)
        out.append(d / np.sqrt(np.mean(d * d)))
    return out


def sample_index(shape, count=256, seed=7):
    rng = np.random.default_rng(seed)
    return [tuple(int(rng.integers(0, m)) for m in shape) for _ in range(count)]


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 96
    steps = int(sys.argv[2]) if len(sys.argv) > 2 else 10
    lam, mu = lame()
    p = stz_constants()
    h, dt, U = 1.0 / n, 10.0, 1e-5
    st = shear_state(n, n, n, seed=4, U=U)
    mg = MGOracle(n, n, n, h, lam, mu)
    t0 = time.time()
    loss, g = adj.rollout_grad_chi0(st["v"], st["sigma"], st["chi"], h, dt, lam, mu, p, U, mg,
                                    steps, rtol=0.0, max_cycles=40)
    dirs = directions(g.shape)
    idx = sample_index(g.shape)
    out = {
        "_source": "oracle.adjoint.rollout_grad_chi0 via tests/golden/make_adjoint96.py",
        "n": n, "steps": steps, "dt": dt, "U": U, "chi_seed": 4, "cycles_per_solve": 40,
        "loss": loss,
        "dir_seeds": list(range(100, 116)),
        "dir_derivs": [float(np.sum(g * d)) for d in dirs],
        "sample_index": idx,
        "sample_grad": [float(g[i]) for i in idx],
        "grad_rms": float(np.sqrt(np.mean(g * g))),
        "seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint%d.json" % n)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["loss"], out["seconds"])


if __name__ == "__main__":
    main()
