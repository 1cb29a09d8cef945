"""The oracle's STZ step (Sec. 3.1, Eq. sig_star_qs; with Eq. sig_star_evol
and Eq. ENO for the advection) evaluated at single cells of a large grid.

The step at a cell reads the stress and chi of the cells up to two away
along each axis (the ENO stencils of the advection; the chi diffusion term
reads D^pl, a function of stress and chi, one cell away) and the velocity at
its own eight corner nodes.  The oracle's step on the 5 x 5 x 5 cells around
a cell (periodic in x and y, so the patch wraps like the grid) therefore
gives that cell's result.  Within two cells of a wall the patch is shifted to
hold the wall layers, so that the ghost layers are extrapolated from the same
two layers as on the whole grid.

Test infrastructure: uses only `oracle/`.
"""
from __future__ import annotations

import numpy as np

from oracle import stz as ostz


def stz_step_at_cells(v, sigma, chi, h, dt, lam, mu, p, cells):
    """sigma* (6 values) and chi' at each of `cells` ((k, j, i) triples).

    v: node velocity [3][nz+1][ny][nx]; sigma: Voigt cell stress
    [6][nz][ny][nx]; chi: [nz][ny][nx]; p: the oracle's STZ parameters.
    Returns (sigma_star (len(cells), 6), chi_next (len(cells),)).
    """
    nz, ny, nx = chi.shape
    if nz < 5:
        raise ValueError("needs at least 5 cell layers")
    ss = np.empty((len(cells), 6))
    cn = np.empty(len(cells))
    for s, (k, j, i) in enumerate(cells):
        k0 = min(max(k - 2, 0), nz - 5)
        kc = list(range(k0, k0 + 5))
        kn = list(range(k0, k0 + 6))
        jj = [(j + d) % ny for d in range(-2, 3)]
        ii = [(i + d) % nx for d in range(-2, 3)]
        sp = sigma[np.ix_(range(6), kc, jj, ii)]
        cp = chi[np.ix_(kc, jj, ii)]
        vp = v[np.ix_(range(3), kn, jj, ii)]
        rs, rc = ostz.stz_step(vp, sp, cp, h, dt, lam, mu, p)
        ss[s] = rs[:, k - k0, 2, 2]
        cn[s] = rc[k - k0, 2, 2]
    return ss, cn


def near_yield_state(rng, nx, ny, nz, s_y):
    """Seeded inputs for the step: stresses of random direction whose
    deviator norm sbar lies within 10 % of s_y, chi around 0.05 (std 0.003)
    and small random velocities."""
    sig = rng.standard_normal((6, nz, ny, nx))
    pr = (sig[0] + sig[1] + sig[2]) / 3
    d = sig.copy()
    d[:3] -= pr
    sb = np.sqrt(0.5 * (d[0] ** 2 + d[1] ** 2 + d[2] ** 2) + d[3] ** 2 + d[4] ** 2 + d[5] ** 2)
    sig *= s_y * rng.uniform(0.9, 1.1, size=sb.shape) / sb
    chi = 0.05 + 0.003 * rng.standard_normal((nz, ny, nx))
    v = 1e-4 * rng.standard_normal((3, nz + 1, ny, nx))
    return v, sig, chi
