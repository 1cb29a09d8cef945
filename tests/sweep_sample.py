"""One Gauss-Seidel sweep, evaluated node by node with the oracle (Sec. 3.6).

A multicolour sweep visits the eight parity colours in a fixed order and
updates all nodes of one colour together.  The new value of a node therefore
depends only on its 3x3x3 neighbourhood: neighbours of colours that come
earlier in the order contribute their new values, all others (and the walls)
their old ones.  Given the state before and after a sweep at any grid size,
the oracle can thus recompute the sweep at sampled nodes one by one: it runs
its own colour pass on a periodic 3x3x3 patch holding that mixed
neighbourhood and the node's plane stencils, where the centre node is the
only node of its colour.

Test infrastructure: uses only `oracle/`.
"""
from __future__ import annotations

import numpy as np

from oracle.multigrid import Level


def sweep_at_nodes(A, x_old, x_new, b, nodes, order):
    """Oracle values after one sweep at `nodes` ((k, j, i) interior nodes).

    A: per-plane stencils of the level, A[k, oz+1, oy+1, ox+1, c, d];
    x_old, x_new: the level's node vectors before and after the sweep
    ([3][nz+1][ny][nx]); b: its right-hand side; order: the colours as
    (i, j, k) parity triples in the order the sweep visits them.
    Returns an array of shape (len(nodes), 3).
    """
    _, nzp1, ny, nx = x_old.shape
    nz = nzp1 - 1
    rank = {tuple(c): t for t, c in enumerate(order)}
    out = np.empty((len(nodes), 3))
    for s, (k, j, i) in enumerate(nodes):
        if not 1 <= k <= nz - 1:
            raise ValueError("node (%d, %d, %d) is not interior" % (k, j, i))
        mine = rank[(i & 1, j & 1, k & 1)]
        ks = np.arange(k - 1, k + 2)
        js = np.arange(j - 1, j + 2) % ny
        is_ = np.arange(i - 1, i + 2) % nx
        patch = x_old[np.ix_(range(3), ks, js, is_)].copy()
        newer = x_new[np.ix_(range(3), ks, js, is_)]
        for dz in range(3):
            if ks[dz] in (0, nz):
                continue  # walls are never updated
            for dy in range(3):
                for dx in range(3):
                    if rank[(is_[dx] & 1, js[dy] & 1, ks[dz] & 1)] < mine:
                        patch[:, dz, dy, dx] = newer[:, dz, dy, dx]
        bp = b[np.ix_(range(3), ks, js, is_)]
        # the patch's only interior plane is plane 1 (the node's plane k), and
        # the centre is the only node of parity (1, 1, 1) in a 3 x 3 x 3 patch
        Level(3, 3, 2, A[k - 1:k + 2]).colour_pass(patch, bp, (1, 1, 1))
        out[s] = patch[:, 1, 1, 1]
    return out
