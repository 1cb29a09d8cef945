"""Discrete operators on the staggered grid (paper Sec. 3.3-3.4).

Velocity lives on nodes (3, nz+1, ny, nx); nodes k = 0 and k = nz are the
Dirichlet walls, the others are unknowns.  Stress lives on cells
(6, nz, ny, nx), Voigt order (xx, yy, zz, yz, xz, xy).  x and y are periodic.

The projection system (Eq. proj, multiplied by -1/dt so the matrix is SPD)

    K v = D_h sigma* / dt,      K v := -div(C : grad v)

is discretised with the collocated second difference (Eq. col_snd_deriv) for
the pure second derivatives and the four-point mixed difference of Sec. 3.4
for the cross derivatives, both taken at the nodes.  With
div(C : grad v)_c = (lam+2mu) d_cc v_c + mu sum_{a!=c} d_aa v_c
                    + (lam+mu) sum_{d!=c} d_cd v_d
this couples each node to its 3x3x3 neighbourhood (Sec. 3.6), and the
resulting matrix is symmetric positive definite (Sec. 3.3).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# unit offsets (oz, oy, ox) of the coordinate directions x, y, z
UNIT = {0: (0, 0, 1), 1: (0, 1, 0), 2: (1, 0, 0)}
VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def kappa(c: int, a: int, lam: float, mu: float) -> float:
    """Coefficient of d_aa v_c in div(C : grad v)_c."""
    return lam + 2.0 * mu if a == c else mu


def shifted_interior(f: np.ndarray, oz: int, oy: int, ox: int) -> np.ndarray:
    """f at (k+oz, j+oy, i+ox) for every interior node k = 1..nz-1.

    f has node layout (..., nz+1, ny, nx); y and x wrap periodically.
    """
    nz = f.shape[-3] - 1
    w = f[..., 1 + oz: nz + oz, :, :]
    if oy:
        w = np.roll(w, -oy, axis=-2)
    if ox:
        w = np.roll(w, -ox, axis=-1)
    return w


def apply_elastic(v: np.ndarray, h: float, lam: float, mu: float) -> np.ndarray:
    """K v at the interior nodes (wall rows of the result are zero).

    Wall planes of `v` are used as given, so K v here is K_II v_I + K_IB v_B.
    Works for real or complex `v`.
    """
    out = np.zeros_like(v)
    for c in range(3):
        vc = v[c]
        centre = vc[1:-1]
        acc = np.zeros_like(centre)
        for a in range(3):
            o = UNIT[a]
            m = tuple(-t for t in o)
            acc = acc + kappa(c, a, lam, mu) * (
                shifted_interior(vc, *o) + shifted_interior(vc, *m) - 2.0 * centre)
        for d in range(3):
            if d == c:
                continue
            mixed = np.zeros_like(centre)
            for s in (1, -1):
                for t in (1, -1):
                    off = tuple(s * p + t * q for p, q in zip(UNIT[c], UNIT[d]))
                    mixed = mixed + (s * t) * shifted_interior(v[d], *off)
            acc = acc + (lam + mu) * 0.25 * mixed
        out[c, 1:-1] = -acc / (h * h)
    return out


def node_index(nx: int, ny: int, nz: int) -> np.ndarray:
    """Flat index of every (c, k, j, i) in the (3, nz+1, ny, nx) layout."""
    return np.arange(3 * (nz + 1) * ny * nx).reshape(3, nz + 1, ny, nx)


def interior_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    m = np.zeros((3, nz + 1, ny, nx), dtype=bool)
    m[:, 1:nz] = True
    return m.ravel()


def assemble_elastic(nx: int, ny: int, nz: int, h: float, lam: float, mu: float) -> sp.csr_matrix:
    """Sparse K: rows for interior nodes, columns for all nodes (walls included).

    Entry-by-entry assembly of the same stencil; repeated (wrapped) entries
    are summed, which is what periodic wrap means when a dimension is 2.
    """
    idx = node_index(nx, ny, nz)
    K, J, I = np.meshgrid(np.arange(1, nz), np.arange(ny), np.arange(nx), indexing="ij")
    rows, cols, vals = [], [], []

    def add(c, d, oz, oy, ox, coef):
        r = idx[c, K, J, I].ravel()
        q = idx[d, K + oz, (J + oy) % ny, (I + ox) % nx].ravel()
        rows.append(r)
        cols.append(q)
        vals.append(np.full(r.shape, coef))

    ih2 = 1.0 / (h * h)
    for c in range(3):
        diag = 0.0
        for a in range(3):
            k_ = kappa(c, a, lam, mu)
            oz, oy, ox = UNIT[a]
            add(c, c, oz, oy, ox, -k_ * ih2)
            add(c, c, -oz, -oy, -ox, -k_ * ih2)
            diag += 2.0 * k_ * ih2
        add(c, c, 0, 0, 0, diag)
        for d in range(3):
            if d == c:
                continue
            for s in (1, -1):
                for t in (1, -1):
                    oz, oy, ox = (s * p + t * q for p, q in zip(UNIT[c], UNIT[d]))
                    add(c, d, oz, oy, ox, -(lam + mu) * 0.25 * s * t * ih2)
    n = 3 * (nz + 1) * ny * nx
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


# ---------------------------------------------------------------------------
# Staggered differences (Eq. stag_stenc) and the tensors built from them.
# ---------------------------------------------------------------------------

def _cell_diff(f: np.ndarray, axis_dir: int, h: float) -> np.ndarray:
    """d f / d x_axis at cell centres from the 8 corner nodes of each cell.

    f: (..., nz+1, ny, nx) node field -> (..., nz, ny, nx) cell field.
    Average of the four edge differences parallel to `axis_dir` (0=x,1=y,2=z).
    """
    nz = f.shape[-3] - 1

    def corner(bz, by, bx):
        w = f[..., bz: bz + nz, :, :]
        if by:
            w = np.roll(w, -1, axis=-2)
        if bx:
            w = np.roll(w, -1, axis=-1)
        return w

    acc = 0.0
    for b1 in (0, 1):
        for b2 in (0, 1):
            if axis_dir == 0:
                acc = acc + corner(b2, b1, 1) - corner(b2, b1, 0)
            elif axis_dir == 1:
                acc = acc + corner(b2, 1, b1) - corner(b2, 0, b1)
            else:
                acc = acc + corner(1, b2, b1) - corner(0, b2, b1)
    return acc / (4.0 * h)


def grad_cell(v: np.ndarray, h: float) -> np.ndarray:
    """Velocity gradient L[a, b] = d v_a / d x_b at cells: (3, 3, nz, ny, nx)."""
    return np.stack([np.stack([_cell_diff(v[a], b, h) for b in range(3)]) for a in range(3)])


def _node_diff(g: np.ndarray, axis_dir: int, h: float) -> np.ndarray:
    """d g / d x_axis at interior nodes from the 8 cells around each node.

    The staggered formula shifted by half a cell: the node (i, j, k) is the
    centre of the cube of cells (i-1..i, j-1..j, k-1..k).
    g: (..., nz, ny, nx) -> (..., nz-1, ny, nx) for nodes k = 1..nz-1.
    """
    nz = g.shape[-3]

    def cell(bz, by, bx):
        # cell (i - bx, j - by, k - bz) for node (i, j, k), k = 1..nz-1
        w = g[..., 1 - bz: nz - bz, :, :]
        if by:
            w = np.roll(w, 1, axis=-2)
        if bx:
            w = np.roll(w, 1, axis=-1)
        return w

    acc = 0.0
    for b1 in (0, 1):
        for b2 in (0, 1):
            if axis_dir == 0:
                acc = acc + cell(b2, b1, 0) - cell(b2, b1, 1)
            elif axis_dir == 1:
                acc = acc + cell(b2, 0, b1) - cell(b2, 1, b1)
            else:
                acc = acc + cell(0, b2, b1) - cell(1, b2, b1)
    return acc / (4.0 * h)


def voigt_to_full(s: np.ndarray) -> np.ndarray:
    """(6, ...) Voigt -> (3, 3, ...) symmetric tensor."""
    t = np.empty((3, 3) + s.shape[1:], dtype=s.dtype)
    for n, (a, b) in enumerate(VOIGT):
        t[a, b] = s[n]
        t[b, a] = s[n]
    return t


def full_to_voigt(t: np.ndarray) -> np.ndarray:
    return np.stack([t[a, b] for a, b in VOIGT])


def div_node(sig: np.ndarray, h: float) -> np.ndarray:
    """(D_h sigma)_a = sum_b d_b sigma_ab at interior nodes; walls zero.

    sig: Voigt cell tensor (6, nz, ny, nx) -> node vector (3, nz+1, ny, nx).
    """
    nz, ny, nx = sig.shape[1:]
    t = voigt_to_full(sig)
    out = np.zeros((3, nz + 1, ny, nx), dtype=sig.dtype)
    for a in range(3):
        out[a, 1:nz] = sum(_node_diff(t[a, b], b, h) for b in range(3))
    return out


def sym(L: np.ndarray) -> np.ndarray:
    return 0.5 * (L + np.swapaxes(L, 0, 1))


def stiffness(D: np.ndarray, lam: float, mu: float) -> np.ndarray:
    """C : D = lam tr(D) I + 2 mu D for a symmetric tensor field (3, 3, ...)."""
    tr = D[0, 0] + D[1, 1] + D[2, 2]
    out = 2.0 * mu * D
    for a in range(3):
        out[a, a] = out[a, a] + lam * tr
    return out
