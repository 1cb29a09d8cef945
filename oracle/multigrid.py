"""Geometric multigrid for the projection system (paper Sec. 3.6).

Follows the paper's description:
  * hierarchy G_0 ... G_g, each level halving every dimension;
  * T_k : G_k -> G_{k-1} by (tri)linear interpolation, R_{k-1} = T_k^T;
  * coarse operators by recursive products A_k = R_{k-1} A_{k-1} T_k;
  * V-cycle with two pre- and two post-smoothing Gauss-Seidel steps, the
    unknowns being 3-vectors and the matrix entries 3x3 blocks coupling each
    node to its 3x3x3 neighbourhood.

Choices where the paper is silent (each listed in the design notes):
  * coarse node K <-> fine node 2K, walls map to walls (even dimensions);
  * smoothing is block Gauss-Seidel in a multicolour order: the colour of
    node (i, j, k) is its parity triple (i&1, j&1, k&1); a sweep visits the
    8 colours in a given order (pre-smoothing) or the reverse order
    (post-smoothing), updating all nodes of one colour together; nodes of one
    colour are never coupled by a 3x3x3 stencil, so this is plain Gauss-Seidel
    in a colour-major node order;
  * coarsening stops when nz <= min_coarse_nz; the coarsest system is solved
    with a dense FP64 Cholesky factorisation;
  * the cycle repeats until ||b_eff - K x|| <= rtol ||b_eff|| (2-norm over the
    interior unknowns, b_eff = b - K_IB x_B), checked before every cycle.

A level operator is stored as per-plane stencils A[k, oz+1, oy+1, ox+1, c, d]:
the 3x3 block coupling component c of node (i, j, k) to component d of node
(i+ox, j+oy, k+oz).  Every level is invariant under x/y translation (the
stiffness is homogeneous), so one stencil per z-plane describes it exactly;
planes near the walls differ.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .operators import apply_elastic, assemble_elastic, interior_mask, node_index

OFFSETS = [o for o in itertools.product((-1, 0, 1), repeat=3)]  # (oz, oy, ox)


def colour_parities(c: int):
    """(i, j, k) parities of colour c = (i&1) + 2(j&1) + 4(k&1)."""
    return (c & 1, (c >> 1) & 1, (c >> 2) & 1)


ASCENDING_ORDER = [colour_parities(c) for c in range(8)]
# Even rows first (their four colours: even then odd planes, even then odd
# columns), then odd rows; the default sweep order.
ROW_ORDER = [colour_parities(c) for c in (0, 1, 4, 5, 2, 3, 6, 7)]
DEFAULT_ORDER = ROW_ORDER


class ShapeError(ValueError):
    pass


# ---------------------------------------------------------------------------
# Stencils <-> sparse matrices
# ---------------------------------------------------------------------------

def _wrap(d: int, n: int) -> int:
    return d if d <= n // 2 else d - n


def stencil_from_matrix(M: sp.spmatrix, nx: int, ny: int, nz: int) -> np.ndarray:
    """Per-plane 27-point block stencil read off the rows of node (0, 0, k).

    M has the full node indexing of an (nx, ny, nz) grid; nx, ny >= 4 so that
    offsets -1, 0, +1 are told apart.  Raises if a row reaches further.
    """
    assert nx >= 4 and ny >= 4
    M = M.tocsr()
    idx = node_index(nx, ny, nz)
    A = np.zeros((nz + 1, 3, 3, 3, 3, 3))
    for k in range(1, nz):
        for c in range(3):
            row = M.getrow(idx[c, k, 0, 0])
            for col, val in zip(row.indices, row.data):
                d, rem = divmod(col, (nz + 1) * ny * nx)
                kk, rem = divmod(rem, ny * nx)
                jj, ii = divmod(rem, nx)
                oz, oy, ox = kk - k, _wrap(jj, ny), _wrap(ii, nx)
                if max(abs(oz), abs(oy), abs(ox)) > 1:
                    if val != 0.0:
                        raise AssertionError("stencil wider than 3x3x3")
                    continue
                A[k, oz + 1, oy + 1, ox + 1, c, d] += val
    return A


def assemble_from_stencil(A: np.ndarray, nx: int, ny: int, nz: int) -> sp.csr_matrix:
    """Sparse matrix (full node indexing, interior rows) of a per-plane stencil."""
    idx = node_index(nx, ny, nz)
    rows, cols, vals = [], [], []
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    for k in range(1, nz):
        for (oz, oy, ox) in OFFSETS:
            blk = A[k, oz + 1, oy + 1, ox + 1]
            for c in range(3):
                for d in range(3):
                    v = blk[c, d]
                    if v == 0.0:
                        continue
                    r = idx[c, k, J, I].ravel()
                    q = idx[d, k + oz, (J + oy) % ny, (I + ox) % nx].ravel()
                    rows.append(r)
                    cols.append(q)
                    vals.append(np.full(r.shape, v))
    n = 3 * (nz + 1) * ny * nx
    if not rows:
        return sp.csr_matrix((n, n))
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    M.sum_duplicates()
    return M


def prolongation_matrix(nxc: int, nyc: int, nzc: int) -> sp.csr_matrix:
    """T: coarse (nxc, nyc, nzc) -> fine (2nxc, 2nyc, 2nzc), full node indexing.

    Coarse node I sits on fine node 2I.  Each coarse interior node spreads to
    the 27 fine nodes around 2I with weight prod_a (1 if d_a = 0 else 1/2).
    Only interior coarse columns and interior fine rows are populated: the
    coarse correction vanishes on the walls.
    """
    nxf, nyf, nzf = 2 * nxc, 2 * nyc, 2 * nzc
    cidx = node_index(nxc, nyc, nzc)
    fidx = node_index(nxf, nyf, nzf)
    K, J, I = np.meshgrid(np.arange(1, nzc), np.arange(nyc), np.arange(nxc), indexing="ij")
    rows, cols, vals = [], [], []
    for (dz, dy, dx) in OFFSETS:
        w = 1.0
        for dd in (dz, dy, dx):
            w *= 1.0 if dd == 0 else 0.5
        for c in range(3):
            cols.append(cidx[c, K, J, I].ravel())
            rows.append(fidx[c, 2 * K + dz, (2 * J + dy) % nyf, (2 * I + dx) % nxf].ravel())
            vals.append(np.full(K.size, w))
    T = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(fidx.size, cidx.size)).tocsr()
    T.sum_duplicates()
    return T


def fine_stencil(nz: int, h: float, lam: float, mu: float) -> np.ndarray:
    """Per-plane stencil of the fine operator (wall couplings included)."""
    M = assemble_elastic(8, 8, nz, h, lam, mu)
    return stencil_from_matrix(M, 8, 8, nz)


def galerkin_stencil(A_f: np.ndarray, nz_f: int) -> np.ndarray:
    """A_c = T^T A_f T on the interior unknowns, as per-plane coarse stencils.

    Computed by sparse products on a reduced periodic grid (16 x 16 fine,
    8 x 8 coarse) with the full z extent; the stencils are translation
    invariant in x and y, so they hold for any nx, ny.
    """
    nzc = nz_f // 2
    Kf = assemble_from_stencil(A_f, 16, 16, nz_f)
    fm = interior_mask(16, 16, nz_f)
    cm = interior_mask(8, 8, nzc)
    T = prolongation_matrix(8, 8, nzc)
    Kf_II = Kf[fm][:, fm]
    T_II = T[fm][:, cm]
    Kc_II = (T_II.T @ Kf_II @ T_II).tocoo()
    n = cm.size
    where = np.flatnonzero(cm)
    Kc = sp.coo_matrix((Kc_II.data, (where[Kc_II.row], where[Kc_II.col])), shape=(n, n))
    return stencil_from_matrix(Kc, 8, 8, nzc)


# ---------------------------------------------------------------------------
# Matrix-free transfers (same T as `prolongation_matrix`)
# ---------------------------------------------------------------------------

def _interp_periodic(a: np.ndarray, axis: int) -> np.ndarray:
    n = a.shape[axis]
    shape = list(a.shape)
    shape[axis] = 2 * n
    out = np.empty(shape, dtype=a.dtype)
    sl_even = [slice(None)] * a.ndim
    sl_odd = [slice(None)] * a.ndim
    sl_even[axis] = slice(0, None, 2)
    sl_odd[axis] = slice(1, None, 2)
    out[tuple(sl_even)] = a
    out[tuple(sl_odd)] = 0.5 * (a + np.roll(a, -1, axis=axis))
    return out


def _interp_z(a: np.ndarray) -> np.ndarray:
    nzc = a.shape[-3] - 1
    out = np.empty(a.shape[:-3] + (2 * nzc + 1,) + a.shape[-2:], dtype=a.dtype)
    out[..., 0::2, :, :] = a
    out[..., 1::2, :, :] = 0.5 * (a[..., :-1, :, :] + a[..., 1:, :, :])
    return out


def prolong(ec: np.ndarray) -> np.ndarray:
    """T e_c for a coarse node vector whose wall planes are zero."""
    return _interp_z(_interp_periodic(_interp_periodic(ec, -1), -2))


def _restrict_periodic(r: np.ndarray, axis: int) -> np.ndarray:
    sl_even = [slice(None)] * r.ndim
    sl_odd = [slice(None)] * r.ndim
    sl_even[axis] = slice(0, None, 2)
    sl_odd[axis] = slice(1, None, 2)
    odd = r[tuple(sl_odd)]
    return r[tuple(sl_even)] + 0.5 * (odd + np.roll(odd, 1, axis=axis))


def _restrict_z(r: np.ndarray) -> np.ndarray:
    nzf = r.shape[-3] - 1
    nzc = nzf // 2
    out = np.zeros(r.shape[:-3] + (nzc + 1,) + r.shape[-2:], dtype=r.dtype)
    out[..., 1:nzc, :, :] = (r[..., 2:nzf - 1:2, :, :]
                             + 0.5 * (r[..., 3:nzf:2, :, :] + r[..., 1:nzf - 2:2, :, :]))
    return out


def restrict(r: np.ndarray) -> np.ndarray:
    """T^T r for a fine node vector (its wall planes are ignored)."""
    r = r.copy()
    r[:, 0] = 0.0
    r[:, -1] = 0.0
    return _restrict_periodic(_restrict_periodic(_restrict_z(r), -2), -1)


# ---------------------------------------------------------------------------
# Hierarchy, smoother, V-cycle, solve
# ---------------------------------------------------------------------------

class Level:
    def __init__(self, nx: int, ny: int, nz: int, A: np.ndarray):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.A = A
        self.Dinv = np.zeros((nz + 1, 3, 3))
        for k in range(1, nz):
            self.Dinv[k] = np.linalg.inv(A[k, 1, 1, 1])

    @property
    def shape(self):
        return (3, self.nz + 1, self.ny, self.nx)

    def apply(self, x: np.ndarray) -> np.ndarray:
        """A x at interior nodes (walls of x used as given; result walls 0)."""
        nz = self.nz
        out = np.zeros_like(x)
        for (oz, oy, ox) in OFFSETS:
            blk = self.A[1:nz, oz + 1, oy + 1, ox + 1]
            if not blk.any():
                continue
            sh = x[:, 1 + oz: nz + oz]
            if oy:
                sh = np.roll(sh, -oy, axis=-2)
            if ox:
                sh = np.roll(sh, -ox, axis=-1)
            for c in range(3):
                for d in range(3):
                    col = blk[:, c, d]
                    if col.any():
                        out[c, 1:nz] += col[:, None, None] * sh[d]
        return out

    def colour_pass(self, x: np.ndarray, b: np.ndarray, colour) -> None:
        """Block Gauss-Seidel update of every node of one colour, in place."""
        a, bb, e = colour
        nx, ny, nz = self.nx, self.ny, self.nz
        ks = np.arange(1, nz)
        ks = ks[ks % 2 == e]
        if ks.size == 0:
            return
        js = np.arange(bb, ny, 2)
        is_ = np.arange(a, nx, 2)
        comps = np.arange(3)
        acc = b[np.ix_(comps, ks, js, is_)].copy()
        for (oz, oy, ox) in OFFSETS:
            if (oz, oy, ox) == (0, 0, 0):
                continue
            blk = self.A[ks, oz + 1, oy + 1, ox + 1]
            if not blk.any():
                continue
            nb = x[np.ix_(comps, ks + oz, (js + oy) % ny, (is_ + ox) % nx)]
            for c in range(3):
                for d in range(3):
                    col = blk[:, c, d]
                    if col.any():
                        acc[c] -= col[:, None, None] * nb[d]
        x[np.ix_(comps, ks, js, is_)] = np.einsum("kcd,dkji->ckji", self.Dinv[ks], acc)

    def sweep(self, x, b, order) -> None:
        for col in order:
            self.colour_pass(x, b, col)


class MGOracle:
    """Multigrid solver for K x = b (Eq. proj) with Dirichlet walls in x."""

    def __init__(self, nx: int, ny: int, nz: int, h: float, lam: float, mu: float,
                 min_coarse_nz: int = 8, n_pre: int = 2, n_post: int = 2, order=None):
        self.h, self.lam, self.mu = h, lam, mu
        self.n_pre, self.n_post = n_pre, n_post
        self.order = list(order) if order is not None else list(DEFAULT_ORDER)
        if sorted(self.order) != sorted(ASCENDING_ORDER):
            raise ValueError("order must be a permutation of the 8 parity colours")
        if min(nx, ny, nz) < 2:
            raise ShapeError("grid too small")
        A = fine_stencil(nz, h, lam, mu)
        self.levels = [Level(nx, ny, nz, A)]
        while nz > min_coarse_nz:
            if nx % 2 or ny % 2 or nz % 2:
                raise ShapeError("dimensions must be even at every coarsened level")
            if nx < 4 or ny < 4 or nz < 4:
                raise ShapeError("coarse grid would have fewer than 2 cells per dimension")
            A = galerkin_stencil(A, nz)
            nx, ny, nz = nx // 2, ny // 2, nz // 2
            self.levels.append(Level(nx, ny, nz, A))
        L = self.levels[-1]
        M = assemble_from_stencil(L.A, L.nx, L.ny, L.nz)
        m = interior_mask(L.nx, L.ny, L.nz)
        self.coarse_matrix = M[m][:, m].toarray()
        self.coarse_chol = sla.cho_factor(self.coarse_matrix)

    # -- pieces ------------------------------------------------------------
    def apply(self, x: np.ndarray, level: int = 0) -> np.ndarray:
        return self.levels[level].apply(x)

    def residual(self, x: np.ndarray, b: np.ndarray, level: int = 0) -> np.ndarray:
        r = b - self.levels[level].apply(x)
        r[:, 0] = 0.0
        r[:, -1] = 0.0
        return r

    def coarse_solve(self, x: np.ndarray, b: np.ndarray) -> None:
        L = self.levels[-1]
        xw = x.copy()
        xw[:, 1:L.nz] = 0.0
        rhs = (b - L.apply(xw))[:, 1:L.nz].ravel()
        x[:, 1:L.nz] = sla.cho_solve(self.coarse_chol, rhs).reshape(3, L.nz - 1, L.ny, L.nx)

    def vcycle(self, x: np.ndarray, b: np.ndarray, level: int = 0) -> None:
        if level == len(self.levels) - 1:
            self.coarse_solve(x, b)
            return
        L = self.levels[level]
        for _ in range(self.n_pre):
            L.sweep(x, b, self.order)
        bc = restrict(self.residual(x, b, level))
        ec = np.zeros(self.levels[level + 1].shape)
        self.vcycle(ec, bc, level + 1)
        x += prolong(ec)
        for _ in range(self.n_post):
            L.sweep(x, b, self.order[::-1])

    # -- solve -------------------------------------------------------------
    def lifted_rhs_norm(self, b: np.ndarray, x: np.ndarray) -> float:
        xw = x.copy()
        xw[:, 1:-1] = 0.0
        return float(np.linalg.norm(self.residual(xw, b)[:, 1:-1]))

    def solve(self, b: np.ndarray, x0: np.ndarray, rtol: float = 1e-10, max_cycles: int = 100):
        """Repeat V-cycles from x0 until the relative residual is <= rtol.

        rtol <= 0 runs exactly max_cycles cycles.  Returns (x, info).
        """
        x = np.array(x0, dtype=np.float64, copy=True)
        nb = self.lifted_rhs_norm(b, x)
        if nb == 0.0:
            x[:, 1:-1] = 0.0
            return x, dict(cycles=0, rel_res=0.0, hist=[0.0], converged=True)
        rel = float(np.linalg.norm(self.residual(x, b)[:, 1:-1])) / nb
        hist = [rel]
        cycles = 0
        while cycles < max_cycles and (rtol <= 0 or rel > rtol):
            self.vcycle(x, b)
            cycles += 1
            rel = float(np.linalg.norm(self.residual(x, b)[:, 1:-1])) / nb
            hist.append(rel)
        return x, dict(cycles=cycles, rel_res=rel, hist=hist,
                       converged=(rtol <= 0) or rel <= rtol)


def direct_solve(b: np.ndarray, x0: np.ndarray, h: float, lam: float, mu: float) -> np.ndarray:
    """Exact discrete solution by a sparse direct solve of K_II x_I = b - K_IB x_B."""
    import scipy.sparse.linalg as spla
    _, nz1, ny, nx = b.shape
    nz = nz1 - 1
    K = assemble_elastic(nx, ny, nz, h, lam, mu)
    m = interior_mask(nx, ny, nz)
    xw = np.array(x0, dtype=np.float64, copy=True)
    xw[:, 1:nz] = 0.0
    rhs = (b - apply_elastic(xw, h, lam, mu))[:, 1:nz].ravel()
    x = xw.copy()
    x[:, 1:nz] = spla.spsolve(K[m][:, m].tocsc(), rhs).reshape(3, nz - 1, ny, nx)
    return x
