"""Pins of the oracle multigrid (paper Sec. 3.6) against invariants and direct solves."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.multigrid import (DEFAULT_ORDER, Level, MGOracle, assemble_from_stencil,
                              direct_solve, fine_stencil, galerkin_stencil,
                              prolong, prolongation_matrix, restrict)
from oracle.operators import apply_elastic, assemble_elastic, div_node, interior_mask
from workloads import lame, manufactured_source, manufactured_velocity, stress_field

LAM, MU = lame()


def _rand_interior(rng, nx, ny, nz):
    x = np.zeros((3, nz + 1, ny, nx))
    x[:, 1:nz] = rng.standard_normal((3, nz - 1, ny, nx))
    return x


def test_restriction_is_transpose_of_prolongation():
    """R = T^T (Sec. 3.6), matrix-free transfers equal the assembled T."""
    rng = np.random.default_rng(0)
    for (nxc, nyc, nzc) in [(4, 4, 4), (3, 5, 2), (2, 4, 3)]:
        ec = _rand_interior(rng, nxc, nyc, nzc)
        r = _rand_interior(rng, 2 * nxc, 2 * nyc, 2 * nzc)
        T = prolongation_matrix(nxc, nyc, nzc)
        assert np.abs(T @ ec.ravel() - prolong(ec).ravel()).max() < 1e-15
        assert np.abs(T.T @ r.ravel() - restrict(r).ravel()).max() < 1e-14
        assert abs(np.sum(restrict(r) * ec) - np.sum(r * prolong(ec))) < 1e-12


def test_prolongation_reproduces_trilinear():
    """T maps a coarse field that is linear in z (zero on the walls) and
    a constant-in-x,y profile exactly to its fine-grid samples."""
    nzc = 4
    zc = np.arange(nzc + 1) / nzc
    zf = np.arange(2 * nzc + 1) / (2 * nzc)
    prof_c = np.minimum(zc, 1 - zc)  # piecewise linear, kink on a coarse node
    prof_f = np.minimum(zf, 1 - zf)
    ec = np.zeros((3, nzc + 1, 4, 4)) + prof_c[None, :, None, None]
    ef = prolong(ec)
    assert np.abs(ef - prof_f[None, :, None, None]).max() < 1e-15
    # periodic direction: a coarse cosine sampled on even nodes is averaged on odd nodes
    xc = np.arange(4)
    ec = np.zeros((3, 3, 4, 4))
    ec[:, 1] = np.cos(2 * np.pi * xc / 4)[None, None, :]
    ef = prolong(ec)
    mid = ef[:, 2]  # fine plane 2 = coarse plane 1; shape (3, 8, 8)
    cx = np.cos(2 * np.pi * xc / 4)
    assert np.abs(mid[..., 0::2] - cx).max() < 1e-15
    assert np.abs(mid[..., 1::2] - 0.5 * (cx + np.roll(cx, -1))).max() < 1e-15


@pytest.mark.parametrize("nz", [8, 16])
def test_galerkin_two_ways(nz):
    """Per-plane Galerkin stencils (reduced-grid RAP) equal T^T K T on the full grid."""
    n = nz
    h = 1.0 / nz
    A0 = fine_stencil(nz, h, LAM, MU)
    Ac = galerkin_stencil(A0, nz)
    K = assemble_elastic(n, n, nz, h, LAM, MU)
    fm = interior_mask(n, n, nz)
    cm = interior_mask(n // 2, n // 2, nz // 2)
    T = prolongation_matrix(n // 2, n // 2, nz // 2)
    direct = (T[fm][:, cm].T @ K[fm][:, fm] @ T[fm][:, cm]).toarray()
    via_stencil = assemble_from_stencil(Ac, n // 2, n // 2, nz // 2)[cm][:, cm].toarray()
    assert np.abs(direct - via_stencil).max() <= 1e-13 * np.abs(direct).max()
    assert np.abs(direct - direct.T).max() <= 1e-13 * np.abs(direct).max()
    # 27-point support with all offsets present away from the walls (Sec. 3.6)
    k = nz // 4
    assert np.count_nonzero(np.abs(Ac[k]).sum(axis=(-1, -2))) == 27
    # centre blocks are diagonal (reflection symmetry x -> -x, y -> -y)
    cb = Ac[1:nz // 2, 1, 1, 1]
    assert np.abs(cb - np.einsum("kcc->kc", cb)[:, :, None] * np.eye(3)).max() < 1e-12 * np.abs(cb).max()


@pytest.mark.parametrize("n,mc", [((32, 32, 32), 2), ((48, 40, 32), 4)])
def test_galerkin_cross_couplings_vanish_on_zero_offsets(n, mc):
    """On every level, an entry coupling component c to component d != c is
    zero (to rounding) wherever the offset along c or along d is zero.  The
    fine operator's cross-component part is (lam+mu) times the product of the
    central first differences along c and along d, each antisymmetric (also
    restricted to the interior planes); the transfers are tensor products, and
    a Galerkin product B^T D B of an antisymmetric factor is antisymmetric, so
    its zero offset vanishes on every level.  The coarse-level kernels leave
    these entries out.  (A one-sided mixed difference in the fine operator
    fails this test.)"""
    nx, ny, nz = n
    o = MGOracle(nx, ny, nz, 1.0 / nz, LAM, MU, min_coarse_nz=mc)
    assert len(o.levels) >= 4
    for L in o.levels:
        A = L.A
        big = np.abs(A).max()
        worst = 0.0
        for oz in range(3):
            for oy in range(3):
                for ox in range(3):
                    off = (ox - 1, oy - 1, oz - 1)
                    for c in range(3):
                        for d in range(3):
                            if c != d and (off[c] == 0 or off[d] == 0):
                                worst = max(worst, np.abs(A[:, oz, oy, ox, c, d]).max())
        assert worst <= 1e-14 * big, (L.nx, L.ny, L.nz, worst / big)
        # and the cross couplings kept are not all zero on the coarse levels
        # (corner offsets, on planes whose neighbours are interior; the fine
        # operator has no corner couplings)
        if L is not o.levels[0] and L.nz >= 4:
            assert np.abs(A[2:L.nz - 1, 2, 2, 2, 0, 1]).max() > 1e-6 * big


def test_colour_pass_zeroes_colour_residual():
    """After updating colour c, the residual vanishes at every node of colour c."""
    rng = np.random.default_rng(5)
    nx, ny, nz = 8, 12, 8
    h = 1.0 / nz
    mg = MGOracle(nx, ny, nz, h, LAM, MU, min_coarse_nz=2)
    for lvl in (0, 1):
        L = mg.levels[lvl]
        x = rng.standard_normal(L.shape)
        if lvl > 0:
            x[:, 0] = 0
            x[:, -1] = 0
        b = rng.standard_normal(L.shape)
        for col in DEFAULT_ORDER:
            L.colour_pass(x, b, col)
            r = b - L.apply(x)
            a, bb, e = col
            ks = [k for k in range(1, L.nz) if k % 2 == e]
            sel = r[:, ks][:, :, bb::2][:, :, :, a::2]
            assert np.abs(sel).max() <= 1e-12 * np.abs(b).max()


@pytest.mark.parametrize("n,levels", [(4, 2), (8, 3)])
def test_mg_matches_dense_solve(n, levels):
    """Brute force on tiny grids: converged MG == dense numpy.linalg.solve."""
    rng = np.random.default_rng(6)
    h = 1.0 / n
    mg = MGOracle(n, n, n, h, LAM, MU, min_coarse_nz=2)
    assert len(mg.levels) == levels
    b = _rand_interior(rng, n, n, n)
    x0 = np.zeros_like(b)
    x0[:, 0] = rng.standard_normal((3, n, n))
    x0[:, n] = rng.standard_normal((3, n, n))
    x, info = mg.solve(b, x0, rtol=1e-14, max_cycles=200)
    assert info["converged"]
    K = assemble_elastic(n, n, n, h, LAM, MU)
    m = interior_mask(n, n, n)
    xw = x0.copy()
    xw[:, 1:n] = 0
    rhs = (b - apply_elastic(xw, h, LAM, MU))[:, 1:n].ravel()
    xd = np.linalg.solve(K[m][:, m].toarray(), rhs)
    assert np.abs(x[:, 1:n].ravel() - xd).max() <= 1e-12 * np.abs(xd).max()
    assert np.array_equal(x[:, 0], x0[:, 0]) and np.array_equal(x[:, n], x0[:, n])


def test_mg_matches_sparse_direct_12():
    n = 12
    h = 1.0 / n
    mg = MGOracle(n, n, n, h, LAM, MU)
    b = div_node(stress_field(n, n, n, 0), h)
    x, info = mg.solve(b, np.zeros_like(b), rtol=1e-14)
    xd = direct_solve(b, np.zeros_like(b), h, LAM, MU)
    assert np.abs(x - xd).max() <= 1e-12 * np.abs(xd).max()


def test_vcycle_is_symmetric():
    """Post-smoothing in reverse colour order makes the V-cycle a symmetric operator."""
    n = 4
    mg = MGOracle(n, n, n, 1.0 / n, LAM, MU, min_coarse_nz=2)
    m = 3 * (n - 1) * n * n
    M = np.zeros((m, m))
    for q in range(m):
        b = np.zeros((3, n + 1, n, n))
        b[:, 1:n].reshape(-1)[q] = 1.0
        x = np.zeros_like(b)
        mg.vcycle(x, b)
        M[:, q] = x[:, 1:n].ravel()
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()


def test_contraction_band_and_rhs_zero():
    n = 16
    mg = MGOracle(n, n, n, 1.0 / n, LAM, MU)
    b = div_node(stress_field(n, n, n, 0), 1.0 / n)
    x, info = mg.solve(b, np.zeros_like(b), rtol=1e-10)
    rates = np.array(info["hist"][1:]) / np.array(info["hist"][:-1])
    assert info["converged"] and 10 <= info["cycles"] <= 30
    assert 0.1 < rates[-1] < 0.4
    # zero lifted right-hand side (zero b, zero walls): x = 0 with no cycle
    x0 = np.ones_like(b)
    x0[:, 0] = 0.0
    x0[:, n] = 0.0
    x, info = mg.solve(np.zeros_like(b), x0, rtol=1e-10)
    assert info["cycles"] == 0 and np.abs(x).max() == 0.0


def test_manufactured_second_order():
    """Discrete solution error against the exact field decays as h^2 (Sec. 3.4)."""
    errs = []
    for n in (8, 16, 32):
        h = 1.0 / n
        mg = MGOracle(n, n, n, h, LAM, MU, min_coarse_nz=2 if n == 8 else 8)
        f = manufactured_source(n, n, n, LAM, MU)
        x, info = mg.solve(f, np.zeros_like(f), rtol=1e-12)
        u = manufactured_velocity(n, n, n)
        errs.append(np.linalg.norm(x - u) / np.linalg.norm(u))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8) and orders[-1] < 2.2, (errs, orders)


@pytest.mark.parametrize("shape,levels", [((16, 16, 8), 3), ((12, 8, 4), 2), ((20, 12, 8), 3)])
def test_mg_matches_sparse_direct_on_flat_grids(shape, levels):
    """The paper's N x N x N/2 and slenderer sample shapes (Secs. 4 and 5) and
    a ragged one: converged multigrid equals a sparse direct solve, with
    nonzero wall data."""
    nx, ny, nz = shape
    rng = np.random.default_rng(31)
    h = 1.0 / nz
    mg = MGOracle(nx, ny, nz, h, LAM, MU, min_coarse_nz=2)
    assert len(mg.levels) == levels
    b = _rand_interior(rng, nx, ny, nz)
    x0 = np.zeros_like(b)
    x0[:, 0] = rng.standard_normal((3, ny, nx))
    x0[:, nz] = rng.standard_normal((3, ny, nx))
    x, info = mg.solve(b, x0, rtol=1e-14, max_cycles=200)
    assert info["converged"]
    xd = direct_solve(b, x0, h, LAM, MU)
    assert np.abs(x - xd).max() <= 1e-11 * np.abs(xd).max()


@pytest.mark.parametrize("lvl", [0, 1])
def test_sweep_at_nodes_matches_the_oracle_sweep(lvl):
    """The node-by-node evaluation of one sweep (which checks the GPU sweep at
    full size on sampled nodes) reproduces the oracle's colour-major sweep at
    every interior node of a fine and a Galerkin level, and notices a sweep
    run in another colour order and a single wrong node."""
    from sweep_sample import sweep_at_nodes
    rng = np.random.default_rng(21)
    mg = MGOracle(16, 12, 8, 1.0 / 8, LAM, MU, min_coarse_nz=2)
    L = mg.levels[lvl]
    x = rng.standard_normal(L.shape)
    b = rng.standard_normal(L.shape)
    xn = x.copy()
    L.sweep(xn, b, DEFAULT_ORDER)
    nodes = [(k, j, i) for k in range(1, L.nz) for j in range(L.ny) for i in range(L.nx)]
    got = sweep_at_nodes(L.A, x, xn, b, nodes, DEFAULT_ORDER)
    want = np.array([xn[:, k, j, i] for (k, j, i) in nodes])
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    # a sweep in the ascending colour order is not the default sweep
    xa = x.copy()
    L.sweep(xa, b, [(c & 1, (c >> 1) & 1, (c >> 2) & 1) for c in range(8)])
    got = sweep_at_nodes(L.A, x, xa, b, nodes, DEFAULT_ORDER)
    want = np.array([xa[:, k, j, i] for (k, j, i) in nodes])
    assert np.abs(got - want).max() > 1e-3 * np.abs(want).max()
    # one wrong new value (colour 0, the first visited) shows at that node
    # and at every neighbour coupled to it, all of later colours: on the fine
    # level a y component reaches the 6 face and the 8 xy and yz edge
    # neighbours, on a Galerkin level all 26
    xw = xn.copy()
    xw[1, 2, 4, 6] += 1e-6
    got = sweep_at_nodes(L.A, x, xw, b, nodes, DEFAULT_ORDER)
    want = np.array([xw[:, k, j, i] for (k, j, i) in nodes])
    bad = {nodes[t] for t in np.flatnonzero(np.abs(got - want).max(axis=1) > 1e-12)}
    assert (2, 4, 6) in bad and len(bad) == 1 + (14 if lvl == 0 else 26)
