"""GPU parity of the multigrid path (libqsmg through its C ABI) against the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.multigrid import MGOracle, direct_solve
from oracle.operators import apply_elastic, div_node
from workloads import lame, stress_field

pytestmark = pytest.mark.gpu
LAM, MU = lame()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


ROW = (0, 1, 4, 5, 2, 3, 6, 7)


def make(nx, ny, nz, **kw):
    from paper_1904_03808_amd.qsmg import MGSolver
    h = 1.0 / nz
    kw.setdefault("colour_order", ROW)
    return MGSolver(nx, ny, nz, h, LAM, MU, **kw), MGOracle(nx, ny, nz, h, LAM, MU,
                                                           min_coarse_nz=kw.get("min_coarse_nz", 8),
                                                           order=[(c & 1, (c >> 1) & 1, (c >> 2) & 1)
                                                                  for c in kw["colour_order"]])


def rand_node(rng, nx, ny, nz, walls=True):
    x = rng.standard_normal((3, nz + 1, ny, nx))
    if not walls:
        x[:, 0] = 0
        x[:, -1] = 0
    return x


GRIDS = [(32, 32, 32), (40, 24, 32)]


@pytest.mark.parametrize("n", GRIDS)
def test_stencils_match_oracle(n):
    """Host Galerkin by stencil composition == oracle Galerkin by sparse RAP."""
    g, o = make(*n)
    assert g.levels == len(o.levels)
    for lvl, L in enumerate(o.levels):
        S = g.level_stencil(lvl)
        assert rel(S[1:-1], L.A[1:-1]) < 1e-13, lvl


@pytest.mark.parametrize("n", GRIDS)
def test_apply(n):
    rng = np.random.default_rng(1)
    g, o = make(*n)
    x = rand_node(rng, *n)
    y = host(g.apply(dev(x)))
    ref = apply_elastic(x, 1.0 / n[2], LAM, MU)
    assert rel(y, ref) < 1e-13
    assert np.all(y[:, 0] == 0) and np.all(y[:, -1] == 0)


@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("level", [0, 1])
def test_colour_passes(n, level):
    rng = np.random.default_rng(2)
    g, o = make(*n)
    L = o.levels[level]
    x = rand_node(rng, L.nx, L.ny, L.nz, walls=(level == 0))
    b = rand_node(rng, L.nx, L.ny, L.nz)
    xd, bd = dev(x), dev(b)
    for c in [0, 5, 2, 7, 1, 6, 3, 4]:
        g.level_colour_pass(level, xd, bd, c)
        L.colour_pass(x, b, (c & 1, (c >> 1) & 1, (c >> 2) & 1))
        assert rel(host(xd), x) < 1e-13, c


def test_colour_passes_wide_coarse_level():
    """A coarse level wider than a wavefront's colour row (80 x 12 x 8): colour
    passes match the oracle colour by colour, and whole V-cycles on this
    hierarchy match the oracle's iterates."""
    rng = np.random.default_rng(11)
    n = (160, 24, 16)
    g, o = make(*n, min_coarse_nz=4)
    L = o.levels[1]
    assert (L.nx, L.ny, L.nz) == (80, 12, 8)
    x = rand_node(rng, L.nx, L.ny, L.nz, walls=False)
    b = rand_node(rng, L.nx, L.ny, L.nz)
    xd, bd = dev(x), dev(b)
    for c in [3, 0, 6, 5, 1, 7, 2, 4]:
        g.level_colour_pass(1, xd, bd, c)
        L.colour_pass(x, b, (c & 1, (c >> 1) & 1, (c >> 2) & 1))
        assert rel(host(xd), x) < 1e-13, c
    bf = rand_node(rng, *n)
    x0 = rand_node(rng, *n)
    for k in (1, 3):
        xd = dev(x0)
        g.solve(dev(bf), xd, rtol=0.0, max_cycles=k)
        x_ref, _ = o.solve(bf, x0, rtol=0.0, max_cycles=k)
        assert rel(host(xd), x_ref) < 1e-12, k


@pytest.mark.parametrize("n", GRIDS)
def test_residual_restrict_prolong(n):
    rng = np.random.default_rng(3)
    g, o = make(*n)
    for level in range(g.levels - 1):
        L, Lc = o.levels[level], o.levels[level + 1]
        x = rand_node(rng, L.nx, L.ny, L.nz, walls=(level == 0))
        b = rand_node(rng, L.nx, L.ny, L.nz)
        r = host(g.level_residual(level, dev(x), dev(b)))
        r_ref = o.residual(x, b, level)
        assert rel(r[:, 1:-1], r_ref[:, 1:-1]) < 1e-13
        from oracle.multigrid import prolong, restrict
        bc = host(g.level_restrict(level, dev(r_ref)))
        assert rel(bc[:, 1:-1], restrict(r_ref)[:, 1:-1]) < 1e-14
        ec = rand_node(rng, Lc.nx, Lc.ny, Lc.nz, walls=False)
        xd = dev(x)
        g.level_prolong_add(level, xd, dev(ec))
        assert rel(host(xd), x + prolong(ec)) < 1e-14


@pytest.mark.parametrize("n", GRIDS)
def test_coarse_solve(n):
    rng = np.random.default_rng(4)
    g, o = make(*n)
    L = o.levels[-1]
    b = rand_node(rng, L.nx, L.ny, L.nz)
    x = np.zeros_like(b)
    xd = dev(x)
    g.coarse_solve(xd, dev(b))
    o.coarse_solve(x, b)
    assert rel(host(xd), x) < 1e-12


@pytest.mark.parametrize("n", GRIDS + [(64, 64, 64)])
def test_vcycle_iterates(n):
    """GPU iterates after each of the first 5 V-cycles match the oracle's (<= 1e-12);
    64^3 runs four levels, with colour pairs on 32^3 and 16^3."""
    rng = np.random.default_rng(5)
    g, o = make(*n)
    b = rand_node(rng, *n)
    x0 = rand_node(rng, *n)
    for k in range(1, 6):
        xd = dev(x0)
        info = g.solve(dev(b), xd, rtol=0.0, max_cycles=k)
        assert info.cycles == k
        x_ref, oi = o.solve(b, x0, rtol=0.0, max_cycles=k)
        assert rel(host(xd), x_ref) < 1e-12, k
        assert abs(info.rel_res - oi["rel_res"]) <= 1e-9 * oi["rel_res"]


def test_solve_config0():
    """32^3, smoothed random stress RHS (seed 0), FP64 V(2,2) to 1e-10."""
    n = 32
    g, o = make(n, n, n)
    b = div_node(stress_field(n, n, n, 0), 1.0 / n)
    xd = dev(np.zeros_like(b))
    info = g.solve(dev(b), xd, rtol=1e-10)
    x_ref, oi = o.solve(b, np.zeros_like(b), rtol=1e-10)
    assert info.cycles == oi["cycles"]
    assert info.rel_res <= 1e-10
    err = np.linalg.norm(host(xd) - x_ref) / np.linalg.norm(x_ref)
    assert err <= 1e-9
    # residual norms near 1e-10 carry rounding of order 1e-16 ||b||
    assert np.allclose(info.hist, oi["hist"], rtol=1e-6, atol=1e-14)


def test_solve_ragged_dirichlet():
    rng = np.random.default_rng(6)
    nx, ny, nz = 40, 24, 32
    g, o = make(nx, ny, nz)
    b = rand_node(rng, nx, ny, nz)
    x0 = np.zeros_like(b)
    x0[:, 0] = rng.standard_normal((3, ny, nx))
    x0[:, -1] = rng.standard_normal((3, ny, nx))
    xd = dev(x0)
    info = g.solve(dev(b), xd, rtol=1e-10)
    xr, _ = o.solve(b, x0, rtol=1e-13)
    assert info.converged
    assert np.linalg.norm(host(xd) - xr) / np.linalg.norm(xr) < 1e-9
    assert np.array_equal(host(xd)[:, 0], x0[:, 0]) and np.array_equal(host(xd)[:, -1], x0[:, -1])


@pytest.mark.parametrize("n", [(32, 32, 32), (48, 48, 48)])
def test_fp32_refinement(n):
    """FP32 V-cycles inside FP64 refinement reach the FP64 residual target and
    the FP64 solution (reference solved to 1e-13)."""
    g, o = make(*n, precision="fp32-ir")
    b = div_node(stress_field(*n, 2), 1.0 / n[2])
    xd = dev(np.zeros_like(b))
    info = g.solve(dev(b), xd, rtol=1e-10)
    assert info.converged and info.rel_res <= 1e-10
    x_ref, _ = o.solve(b, np.zeros_like(b), rtol=1e-13)
    err = np.linalg.norm(host(xd) - x_ref) / np.linalg.norm(x_ref)
    assert err < 1e-8, err
    # contraction per cycle close to the FP64 cycle's
    _, oi = o.solve(b, np.zeros_like(b), rtol=1e-10)
    assert info.cycles <= oi["cycles"] + 2


@pytest.mark.parametrize("n,mc", [((32, 32, 32), 4), ((40, 24, 32), 4), ((16, 16, 64), 16),
                                  ((256, 16, 16), 4), ((512, 16, 16), 4), ((128, 10, 8), 4),
                                  ((8, 8, 16), 8), ((384, 24, 16), 4), ((768, 16, 32), 4)])
@pytest.mark.parametrize("prec", ["fp64", "fp32-ir"])
def test_row_sweep_matches_oracle(n, mc, prec):
    """The row-parity sweep kernel (ping-pong, z-segments, halo recomputation,
    row lengths with and without a specialised kernel (384 and 768 columns
    with one row per workgroup, 768 with 384 threads), last row groups that
    repeat a row: 16 x 16, 128 x 10, and 8 x 8, where one group of 64 rows
    holds the 4 rows of a parity) equals the oracle's colour-by-colour
    Gauss-Seidel sweep on every smoothed level, for 1 and 3 sweeps."""
    rng = np.random.default_rng(10)
    g, o = make(*n, precision=prec, min_coarse_nz=mc)
    dt = torch.float64 if prec == "fp64" else torch.float32
    tol = 1e-13 if prec == "fp64" else 2e-6
    for level in range(g.levels - 1):
        L = o.levels[level]
        x = rand_node(rng, L.nx, L.ny, L.nz, walls=(level == 0))
        b = rand_node(rng, L.nx, L.ny, L.nz)
        for sweeps in (1, 3):
            xd = torch.from_numpy(x).to("cuda", dt)
            bd = torch.from_numpy(b).to("cuda", dt)
            g.smooth(level, xd, bd, sweeps)
            xr = x.astype(np.float32).astype(np.float64) if prec != "fp64" else x.copy()
            br = b.astype(np.float32).astype(np.float64) if prec != "fp64" else b
            for _ in range(sweeps):
                L.sweep(xr, br, o.order)
            assert rel(host(xd).astype(np.float64), xr) < tol, (level, sweeps)


@pytest.mark.parametrize("prec", ["fp64", "fp32-ir"])
def test_rows_beyond_the_row_sweep(prec):
    """Rows of 1024 nodes (1024 x 16 x 16, coarsened to 128 x 2 x 2): too
    long for the fine row sweep's LDS ring, so the fine level is smoothed one
    colour per launch; its 512-wide level 1 is the widest row the two-colour
    launch takes (one row of 256 column pairs per workgroup, the neighbour
    pairs' new values through LDS), and 256 x 4 x 4 below it.  One and three
    sweeps on every smoothed level match the oracle's; the first two FP64
    V-cycles match it element by element, and the FP32-IR solve reaches a
    relative residual of 1e-10 by the oracle's operator (the domain is 64
    units long in x, so its condition number is large and the residual, not
    the distance to another solution, is the bar)."""
    rng = np.random.default_rng(17)
    n = (1024, 16, 16)
    g, o = make(*n, precision=prec, min_coarse_nz=2)
    assert g.levels == len(o.levels) == 4
    assert [g.level_dims(lv) for lv in range(4)] == [(1024, 16, 16), (512, 8, 8), (256, 4, 4),
                                                     (128, 2, 2)]
    dt = torch.float64 if prec == "fp64" else torch.float32
    tol = 1e-13 if prec == "fp64" else 2e-6
    for level in range(3):
        L = o.levels[level]
        x = rand_node(rng, L.nx, L.ny, L.nz, walls=(level == 0))
        b = rand_node(rng, L.nx, L.ny, L.nz)
        for sweeps in (1, 3):
            xd = torch.from_numpy(x).to("cuda", dt)
            g.smooth(level, xd, torch.from_numpy(b).to("cuda", dt), sweeps)
            xr = x.astype(np.float32).astype(np.float64) if prec != "fp64" else x.copy()
            br = b.astype(np.float32).astype(np.float64) if prec != "fp64" else b
            for _ in range(sweeps):
                L.sweep(xr, br, o.order)
            assert rel(host(xd).astype(np.float64), xr) < tol, (level, sweeps)
    b = rand_node(rng, *n)
    x0 = rand_node(rng, *n)
    if prec == "fp64":
        for k in (1, 2):
            xd = dev(x0)
            g.solve(dev(b), xd, rtol=0.0, max_cycles=k)
            x_ref, _ = o.solve(b, x0, rtol=0.0, max_cycles=k)
            assert rel(host(xd), x_ref) < 1e-12, k
    else:
        xd = dev(x0)
        info = g.solve(dev(b), xd, rtol=1e-10)
        assert info.converged
        x = host(xd)
        assert np.array_equal(x[:, 0], x0[:, 0]) and np.array_equal(x[:, -1], x0[:, -1])
        res = np.linalg.norm(o.residual(x, b)[:, 1:-1]) / o.lifted_rhs_norm(b, x0)
        assert res <= 1.2e-10, res


def test_colour_passes_128_wide_level():
    """256 x 256 x 32 on five levels (coarsest 16 x 16 x 2): level 1 is
    128 x 128 x 16, the row width of the 128^3 level, smoothed by the
    two-colour launch with one thread per column pair and the XCD-ordered
    grid.  Colour passes match the oracle colour by colour, a whole sweep
    matches, and so does a whole V-cycle from a random start."""
    rng = np.random.default_rng(13)
    n = (256, 256, 32)
    g, o = make(*n, min_coarse_nz=2)
    L = o.levels[1]
    assert (L.nx, L.ny, L.nz) == (128, 128, 16) and g.levels == 5
    x = rand_node(rng, L.nx, L.ny, L.nz, walls=False)
    b = rand_node(rng, L.nx, L.ny, L.nz)
    xd, bd = dev(x), dev(b)
    for c in ROW:
        g.level_colour_pass(1, xd, bd, c)
        L.colour_pass(x, b, (c & 1, (c >> 1) & 1, (c >> 2) & 1))
        assert rel(host(xd), x) < 1e-13, c
    xd = dev(x)
    g.smooth(1, xd, bd, 1)
    L.sweep(x, b, o.order)
    assert rel(host(xd), x) < 1e-13
    bf = rand_node(rng, *n)
    x0 = rand_node(rng, *n)
    xd = dev(x0)
    g.solve(dev(bf), xd, rtol=0.0, max_cycles=1)
    x_ref, _ = o.solve(bf, x0, rtol=0.0, max_cycles=1)
    assert rel(host(xd), x_ref) < 1e-12


@pytest.mark.parametrize("n,mc", [((160, 24, 16), 4), ((64, 64, 64), 8)])
@pytest.mark.parametrize("order", [ROW, (7, 6, 3, 2, 5, 4, 1, 0), (1, 0, 3, 2, 5, 4, 7, 6),
                                   (2, 3, 0, 1, 6, 7, 4, 5)])
def test_paired_colour_sweeps(n, mc, order):
    """On coarse levels two colours that differ only in the x parity and follow
    each other in the order share one launch, with either parity first; whole
    sweeps match the oracle's colour-by-colour sweep (rows of 80 and 32 nodes,
    six and sixteen rows per workgroup), for 1 and 3 sweeps."""
    rng = np.random.default_rng(12)
    g, o = make(*n, min_coarse_nz=mc, colour_order=order)
    for level in range(1, g.levels - 1):
        L = o.levels[level]
        x = rand_node(rng, L.nx, L.ny, L.nz, walls=False)
        b = rand_node(rng, L.nx, L.ny, L.nz)
        for sweeps in (1, 3):
            xd = dev(x)
            g.smooth(level, xd, dev(b), sweeps)
            xr = x.copy()
            for _ in range(sweeps):
                L.sweep(xr, b, o.order)
            assert rel(host(xd), xr) < 1e-13, (level, sweeps)


def test_other_colour_order():
    """A colour permutation with no two x-parity partners next to each other
    runs one launch per colour on every level and matches the oracle."""
    rng = np.random.default_rng(7)
    order = [0, 4, 1, 5, 2, 6, 3, 7]
    g, o = make(32, 32, 32, colour_order=order)
    b = rand_node(rng, 32, 32, 32)
    x0 = np.zeros_like(b)
    xd = dev(x0)
    g.solve(dev(b), xd, rtol=0.0, max_cycles=3)
    x_ref, _ = o.solve(b, x0, rtol=0.0, max_cycles=3)
    assert rel(host(xd), x_ref) < 1e-12


def test_edge_cases():
    from paper_1904_03808_amd._capi import (QS_ERR_NONFINITE, QS_ERR_NOT_CONVERGED)
    rng = np.random.default_rng(8)
    n = 16
    g, o = make(n, n, n)
    # zero lifted right-hand side: x = 0, no cycle
    x0 = rand_node(rng, n, n, n, walls=False)
    xd = dev(x0)
    info = g.solve(dev(np.zeros_like(x0)), xd, rtol=1e-10)
    assert info.cycles == 0 and np.abs(host(xd)).max() == 0.0
    # not converged within max_cycles: last iterate kept, status reported
    b = rand_node(rng, n, n, n)
    xd = dev(np.zeros_like(b))
    info = g.solve(dev(b), xd, rtol=1e-14, max_cycles=2, raise_on_failure=False)
    assert info.status == QS_ERR_NOT_CONVERGED and info.cycles == 2
    x_ref, _ = o.solve(b, np.zeros_like(b), rtol=0.0, max_cycles=2)
    assert rel(host(xd), x_ref) < 1e-12
    # non-finite data
    b[0, 3, 2, 1] = np.nan
    info = g.solve(dev(b), dev(np.zeros_like(b)), rtol=1e-10, raise_on_failure=False)
    assert info.status == QS_ERR_NONFINITE
    # a node vector that is not 16-byte aligned is refused before any launch
    from paper_1904_03808_amd._capi import QS_ERR_ARG
    flat = torch.zeros(b.size + 1, dtype=torch.float64, device="cuda")
    xm = flat[1:].view(b.shape)
    assert xm.data_ptr() % 16 == 8
    info = g.solve(dev(np.nan_to_num(b)), xm, rtol=1e-10, raise_on_failure=False)
    assert info.status == QS_ERR_ARG
    assert torch.count_nonzero(flat).item() == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32-ir"])
def test_zero_cycles_and_a_converged_start(prec):
    """max_cycles = 0 runs no cycle: x is left as it was, bit for bit, the
    status says not converged, and the relative residual reported is the
    oracle's for the start; a start that already meets rtol (the oracle's
    direct solution) returns after no cycle with status OK and x unchanged."""
    from paper_1904_03808_amd._capi import QS_ERR_NOT_CONVERGED, QS_OK
    rng = np.random.default_rng(23)
    n = (16, 16, 16)
    g, o = make(*n, precision=prec)
    b = rand_node(rng, *n)
    x0 = rand_node(rng, *n)
    xd = dev(x0)
    info = g.solve(dev(b), xd, rtol=1e-10, max_cycles=0, raise_on_failure=False)
    assert info.status == QS_ERR_NOT_CONVERGED and info.cycles == 0
    assert np.array_equal(host(xd), x0)
    rel0 = np.linalg.norm(o.residual(x0, b)[:, 1:-1]) / o.lifted_rhs_norm(b, x0)
    assert abs(info.rel_res - rel0) <= 1e-12 * rel0, (info.rel_res, rel0)
    xs = direct_solve(b, x0, 1.0 / n[2], LAM, MU)
    xd = dev(xs)
    info = g.solve(dev(b), xd, rtol=1e-10, max_cycles=10, raise_on_failure=False)
    assert info.status == QS_OK and info.cycles == 0 and info.rel_res <= 1e-10
    assert np.array_equal(host(xd), xs)


def test_single_level_direct():
    """nz <= min_coarse_nz: one level solved by the dense inverse, walls lifted."""
    rng = np.random.default_rng(9)
    n = 8
    g, _ = make(n, n, n)
    assert g.levels == 1
    b = rand_node(rng, n, n, n)
    x0 = np.zeros_like(b)
    x0[:, 0] = rng.standard_normal((3, n, n))
    xd = dev(x0)
    info = g.solve(dev(b), xd, rtol=1e-12)
    assert info.cycles == 1
    xr = direct_solve(b, x0, 1.0 / n, LAM, MU)
    assert rel(host(xd), xr) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32-ir"])
@pytest.mark.parametrize("n", [(7, 5, 6), (5, 9, 3), (2, 2, 2), (2, 3, 4), (3, 2, 2)])
def test_single_level_odd_shapes(n, prec):
    """Odd dimensions are allowed on a grid that is not coarsened (nz <=
    min_coarse_nz), and so are the degenerate periodic lengths of 2, where a
    node's two neighbours along x (or y) are one node and their couplings add
    up (one interior plane at nz = 2): the operator matches the oracle's, and
    the solve (the dense inverse, with Dirichlet data on the walls) reaches
    the oracle's direct solution: 1e-12 in FP64, 1e-8 in FP32-IR after its
    refinement to a relative residual of 1e-12."""
    rng = np.random.default_rng(19)
    g, _ = make(*n, precision=prec)
    assert g.levels == 1
    h = 1.0 / n[2]
    x = rand_node(rng, *n)
    if prec == "fp64":
        assert rel(host(g.apply(dev(x))), apply_elastic(x, h, LAM, MU)) < 1e-13
    b = rand_node(rng, *n)
    x0 = np.zeros_like(b)
    x0[:, 0] = rng.standard_normal(x0[:, 0].shape)
    x0[:, -1] = rng.standard_normal(x0[:, -1].shape)
    xd = dev(x0)
    info = g.solve(dev(b), xd, rtol=1e-12)
    assert info.converged
    xr = direct_solve(b, x0, h, LAM, MU)
    assert rel(host(xd), xr) < (1e-12 if prec == "fp64" else 1e-8)
    assert np.array_equal(host(xd)[:, 0], x0[:, 0]) and np.array_equal(host(xd)[:, -1], x0[:, -1])


def test_calls_under_another_stream_are_refused():
    """The handle is bound to the stream current at construction: a call made
    while another torch stream is current raises instead of running unordered
    with the caller's work; under the bound stream it runs."""
    g, _ = make(16, 16, 16)
    b = dev(div_node(stress_field(16, 16, 16, 0), 1.0 / 16))
    x = torch.zeros_like(b)
    other = torch.cuda.Stream()
    with torch.cuda.stream(other):
        with pytest.raises(RuntimeError, match="stream"):
            g.solve(b, x, rtol=1e-10)
    torch.cuda.synchronize()
    assert not x.any()
    with torch.cuda.stream(g.stream):
        assert g.solve(b, x, rtol=1e-10).converged
