"""Pins of the oracle STZ update and projection step (paper Secs. 3.1 and 3.3)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import stz
from oracle.multigrid import MGOracle
from oracle.operators import voigt_to_full
from workloads import chi_field, lame, shear_velocity, stz_constants

LAM, MU = lame()
P = stz_constants()
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_table1_conversion_matches_printed_values():
    """Derived quantities printed in the paper: mu = 37.4 GPa, c_s = 2.47 km/s,
    t_s = L/c_s = 4.05 us (Table 1 and Sec. 4)."""
    g = json.load(open(os.path.join(GOLDEN, "table1.json")))
    E = g["E_GPa"] * 1e9
    mu = E / (2 * (1 + g["nu"]))
    assert round(mu / 1e9, 1) == g["mu_GPa_printed"]
    cs = math.sqrt(mu / g["rho_kg_m3"])
    assert round(cs / 1e3, 2) == g["c_s_km_s_printed"]
    assert round(0.01 / cs * 1e6, 2) == g["t_s_us_printed"]
    assert P["tau0"] == pytest.approx(g["tau0_s"] / (0.01 / cs), rel=1e-12)
    assert P["s_y"] == pytest.approx(0.85 / 101, rel=1e-12)
    assert P["chi_inf"] == pytest.approx(900 / 21000, rel=1e-12)
    assert P["delta_over_T"] == 20.0


def test_transition_rate_identity():
    """C = (R(+s) + R(-s))/2 = exp(-Delta/kT) cosh(Omega eps0 s/kT) (Eqs. stz_R, stz_C_form)."""
    s = np.linspace(0.0, 0.02, 101)
    a = stz.transition_rate(s, P)
    b = stz.transition_rate_from_R(s, P)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()


def test_deviator_and_yield():
    rng = np.random.default_rng(0)
    sig = rng.standard_normal((6, 2, 3, 4)) * 0.01
    S0, sbar = stz.deviator(voigt_to_full(sig))
    assert np.abs(S0[0, 0] + S0[1, 1] + S0[2, 2]).max() < 1e-16
    # pure shear: sbar = |sigma_xz|
    pure = np.zeros((6, 1, 1, 1))
    pure[4] = -0.0123
    _, sb = stz.deviator(voigt_to_full(pure))
    assert sb.item() == pytest.approx(0.0123, rel=1e-15)
    # no plastic flow at or below yield
    assert np.all(stz.plastic_rate(np.array([0.0, P["s_y"] * 0.999, P["s_y"]]), 0.05, P) == 0.0)
    assert stz.plastic_rate(np.array([P["s_y"] * 1.01]), 0.05, P)[0] > 0.0


def _uniform(nz, vals):
    s = np.zeros((6, nz, nz, nz))
    for n, v in enumerate(vals):
        s[n] = v
    return s


def test_plastic_relaxation_closed_form():
    """With L = 0 the update only shrinks the deviator: sbar* = sbar - 2 mu dt D^pl,
    pressure and deviator direction unchanged; chi moves toward chi_inf."""
    n, dt = 4, 3.0
    rng = np.random.default_rng(1)
    vals = rng.standard_normal(6) * 0.006
    sig = _uniform(n, vals)
    chi = np.full((n, n, n), 0.05)
    v = np.zeros((3, n + 1, n, n))
    S = voigt_to_full(sig)
    S0, sbar = stz.deviator(S)
    Dpl = stz.plastic_rate(sbar, chi, P)
    assert np.all(Dpl > 0)
    sstar, chi1 = stz.stz_step(v, sig, chi, 1.0 / n, dt, LAM, MU, P)
    T = voigt_to_full(sstar)
    T0, tbar = stz.deviator(T)
    assert np.abs(tbar - (sbar - 2 * MU * dt * Dpl)).max() < 1e-15
    assert np.abs(np.trace(T) - np.trace(S)).max() < 1e-16
    assert np.abs(T0 / tbar - S0 / sbar).max() < 1e-12
    assert np.all(chi1 < chi) and np.all(chi1 > P["chi_inf"])


def test_truesdell_kinematics_closed_form():
    """Below yield: simple shear v_x = g z acting on sigma_zz = s gives
    sigma*_xz = dt g s (L sigma + sigma L^T); a dilatation L = e I scales an
    isotropic stress by 1 - dt e (2 - 3)."""
    n, dt, g, s = 4, 0.5, 1e-3, 2e-3
    h = 1.0 / n
    sig = _uniform(n, [0, 0, s, 0, 0, 0])
    chi = np.full((n, n, n), 0.05)
    v = shear_velocity(n, n, n, g / 2.0)  # v_x = (g/2)(2z - 1), so dv_x/dz = g
    sstar, chi1 = stz.stz_step(v, sig, chi, h, dt, LAM, MU, P)
    expect = sig.copy()
    expect[4] += dt * g * s
    assert np.abs(sstar - expect).max() < 1e-17
    assert np.array_equal(chi1, chi)
    # pure dilatation in z only is the one linear field allowed with periodic x, y:
    # L = diag(0, 0, e): sigma = p I -> sigma* = p I + dt (2 e p e_z e_z - e p I)
    e, p = 2e-3, 1e-3
    v = np.zeros((3, n + 1, n, n))
    v[2] = (e * np.arange(n + 1) * h)[:, None, None]
    sig = _uniform(n, [p, p, p, 0, 0, 0])
    sstar, _ = stz.stz_step(v, sig, chi, h, dt, LAM, MU, P)
    want = np.array([p - dt * e * p, p - dt * e * p, p + dt * (2 * e * p - e * p), 0, 0, 0])
    assert np.abs(sstar - want[:, None, None, None]).max() < 1e-18


def test_homogeneous_shear_step_reduces_to_scalar_recursion():
    """Uniform chi and sigma with a linear wall-to-wall velocity: the step keeps
    the linear profile (0 cycles from a warm start) and a uniform stress that
    follows the one-cell update plus dt * 2 mu * U of elastic loading."""
    n, dt, U = 8, 10.0, 1e-5
    h = 1.0 / n
    mg = MGOracle(n, n, n, h, LAM, MU)
    sig = _uniform(n, [0, 0, 0, 0, 1.01 * P["s_y"], 0])
    chi = np.full((n, n, n), 0.05)
    v = shear_velocity(n, n, n, U)
    v1, s1, chi1, info = stz.projection_step(v, sig, chi, h, dt, LAM, MU, P, U, mg)
    assert info["cycles"] == 0
    assert np.abs(v1 - v).max() == 0.0
    # one-cell evaluation of the same step
    one = stz.stz_step(shear_velocity(1, 1, 1, U), sig[:, :1, :1, :1], chi[:1, :1, :1],
                       1.0, dt, LAM, MU, P)[0]
    # sym(grad v)_xz = U (dv_x/dz = 2U), C : D adds 2 mu U to sigma_xz
    expect = one[:, 0, 0, 0].copy()
    expect[4] += dt * 2 * MU * U
    assert np.abs(s1 - expect[:, None, None, None]).max() < 1e-18
    # from a zero initial guess the solve converges to the same profile
    v0 = stz.set_shear_walls(np.zeros_like(v), U)
    x, info = mg.solve(np.zeros_like(v), v0, rtol=1e-12)
    assert np.abs(x - v).max() < 1e-11 * U


def test_chi_field_statistics():
    """Eq. convolve keeps the pointwise mean and std of the random field."""
    chi = chi_field(96, 96, 96, seed=3, mean=0.05, std=0.003, lc_cells=4.0)
    assert abs(chi.mean() - 0.05) < 2e-4
    assert abs(chi.std() / 0.003 - 1.0) < 0.08


def test_chi_diffusion_operator_closed_forms():
    """The 7-point flux form of div(D grad chi) (Eq. chi_evo): for constant D
    a Fourier mode in x and y is an eigenfunction with eigenvalue
    D (2 cos(2 pi m/nx) - 2 + 2 cos(2 pi q/ny) - 2) / h^2; a field linear in z
    (its linearly extrapolated ghosts continue it) and a constant field give
    zero for any D."""
    nx, ny, nz, h = 12, 10, 6, 0.1
    rng = np.random.default_rng(5)
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    kz = np.arange(nz + 2)[:, None, None]
    D = 0.7
    m, q = 3, 2
    mode = np.cos(2 * np.pi * m * i / nx) * np.cos(2 * np.pi * q * j / ny) * (1.0 + 0 * kz)
    out = stz.flux_divergence(np.full(mode.shape, D), mode, h)
    lam_ = D * ((2 * np.cos(2 * np.pi * m / nx) - 2) + (2 * np.cos(2 * np.pi * q / ny) - 2)) / h**2
    assert np.abs(out - lam_ * mode[1:-1]).max() <= 1e-12 * abs(lam_)
    zlin = stz.z_ghosts(np.broadcast_to(0.3 + 0.05 * np.arange(nz)[:, None, None], (nz, ny, nx)))
    assert np.abs(zlin[0] - 0.25).max() < 1e-15 and np.abs(zlin[-1] - (0.3 + 0.05 * nz)).max() < 1e-15
    out = stz.flux_divergence(np.full(zlin.shape, D), zlin, h)
    assert np.abs(out).max() <= 1e-12
    Dr = rng.uniform(0.1, 1.0, (nz + 2, ny, nx))
    assert np.abs(stz.flux_divergence(Dr, np.full(Dr.shape, 0.04), h)).max() == 0.0


def test_chi_diffusion_flux_form_is_conservative_in_x_and_y():
    """With D and chi constant in z, the z faces carry no flux, and the x and y
    faces are shared by two cells with opposite signs, so the cell sum of
    div(D grad chi) over a periodic x-y plane vanishes for any D, chi."""
    rng = np.random.default_rng(6)
    nx, ny, nz = 9, 7, 4
    Dp = rng.uniform(0.1, 1.0, (1, ny, nx))
    cp = rng.uniform(0.02, 0.06, (1, ny, nx))
    D = np.repeat(Dp, nz + 2, axis=0)
    c = np.repeat(cp, nz + 2, axis=0)
    out = stz.flux_divergence(D, c, 0.2)
    assert np.abs(out.sum(axis=(1, 2))).max() <= 1e-12 * np.abs(out).max()


def test_chi_diffusion_operator_is_symmetric_negative_semidefinite():
    """For D^pl varying in x and y (constant in z, so no z flux), the map
    chi -> div(D grad chi) on a periodic plane is a weighted graph Laplacian:
    symmetric (each face coefficient is shared by its two cells), negative
    semidefinite, with the constants in its null space.  Using D of one cell
    instead of the face mean, or a shifted neighbour index, breaks the
    symmetry."""
    rng = np.random.default_rng(8)
    nx, ny, nz = 5, 4, 3
    Dp = rng.uniform(0.1, 1.0, (ny, nx))
    D = np.broadcast_to(Dp, (nz + 2, ny, nx)).copy()
    M = np.zeros((ny * nx, ny * nx))
    for q in range(ny * nx):
        e = np.zeros(ny * nx)
        e[q] = 1.0
        c = np.broadcast_to(e.reshape(ny, nx), (nz + 2, ny, nx)).copy()
        out = stz.flux_divergence(D, c, 0.5)
        assert np.abs(out - out[0]).max() == 0.0
        M[:, q] = out[0].ravel()
    assert np.abs(M - M.T).max() <= 1e-14
    assert np.linalg.eigvalsh(M).max() <= 1e-12
    assert np.abs(M.sum(axis=1)).max() <= 1e-13
    # a face's coefficient is the mean of its two cells' D
    assert np.isclose(M[0, 1], (Dp[0, 0] + Dp[0, 1]) / 2 / 0.25)


def test_chi_step_with_diffusion_adds_the_flux_term():
    """stz_step with l > 0 adds (dt/c0) l^2 div(D^pl grad chi) to the chi of
    the l = 0 step, with D^pl evaluated on sigma and chi of step n (ghost
    layers by linear extrapolation); above yield the term is nonzero."""
    rng = np.random.default_rng(7)
    nx, ny, nz = 8, 6, 5
    h = 1.0 / nz
    v = shear_velocity(nx, ny, nz, 1e-5)
    sigma = np.zeros((6, nz, ny, nx))
    sigma[4] = P["s_y"] * rng.uniform(1.02, 1.06, (nz, ny, nx))
    chi = chi_field(nx, ny, nz, 3, 0.05, 0.003, 2.0)
    p0 = dict(P)
    p1 = dict(P, l_diff=h)
    dt = 10.0
    s0, c0 = stz.stz_step(v, sigma, chi, h, dt, LAM, MU, p0)
    s1, c1 = stz.stz_step(v, sigma, chi, h, dt, LAM, MU, p1)
    assert np.array_equal(s0, s1)
    term = stz.chi_diffusion(sigma, chi, h, P)
    assert np.abs(term).max() > 0.0
    # (the difference of two chi values carries their rounding, 1e-16 absolute)
    assert np.allclose(c1 - c0, (dt / P["c0"]) * h * h * term, rtol=1e-12, atol=1e-16)
    # the ghost layer of a cell next to a wall: D^pl of the extrapolated state
    sg, cg = stz.z_ghosts(sigma), stz.z_ghosts(chi)
    assert np.allclose(sg[:, 0], 2 * sigma[:, 0] - sigma[:, 1])
    assert np.allclose(cg[-1], 2 * chi[-1] - chi[-2])


def test_projection_step_with_node_walls_reduces_to_the_shear_walls():
    """Wall data given node by node, equal to the walls of Eq. u_bc, gives the
    step of the U path bit for bit; other wall data ends up in the wall
    planes of v^{n+1} exactly, with the interior solving K v = b."""
    from oracle.multigrid import MGOracle
    from oracle.operators import apply_elastic
    from workloads import weld_walls
    nx, ny, nz = 8, 8, 8
    h = 1.0 / nz
    U, dt = 1e-5, 10.0
    v = shear_velocity(nx, ny, nz, U)
    sigma = np.zeros((6, nz, ny, nx))
    sigma[4] = 1.02 * P["s_y"]
    chi = chi_field(nx, ny, nz, 3, 0.05, 0.003, 2.0)
    o = MGOracle(nx, ny, nz, h, LAM, MU, min_coarse_nz=4)
    ref = stz.projection_step(v, sigma, chi, h, dt, LAM, MU, P, U, o, rtol=1e-12)
    w = stz.set_shear_walls(np.zeros_like(v), U)
    got = stz.projection_step(v, sigma, chi, h, dt, LAM, MU, P, 0.0, o, rtol=1e-12,
                              walls=(w[:, 0], w[:, -1]))
    for a, b in zip(ref[:3], got[:3]):
        assert np.array_equal(a, b)
    lo, hi = weld_walls(nx, ny, nz, 1e-4, h, top=True, bottom=True)
    v1, s1, c1, info = stz.projection_step(v, sigma, chi, h, dt, LAM, MU, P, 0.0, o, rtol=1e-12,
                                           walls=(lo, hi))
    assert np.array_equal(v1[:, 0], lo) and np.array_equal(v1[:, -1], hi)
    sstar, _ = stz.stz_step(v, sigma, chi, h, dt, LAM, MU, P)
    b = stz.rhs(sstar, h, dt)
    r = (b - apply_elastic(v1, h, LAM, MU))[:, 1:nz]
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b[:, 1:nz] - apply_elastic(
        stz.set_walls(np.zeros_like(v), lo, hi), h, LAM, MU)[:, 1:nz])


def _relaxation_exact(sbar0, chi0, dt, p):
    """The local plastic relaxation with L = 0 as an ODE in (sbar, chi):
    dsbar/dt = -2 mu D^pl, c0 dchi/dt = (2 sbar D^pl / s_Y)(chi_inf - chi)
    (the deviator keeps its direction), integrated by scipy's Radau."""
    from scipy.integrate import solve_ivp

    def f(t, y):
        D = float(stz.plastic_rate(np.array([y[0]]), np.array([y[1]]), p)[0])
        return [-2.0 * MU * D, (2.0 * y[0] * D / p["s_y"]) * (p["chi_inf"] - y[1]) / p["c0"]]

    r = solve_ivp(f, (0.0, dt), [sbar0, chi0], method="Radau", rtol=1e-12, atol=[1e-16, 1e-16])
    return r.y[0, -1], r.y[1, -1]


def _one_cell(vals, chi, dt, p):
    sig = _uniform(1, vals)
    L = np.zeros((3, 3, 1, 1, 1))
    ss, c1 = stz.stz_pointwise(L, sig, np.full((1, 1, 1), chi), dt, LAM, MU, p)
    T = voigt_to_full(ss)
    T0, tbar = stz.deviator(T)
    return T, T0, float(tbar.ravel()[0]), float(c1.ravel()[0])


def test_plastic_substeps_converge_to_the_local_relaxation():
    """Sub-stepped plastic terms (an extension: the paper takes one step) are
    forward Euler of the local relaxation ODE, so with L = 0 they converge to
    its solution at first order in the sub-step, here on a step whose single
    forward-Euler update is unstable (2 mu dt dD/dsbar = 6); pressure and the
    deviator's direction are kept."""
    rng = np.random.default_rng(11)
    vals = rng.standard_normal(6)
    S = voigt_to_full(_uniform(1, vals))
    _, sb = stz.deviator(S)
    vals = vals * (1.3 * P["s_y"] / float(sb.ravel()[0]))
    chi = 0.04
    slope = float(stz.plastic_rate_slope(np.array([1.3 * P["s_y"]]), np.array([chi]), P)[0])
    dt = 6.0 / (2 * MU * slope)
    s_ex, c_ex = _relaxation_exact(1.3 * P["s_y"], chi, dt, P)
    assert P["s_y"] < s_ex < 1.3 * P["s_y"] and chi < c_ex
    errs = []
    for M in (64, 128, 256, 512):
        T, T0, tbar, c1 = _one_cell(vals, chi, dt, dict(P, n_sub=M))
        errs.append(abs(tbar - s_ex))
        S0, _ = stz.deviator(voigt_to_full(_uniform(1, vals)))
        assert np.allclose(T0 / tbar, S0 / (1.3 * P["s_y"]), rtol=1e-12, atol=1e-14)
        assert np.isclose(np.trace(T).item(), np.trace(voigt_to_full(_uniform(1, vals))).item(),
                          rtol=1e-14, atol=1e-18)
        assert abs(c1 - c_ex) <= 20.0 * abs(c_ex - chi) / M
    ratios = np.array(errs[1:]) / np.array(errs[:-1])
    assert np.all(ratios > 0.4) and np.all(ratios < 0.6), ratios
    assert errs[-1] < 2e-3 * (1.3 * P["s_y"] - s_ex)
    # the single step overshoots below yield on this step
    _, _, t1, _ = _one_cell(vals, chi, dt, P)
    assert t1 < P["s_y"]


def test_adaptive_substeps_keep_a_stiff_cell_stable():
    """n_sub = -1: a cell where 2 mu dt dD/dsbar = 400 takes enough sub-steps
    (each with tau 2 mu dD/dsbar <= 1/2) that sbar decreases monotonically to
    between s_Y and its start, chi rises toward chi_inf, and both land near
    the ODE solution; n_sub = 0 and 1 are the paper's single step."""
    vals = np.array([0.0, 0.0, 0.0, 0.0, 1.25 * P["s_y"], 0.0])
    chi = 0.04
    slope = float(stz.plastic_rate_slope(np.array([1.25 * P["s_y"]]), np.array([chi]), P)[0])
    dt = 400.0 / (2 * MU * slope)
    M = stz.substep_count(np.array([1.25 * P["s_y"]]), np.array([chi]), dt, MU, dict(P, n_sub=-1))
    assert M[0] >= 800 and M[0] <= 802
    _, _, tbar, c1 = _one_cell(vals, chi, dt, dict(P, n_sub=-1))
    s_ex, c_ex = _relaxation_exact(1.25 * P["s_y"], chi, dt, P)
    assert P["s_y"] < tbar < 1.25 * P["s_y"] and chi < c1 < P["chi_inf"]
    assert abs(tbar - s_ex) < 0.01 * (1.25 * P["s_y"] - s_ex)
    a = _one_cell(vals, chi, dt, dict(P, n_sub=0))
    b = _one_cell(vals, chi, dt, dict(P, n_sub=1))
    c = _one_cell(vals, chi, dt, P)
    assert a[2] == b[2] == c[2] and a[3] == b[3] == c[3]
    # the single step flips the deviator and leaves it larger than it started
    assert a[2] > 10 * 1.25 * P["s_y"]


def test_eno_derivative_branches_by_hand():
    """Eq. ENO on five values f(i-2 .. i+2) = 0, 0, 0, 1, 4 with h = 1/2 (so
    the factor 1/(2h) is 1): the curvatures |f_xx| h^2 at i-1, i, i+1 are
    0, 1, 2.  Moving right (u > 0), i is more curved than i-1: the backward
    three-point formula gives 3*0 - 4*0 + 0 = 0.  Moving left, i is less
    curved than i+1: the centred difference 1 - 0 = 1.  At rest: centred."""
    g = np.array([0.0, 0.0, 0.0, 1.0, 4.0])
    for u, want in ((1.0, 0.0), (-1.0, 1.0), (0.0, 1.0)):
        d = stz.eno_derivative(g, np.array([u]), 0.5, 0)
        assert d.shape == (1,) and d[0] == want
    # mirrored values: moving left now takes the forward formula
    g = np.array([4.0, 1.0, 0.0, 0.0, 0.0])
    assert stz.eno_derivative(g, np.array([-1.0]), 0.5, 0)[0] == -(-0.0 + 4 * 0.0 - 3 * 0.0)
    assert stz.eno_derivative(g, np.array([1.0]), 0.5, 0)[0] == 0.0 - 1.0
    # every branch is exact for a quadratic
    x = np.arange(-2, 9) * 0.1
    f = 0.3 - 1.7 * x + 2.5 * x * x
    for u in (-1.0, 0.0, 1.0):
        d = stz.eno_derivative(f, np.full(7, u), 0.1, 0)
        assert np.allclose(d, -1.7 + 5.0 * x[2:-2], rtol=0, atol=1e-12)


def test_advection_of_a_field_linear_in_z_is_exact():
    """sigma = a + b z (every component its own a, b) is continued exactly by
    the linear ghost layers, so (v . grad) sigma = w_cell b at every cell,
    including those next to the walls, for any velocity; w_cell is the mean
    of the cell's eight corners."""
    rng = np.random.default_rng(13)
    nx, ny, nz = 6, 5, 4
    h = 0.25
    zc = (np.arange(nz) + 0.5) * h
    a, b = rng.standard_normal(6), rng.standard_normal(6)
    sigma = np.broadcast_to((a[:, None] + b[:, None] * zc)[:, :, None, None],
                            (6, nz, ny, nx)).copy()
    v = rng.standard_normal((3, nz + 1, ny, nx))
    adv = stz.advection(sigma, v, h)
    w = np.zeros((nz, ny, nx))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w += v[2, dz:nz + dz][:, (np.arange(ny) + dy) % ny][:, :, (np.arange(nx) + dx) % nx]
    w /= 8.0
    assert np.allclose(adv, b[:, None, None, None] * w, rtol=1e-12, atol=1e-13)


def test_advection_is_second_order_for_smooth_fields():
    """A smooth periodic-in-x,y field advected by a uniform velocity: the
    error against the exact u . grad sigma at cells at least two layers from
    the walls falls by about 4 when h halves."""
    U = np.array([0.7, -0.4, 0.3])
    errs = []
    for n in (16, 32):
        h = 1.0 / n
        xc = (np.arange(n) + 0.5) * h
        Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")
        f = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) * (1 + Z * Z)
        df = (U[0] * 2 * np.pi * np.cos(2 * np.pi * X) * np.cos(2 * np.pi * Y) * (1 + Z * Z)
              - U[1] * 2 * np.pi * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) * (1 + Z * Z)
              + U[2] * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) * 2 * Z)
        sigma = np.broadcast_to(f, (6, n, n, n)).copy()
        v = np.broadcast_to(U[:, None, None, None], (3, n + 1, n, n)).copy()
        adv = stz.advection(sigma, v, h)
        errs.append(np.abs(adv[:, 2:-2] - df[2:-2]).max())
    assert 3.3 < errs[0] / errs[1] < 4.7, errs


def test_node_laplacian_and_advection_closed_forms():
    """The explicit method's node operators: a Fourier mode in x is an
    eigenfunction of the Laplacian with eigenvalue -(4/h^2) sin^2(pi m/nx);
    a quadratic in z gives its second derivative exactly; a velocity linear
    in z (v_x = a + b z, v_y = c + d z, v_z = w) has (v . grad) v = (w b, w d, 0)
    exactly at every interior node, the ones next to the walls included (the
    reflected ghost nodes continue a linear profile)."""
    nx, ny, nz, h = 12, 6, 8, 0.125
    i = np.arange(nx)[None, None, :]
    k = np.arange(nz + 1)[:, None, None]
    m = 3
    f = np.cos(2 * np.pi * m * i / nx) * np.ones((nz + 1, ny, 1))
    v = np.stack([f, 0 * f, 0 * f])
    lap = stz.node_laplacian(v, h)
    lam_ = -(4.0 / h**2) * np.sin(np.pi * m / nx) ** 2
    assert np.allclose(lap[0, 1:-1], lam_ * f[1:-1], rtol=0, atol=1e-11)
    assert not lap[:, 0].any() and not lap[:, -1].any()
    q = (0.3 + 0.7 * (k * h) ** 2) * np.ones((1, ny, nx))
    lap = stz.node_laplacian(np.stack([q, q, q]), h)
    assert np.allclose(lap[:, 1:-1], 1.4, rtol=1e-12)
    a, b, c, d, w = 0.2, -1.3, 0.5, 0.9, -0.4
    z = k * h * np.ones((1, ny, nx))
    v = np.stack([a + b * z, c + d * z, w + 0 * z])
    adv = stz.node_advection(v, h)
    assert np.allclose(adv[0, 1:-1], w * b, rtol=1e-12)
    assert np.allclose(adv[1, 1:-1], w * d, rtol=1e-12)
    assert np.abs(adv[2]).max() < 1e-15


def test_explicit_step_simple_shear_from_rest():
    """Sec. 3.2 on a linear shear profile between walls moving at -U and +U,
    stress free and below yield: the velocity has no divergence of stress,
    no curvature and no advection, so it stays; the stress takes
    dt C : D with D_xz = U (the Truesdell terms vanish at sigma = 0), i.e.
    sigma_xz = 2 mu U dt and nothing else; chi does not move."""
    nx, ny, nz = 6, 4, 8
    h, dt, U = 1.0 / nz, 0.01, 1e-3
    v = shear_velocity(nx, ny, nz, U)
    sigma = np.zeros((6, nz, ny, nx))
    chi = np.full((nz, ny, nx), 0.03)
    v1, s1, c1 = stz.explicit_step(v, sigma, chi, h, dt, LAM, MU, P, U, MU, 4.8 * h)
    assert np.allclose(v1, v, rtol=0, atol=1e-18)
    want = np.zeros_like(sigma)
    want[4] = 2 * MU * U * dt
    assert np.allclose(s1, want, rtol=1e-12, atol=1e-20)
    assert np.array_equal(c1, chi)


def test_chi_diffusion_closed_walls_conserve_chi():
    """chi_wall = 1: with sigma and chi constant in x and y the x, y faces
    carry no flux and the interior z faces cancel in the column sum, so with
    closed wall faces the column sum vanishes; with chi_wall = 0 the two
    wall faces remain, each carrying the mean of its cell's D^pl and the
    ghost state's times the extrapolated difference."""
    nx, ny, nz, h = 3, 2, 6, 0.2
    z = np.arange(nz)
    sigma = np.zeros((6, nz, ny, nx))
    sigma[4] = (P["s_y"] * (1.05 + 0.04 * z + 0.01 * z * z))[:, None, None]
    chi = np.broadcast_to((0.03 + 0.002 * z + 0.0005 * z * z)[:, None, None], (nz, ny, nx)).copy()
    p1 = dict(P, chi_wall=1)
    t1 = stz.chi_diffusion(sigma, chi, h, p1)
    assert abs(t1[:, 0, 0].sum()) <= 1e-12 * np.abs(t1).max()
    assert np.allclose(t1, t1[:, :1, :1], rtol=1e-14)
    t0 = stz.chi_diffusion(sigma, chi, h, P)
    assert np.array_equal(t0[1:-1], t1[1:-1])
    sg = stz.z_ghosts(sigma)
    _, sb = stz.deviator(voigt_to_full(sg))
    D = stz.plastic_rate(sb, stz.z_ghosts(chi), P)[:, 0, 0]
    c = chi[:, 0, 0]
    want = (0.5 * (D[1] + D[0]) * (c[0] - c[1]) + 0.5 * (D[-2] + D[-1]) * (c[-1] - c[-2])) / h**2
    assert np.isclose(t0[:, 0, 0].sum(), want, rtol=1e-10)


def test_implicit_plastic_update_bounds_and_consistency():
    """n_sub = -2 (backward Euler of the local relaxation, an extension): for
    any dt, even 1e8 t_s, sbar lands in [s_Y, sbar^n] and chi between chi^n
    and chi_inf, with pressure and deviator direction kept; the bisection
    solves its equation s - sbar + 2 mu dt D^pl(s) = 0 to the last bits; its
    one-step error against scipy's Radau solution of the local ODE falls as
    dt^2 (a consistent first-order method), as does its distance to the
    single forward-Euler step."""
    rng = np.random.default_rng(21)
    vals = rng.standard_normal(6)
    S = voigt_to_full(_uniform(1, vals))
    _, sb = stz.deviator(S)
    s0 = 1.4 * P["s_y"]
    vals = vals * (s0 / float(sb.ravel()[0]))
    chi = 0.04
    p2 = dict(P, n_sub=-2)
    S0n, _ = stz.deviator(voigt_to_full(_uniform(1, vals)))
    for dt in (10.0, 1e4, 1e8):
        T, T0, tbar, c1 = _one_cell(vals, chi, dt, p2)
        assert P["s_y"] <= tbar <= s0 and chi <= c1 <= P["chi_inf"]
        assert np.allclose(T0 / tbar, S0n / s0, rtol=1e-12, atol=1e-14)
        assert np.isclose(np.trace(T).item(), np.trace(voigt_to_full(_uniform(1, vals))).item(),
                          rtol=1e-14, atol=1e-18)
        g = tbar - s0 + 2 * MU * dt * float(stz.plastic_rate(np.array([tbar]), np.array([chi]), P)[0])
        slope = float(stz.plastic_rate_slope(np.array([tbar]), np.array([chi]), P)[0])
        assert abs(g) <= 1e-14 * s0 * (1 + 2 * MU * dt * slope)
    slope0 = float(stz.plastic_rate_slope(np.array([s0]), np.array([chi]), P)[0])
    base = 0.05 / (2 * MU * slope0)
    errs, gaps = [], []
    for k in range(3):
        dt = base / 2 ** k
        s_ex, _ = _relaxation_exact(s0, chi, dt, P)
        _, _, tb, _ = _one_cell(vals, chi, dt, p2)
        _, _, tf, _ = _one_cell(vals, chi, dt, P)
        errs.append(abs(tb - s_ex))
        gaps.append(abs(tb - tf))
    for e in (errs, gaps):
        r = np.array(e[:-1]) / np.array(e[1:])
        assert np.all(r > 3.3) and np.all(r < 4.7), e


@pytest.mark.slow
def test_explicit_method_reaches_the_quasi_static_state():
    """The explicit method (Sec. 3.2) and the quasi-static method (Sec. 3.3)
    discretise the same equations, the first with inertia and damping: on an
    elastic simple shear whose wall speed ramps up over one t_s (Eq. u_bc) and
    then holds, both must give the linear shear profile once the waves have
    died out (here at t = 6 t_s on 8^3 with kappa = 4.8 h).  The stress means
    then differ only by the quasi-static step's first-order time error:
    each of its steps adds dt C : D at the end of the step, which is
    mu U dt ahead of the continuous integral while U ramps, so the gap halves
    with dt."""
    from workloads import shear_velocity as sv
    n = 8
    h, UB, T = 1.0 / n, 1e-3, 6.0
    chi = np.full((n, n, n), 0.02)  # far below any plastic activity
    dt = h * h / 20
    v = sv(n, n, n, 0.0)
    s = np.zeros((6, n, n, n))
    c = chi.copy()
    for i in range(int(round(T / dt))):
        U = UB * min((i + 1) * dt, 1.0)
        v, s, c = stz.explicit_step(v, s, c, h, dt, LAM, MU, P, U, MU, 4.8 * h)
    o = MGOracle(n, n, n, h, LAM, MU, min_coarse_nz=4)
    gaps = []
    for dq in (0.25, 0.125):
        vq = sv(n, n, n, 0.0)
        sq = np.zeros((6, n, n, n))
        cq = chi.copy()
        for i in range(int(round(T / dq))):
            U = UB * min((i + 1) * dq, 1.0)
            vq, sq, cq, _ = stz.projection_step(vq, sq, cq, h, dq, LAM, MU, P, U, o, rtol=1e-12)
        assert np.abs(v - vq).max() <= 1e-4 * UB
        assert np.abs(sq[4] - sq[4].mean()).max() <= 1e-12 * sq[4].mean()
        gaps.append(sq[4].mean() - s[4].mean())
        assert abs(gaps[-1] - MU * UB * dq) <= 0.05 * MU * UB * dq
    # the explicit stress is uniform too: the waves are gone
    assert np.abs(s[4] - s[4].mean()).max() <= 1e-3 * s[4].mean()


@pytest.mark.parametrize("advect,diff", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_stz_step_at_cells_matches_the_whole_grid(advect, diff):
    """The cell-by-cell evaluation of the oracle's STZ step (which checks the
    GPU step at full size on sampled cells) equals the oracle's step on the
    whole grid at every cell of a 12 x 10 x 9 grid, the wall layers and the
    wrapped first and last rows and columns included, with and without the
    ENO advection of the stress, and with and without the chi diffusion term
    (l = h, per-cell plastic sub-steps)."""
    from cell_sample import near_yield_state, stz_step_at_cells
    rng = np.random.default_rng(23)
    nx, ny, nz = 12, 10, 9
    h, dt = 1.0 / nz, 10.0
    P = stz_constants()
    v, sig, chi = near_yield_state(rng, nx, ny, nz, P["s_y"])
    p = dict(P, advect=advect)
    if diff:
        p.update(l_diff=h, n_sub=-1)
    rs, rc = stz.stz_step(v, sig, chi, h, dt, LAM, MU, p)
    cells = [(k, j, i) for k in range(nz) for j in range(ny) for i in range(nx)]
    ss, cn = stz_step_at_cells(v, sig, chi, h, dt, LAM, MU, p, cells)
    want_s = np.array([rs[:, k, j, i] for k, j, i in cells])
    want_c = np.array([rc[k, j, i] for k, j, i in cells])
    assert np.abs(ss - want_s).max() <= 1e-14 * np.abs(want_s).max()
    assert np.abs(cn - want_c).max() <= 1e-14 * np.abs(want_c - chi.ravel()).max()
    if advect:
        r0, _ = stz.stz_step(v, sig, chi, h, dt, LAM, MU, dict(p, advect=0))
        assert np.abs(rs - r0).max() > 1e-3 * np.abs(rs).max()
    if diff:
        _, c0 = stz.stz_step(v, sig, chi, h, dt, LAM, MU, dict(p, l_diff=0.0))
        assert np.abs(rc - c0).max() > 1e-3 * np.abs(rc - chi).max()
