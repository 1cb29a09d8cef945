"""Athermal STZ plasticity and the quasi-static projection step.

Paper Sec. 3.1 (plastic rate of deformation, effective temperature) and
Sec. 3.3 (intermediate stress, projection, stress correction), written in the
nondimensional units of `workloads.stz_constants` (stress in E, time in t_s,
length in L, chi in e_z/k_B).

Readings where the paper is silent or inconsistent (also in the design notes):
  * the objective-rate term is -tr(L) sigma, as in the definition of the
    Truesdell rate (Sec. 2.1) and Eq. sig_star_qs;
  * D^pl = 0 when sbar <= s_Y (the factor 1 - s_Y/sbar would be negative);
  * the effective temperature takes a forward-Euler step with the state at
    step n (Eq. chi_evo_exp written for the quasi-static step);
  * its diffusion term l^2 div(D^pl grad chi) is the 7-point flux form on
    cells, each face carrying the mean of D^pl in its two cells; in z the
    ghost layer of sigma and chi is the linear extrapolation of the two
    nearest layers (Sec. 3.5), and D^pl there is evaluated on the ghost
    values (D^pl = 0 where the extrapolated chi is not positive); x and y
    wrap; l = 0 leaves the term out; p["chi_wall"] = 1 (not the paper's)
    closes the wall faces to the flux instead;
  * Eq. sig_star_qs has no advection term, so none is applied.
"""
from __future__ import annotations

import numpy as np

from .operators import (div_node, full_to_voigt, grad_cell, stiffness, sym,
                        voigt_to_full)


def transition_rate(sbar, p):
    """C(sbar, T) = exp(-Delta/kT) cosh(Omega eps0 sbar / kT) (Eq. stz_C_form)."""
    return np.exp(-p["delta_over_T"]) * np.cosh(p["beta"] * sbar)


def transition_rate_from_R(sbar, p):
    """C = (R(+sbar) + R(-sbar)) / 2 with the stress-biased rates of Eq. stz_R."""
    Rp = np.exp(-p["delta_over_T"] + p["beta"] * sbar)
    Rm = np.exp(-p["delta_over_T"] - p["beta"] * sbar)
    return 0.5 * (Rp + Rm)


def deviator(S):
    """sigma_0 = sigma - tr(sigma)/3 I and sbar = sqrt(sum sigma_0,ij^2 / 2)."""
    p = (S[0, 0] + S[1, 1] + S[2, 2]) / 3.0
    S0 = S.copy()
    for a in range(3):
        S0[a, a] = S0[a, a] - p
    sbar = np.sqrt(0.5 * np.sum(S0 * S0, axis=(0, 1)))
    return S0, sbar


def plastic_rate(sbar, chi, p):
    """Scalar D^pl of Eq. stz_dpl; zero at or below the yield stress.

    Complex-safe (the yield test looks at the real part), so that the
    complex-step method can differentiate it.
    """
    sbar = np.asarray(sbar)
    act = np.real(sbar) > p["s_y"]
    sb = np.where(act, sbar, p["s_y"])
    val = (np.exp(-1.0 / chi) * transition_rate(sb, p) * (1.0 - p["s_y"] / sb) / p["tau0"])
    return np.where(act, val, 0.0 * val)


def z_ghosts(f):
    """f [..., nz, ny, nx] extended by one cell layer below and above in z,
    each the linear extrapolation of the two nearest layers."""
    lo = 2.0 * f[..., :1, :, :] - f[..., 1:2, :, :]
    hi = 2.0 * f[..., -1:, :, :] - f[..., -2:-1, :, :]
    return np.concatenate([lo, f, hi], axis=-3)


def flux_divergence(D, chi, h):
    """div(D grad chi) at the cells of the z-ghosted arrays D, chi
    [nz+2, ny, nx] (layer 0 and nz+1 are ghosts): the 7-point flux form with
    face coefficients (D_c + D_n) / 2; x and y wrap.  Returns [nz, ny, nx]."""
    Dc, xc = D[1:-1], chi[1:-1]
    out = np.zeros_like(xc)
    for axis in (1, 2):  # y, x of the interior block (periodic)
        for s in (-1, 1):
            Dn, xn = np.roll(Dc, s, axis=axis), np.roll(xc, s, axis=axis)
            out = out + 0.5 * (Dc + Dn) * (xn - xc)
    for Dn, xn in ((D[:-2], chi[:-2]), (D[2:], chi[2:])):  # z - 1, z + 1
        out = out + 0.5 * (Dc + Dn) * (xn - xc)
    return out / (h * h)


def z_ghosts2(f):
    """f [..., nz, ny, nx] extended by two cell layers below and above in z,
    the linear continuation of the two nearest layers (Sec. 3.5)."""
    d0 = f[..., 1:2, :, :] - f[..., :1, :, :]
    d1 = f[..., -1:, :, :] - f[..., -2:-1, :, :]
    lo = [f[..., :1, :, :] - 2.0 * d0, f[..., :1, :, :] - d0]
    hi = [f[..., -1:, :, :] + d1, f[..., -1:, :, :] + 2.0 * d1]
    return np.concatenate(lo + [f] + hi, axis=-3)


def eno_derivative(g, u, h, axis):
    """Eq. ENO along `axis` of the ghosted array g, whose cells 2 .. n+1 along
    that axis are the interior (two extra cells each side); u is the velocity
    component along the axis at the interior cells.  Upwinded second-order
    one-sided difference where the curvature on the upwind side is smaller,
    the centred difference otherwise."""
    n = g.shape[axis] - 4

    def at(o):  # values at interior offset o (-2 .. 2)
        return np.take(g, np.arange(2 + o, 2 + o + n), axis=axis)

    fm2, fm1, f0, fp1, fp2 = at(-2), at(-1), at(0), at(1), at(2)
    cm = np.abs(f0 - 2.0 * fm1 + fm2)   # |f_xx| at i-1, times h^2
    c0 = np.abs(fp1 - 2.0 * f0 + fm1)   # at i
    cp = np.abs(fp2 - 2.0 * fp1 + f0)   # at i+1
    fwd = -fp2 + 4.0 * fp1 - 3.0 * f0
    bwd = 3.0 * f0 - 4.0 * fm1 + fm2
    ctr = fp1 - fm1
    d = np.where((u < 0.0) & (c0 > cp), fwd, np.where((u > 0.0) & (c0 > cm), bwd, ctr))
    return d / (2.0 * h)


def cell_velocity(v):
    """Velocity at the cell centres: mean of the cell's eight corner nodes."""
    acc = 0.0
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                acc = acc + np.roll(np.roll(v[:, dz:v.shape[1] - 1 + dz], -dy, axis=2), -dx, axis=3)
    return acc / 8.0


def advection(sigma, v, h):
    """(v . grad) sigma at the cells (Eq. sig_star_evol), each component of
    the Voigt stress differentiated by Eq. ENO in x, y and z with the
    velocity at the cell centre; x and y wrap, z uses two extrapolated ghost
    layers."""
    u = cell_velocity(v)
    gz = z_ghosts2(sigma)
    gy = np.concatenate([sigma[..., -2:, :], sigma, sigma[..., :2, :]], axis=-2)
    gx = np.concatenate([sigma[..., -2:], sigma, sigma[..., :2]], axis=-1)
    return (u[0] * eno_derivative(gx, u[0], h, -1) + u[1] * eno_derivative(gy, u[1], h, -2)
            + u[2] * eno_derivative(gz, u[2], h, -3))


def node_laplacian(v, h):
    """Eq. col_snd_deriv summed over x, y and z at the interior nodes (x, y
    wrap; the z neighbours of the first and last interior planes are the
    walls); zero on the wall planes."""
    out = np.zeros_like(v)
    c = v[:, 1:-1]
    lx = np.roll(c, 1, axis=-1) + np.roll(c, -1, axis=-1) - 2.0 * c
    ly = np.roll(c, 1, axis=-2) + np.roll(c, -1, axis=-2) - 2.0 * c
    lz = v[:, 2:] + v[:, :-2] - 2.0 * c
    out[:, 1:-1] = (lx + ly + lz) / (h * h)
    return out


def node_advection(v, h):
    """(v . grad) v at the interior nodes, each component differentiated by
    Eq. ENO along x, y and z with the node's own velocity; x and y wrap, and
    the ghost node beyond a wall is the reflection 2 v_wall - v of the node
    inside it (Sec. 3.5, Dirichlet walls).  Zero on the wall planes."""
    out = np.zeros_like(v)
    c = v[:, 1:-1]
    gx = np.concatenate([c[..., -2:], c, c[..., :2]], axis=-1)
    gy = np.concatenate([c[..., -2:, :], c, c[..., :2, :]], axis=-2)
    gz = np.concatenate([2.0 * v[:, :1] - v[:, 1:2], v, 2.0 * v[:, -1:] - v[:, -2:-1]], axis=1)
    for a in range(3):
        out[a, 1:-1] = (c[0] * eno_derivative(gx[a], c[0], h, -1)
                        + c[1] * eno_derivative(gy[a], c[1], h, -2)
                        + c[2] * eno_derivative(gz[a], c[2], h, -3))
    return out


def explicit_step(v, sigma, chi, h, dt, lam, mu, p, U, rho, kappa):
    """One forward-Euler step of the explicit method (Sec. 3.2), all terms
    from the state of step n:
      v'     = v + dt ((D_h sigma)/rho - (v . grad) v + kappa lap v)   (Eq. vel_evo_exp
               per unit mass: the damping kappa = kappa' h is a kinematic
               viscosity, which makes its units and the stability bound
               dt <= h^2 / (6 kappa) consistent),
      sigma' = sigma* + dt C : sym(G_h v), sigma* the STZ step with the
               advection of Eq. stress_evo_exp (Truesdell term -tr(L) sigma
               as everywhere else),
      chi'   = the chi of the STZ step (Eq. chi_evo_exp);
    walls of v' at (-U, 0, 0) and (+U, 0, 0) (Eq. u_bc)."""
    acc = div_node(sigma, h) / rho - node_advection(v, h) + kappa * node_laplacian(v, h)
    v_next = set_shear_walls(v + dt * acc, U)
    sstar, chi_next = stz_step(v, sigma, chi, h, dt, lam, mu, dict(p, advect=1))
    s_next = stress_update(sstar, v, h, dt, lam, mu)
    return v_next, s_next, chi_next


def chi_diffusion(sigma, chi, h, p):
    """div(D^pl grad chi) per cell for the state (sigma, chi) of step n.
    With p["chi_wall"] = 1 the wall faces carry no flux: the ghost layers
    take the chi of the cell next to them, so the difference across a wall
    face is zero (an extension; see the module's readings)."""
    sg, cg = z_ghosts(sigma), z_ghosts(chi)
    _, sbar = deviator(voigt_to_full(sg))
    pos = np.real(cg) > 0.0
    D = np.where(pos, plastic_rate(sbar, np.where(pos, cg, 1.0), p), 0.0)
    if p.get("chi_wall", 0):
        cg = cg.copy()
        cg[0], cg[-1] = cg[1], cg[-2]
    return flux_divergence(D, cg, h)


def plastic_rate_slope(sbar, chi, p):
    """d D^pl / d sbar of Eq. stz_dpl above yield (0 at or below):
    A (beta sinh(beta sbar) (1 - s_Y/sbar) + cosh(beta sbar) s_Y / sbar^2)
    with A = exp(-1/chi) exp(-Delta/kT) / tau0."""
    act = sbar > p["s_y"]
    sb = np.where(act, sbar, p["s_y"])
    A = np.exp(-1.0 / chi) * np.exp(-p["delta_over_T"]) / p["tau0"]
    bs = p["beta"] * sb
    f = 1.0 - p["s_y"] / sb
    return np.where(act, A * (p["beta"] * np.sinh(bs) * f + np.cosh(bs) * p["s_y"] / (sb * sb)),
                    0.0)


MAX_SUBSTEPS = 65536


def substep_count(sbar, chi, dt, mu, p):
    """Sub-steps of the local plastic relaxation per cell (see stz_pointwise):
    n_sub in {0, 1} gives 1 (the single forward-Euler step of Eq. sig_star_qs),
    n_sub > 1 gives n_sub, and n_sub = -1 gives ceil(4 mu dt dD^pl/dsbar) at
    the state of step n, between 1 and MAX_SUBSTEPS, so that each sub-step
    tau keeps tau 2 mu dD^pl/dsbar <= 1/2 (the explicit step of
    dsbar/dt = -2 mu D^pl is stable below 2 and monotone below 1)."""
    n = int(p.get("n_sub", 1))
    if n == -1:
        m = np.ceil(4.0 * mu * dt * plastic_rate_slope(sbar, chi, p))
        return np.clip(np.nan_to_num(m, nan=MAX_SUBSTEPS), 1, MAX_SUBSTEPS).astype(np.int64)
    return np.full(np.shape(sbar), max(n, 1), dtype=np.int64)


def stz_pointwise(L, sigma, chi, dt, lam, mu, p):
    """The cellwise part of the step: (L, sigma, chi) -> (sigma*, chi').

    L[a, b] = d v_a / d x_b at the cell, sigma in Voigt order.  Implements
    Eq. sig_star_qs and the forward-Euler step of Eq. chi_evo; complex-safe.

    With p["n_sub"] set (see substep_count) a cell may take M > 1 sub-steps
    of tau = dt/M for its plastic terms, an extension beyond the paper: the
    kinematic terms L sigma + sigma L^T - tr(L) sigma are taken once from
    sigma^n, while the relaxation -2 mu (D^pl/sbar) sigma_0 and the growth
    term of chi are stepped M times, each from the state the previous
    sub-step left: sigma* = sigma_M + dt (kinematic terms).  M = 1 is the
    single step of Eq. sig_star_qs.
    """
    if int(p.get("n_sub", 1)) == -2:
        return _stz_pointwise_implicit(L, sigma, chi, dt, lam, mu, p)
    if int(p.get("n_sub", 1)) not in (0, 1):
        return _stz_pointwise_substeps(L, sigma, chi, dt, lam, mu, p)
    S = voigt_to_full(sigma)
    S0, sbar = deviator(S)
    Dpl = plastic_rate(sbar, chi, p)
    act = np.real(Dpl) > 0.0
    ratio = np.where(act, Dpl / np.where(act, sbar, 1.0), 0.0 * Dpl)
    trL = L[0, 0] + L[1, 1] + L[2, 2]
    LS = np.einsum("ab...,bc...->ac...", L, S)
    SLt = np.einsum("ab...,cb...->ac...", S, L)
    plastic = stiffness(ratio * S0, lam, mu)
    Sstar = S + dt * (LS + SLt - trL * S - plastic)
    # D^pl (tensor) : sigma_0 = (D^pl / sbar) sigma_0 : sigma_0 = 2 sbar D^pl
    chi_next = chi + (dt / p["c0"]) * (2.0 * sbar * Dpl / p["s_y"]) * (p["chi_inf"] - chi)
    return full_to_voigt(Sstar), chi_next


IMPLICIT_BISECTIONS = 64


def implicit_sbar(sbar, chi, dt, mu, p):
    """Backward-Euler s of the local relaxation dsbar/dt = -2 mu D^pl(sbar, chi)
    with chi held at step n: the root of g(s) = s - sbar + 2 mu dt D^pl(s, chi)
    in [s_Y, sbar] for sbar > s_Y (g is increasing there, g(s_Y) < 0 <= g(sbar)),
    found by IMPLICIT_BISECTIONS halvings of that interval; sbar itself at or
    below yield."""
    sbar = np.asarray(sbar, dtype=float)
    act = sbar > p["s_y"]
    lo = np.where(act, p["s_y"], sbar)
    hi = sbar.copy()
    for _ in range(IMPLICIT_BISECTIONS):
        mid = 0.5 * (lo + hi)
        g = mid - sbar + 2.0 * mu * dt * plastic_rate(mid, chi, p)
        lo = np.where(act & (g < 0.0), mid, lo)
        hi = np.where(act & (g >= 0.0), mid, hi)
    return np.where(act, hi, sbar)


def _stz_pointwise_implicit(L, sigma, chi, dt, lam, mu, p):
    """n_sub = -2 (an extension, not the paper's): the plastic terms by
    backward Euler.  The deviator keeps its direction and shrinks to the
    implicit_sbar value; the pressure is kept; chi takes
    chi' = (chi + a chi_inf) / (1 + a), a = (dt/c0) 2 s' D^pl(s', chi)/s_Y,
    which stays between chi and chi_inf; the kinematic terms come from
    sigma^n as in the sub-stepped form."""
    S = voigt_to_full(sigma)
    S0, sbar = deviator(S)
    s1 = implicit_sbar(sbar, chi, dt, mu, p)
    scale = np.where(sbar > p["s_y"], s1 / np.where(sbar > 0.0, sbar, 1.0), 1.0)
    Sp = S - (1.0 - scale) * S0
    D1 = plastic_rate(s1, chi, p)
    a = (dt / p["c0"]) * (2.0 * s1 * D1 / p["s_y"])
    chi_next = (chi + a * p["chi_inf"]) / (1.0 + a)
    trL = L[0, 0] + L[1, 1] + L[2, 2]
    kin = (np.einsum("ab...,bc...->ac...", L, S) + np.einsum("ab...,cb...->ac...", S, L)
           - trL * S)
    return full_to_voigt(Sp + dt * kin), chi_next


def _stz_pointwise_substeps(L, sigma, chi, dt, lam, mu, p):
    S = voigt_to_full(sigma)
    _, sbar = deviator(S)
    M = substep_count(sbar, chi, dt, mu, p)
    tau = dt / M
    trL = L[0, 0] + L[1, 1] + L[2, 2]
    kin = (np.einsum("ab...,bc...->ac...", L, S) + np.einsum("ab...,cb...->ac...", S, L)
           - trL * S)
    Sp, xp = S.copy(), np.array(chi, dtype=float)
    for m in range(int(M.max())):
        on = m < M
        S0, sb = deviator(Sp)
        D = plastic_rate(sb, xp, p)
        ratio = np.where(D > 0.0, D / np.where(D > 0.0, sb, 1.0), 0.0)
        Sn = Sp - tau * (2.0 * mu * ratio * S0)
        xn = xp + (tau / p["c0"]) * (2.0 * sb * D / p["s_y"]) * (p["chi_inf"] - xp)
        Sp = np.where(on, Sn, Sp)
        xp = np.where(on, xn, xp)
    return full_to_voigt(Sp + dt * kin), xp


def stz_step(v, sigma, chi, h, dt, lam, mu, p):
    """Intermediate stress (Eq. sig_star_qs) and the updated chi (Eq. chi_evo).

    v: node velocity at step n (walls included), sigma: Voigt cell stress,
    chi: cell effective temperature.  Returns (sigma_star, chi_next).  With
    p["l_diff"] = l > 0 the diffusion term l^2 div(D^pl grad chi) joins the
    chi step; with p["advect"] true the advection -(v . grad) sigma of
    Eq. sig_star_evol (the explicit method's Eq. stress_evo_exp carries it too;
    the quasi-static Eq. sig_star_qs does not) joins sigma*, with v and sigma
    of step n.
    """
    sstar, chi_next = stz_pointwise(grad_cell(v, h), sigma, chi, dt, lam, mu, p)
    if p.get("advect", 0):
        sstar = sstar - dt * advection(sigma, v, h)
    l = p.get("l_diff", 0.0)
    if l > 0.0:
        chi_next = chi_next + (dt / p["c0"]) * (l * l) * chi_diffusion(sigma, chi, h, p)
    return sstar, chi_next


def rhs(sigma_star, h, dt):
    """b = D_h sigma* / dt at the interior nodes (Eq. proj, sign flipped)."""
    return div_node(sigma_star, h) / dt


def stress_update(sigma_star, v, h, dt, lam, mu):
    """sigma^{n+1} = sigma* + dt C : D^{n+1}, D = sym(G_h v^{n+1}) (Eq. sig_n+1)."""
    D = sym(grad_cell(v, h))
    return sigma_star + dt * full_to_voigt(stiffness(D, lam, mu))


def set_shear_walls(v, U):
    """Wall velocities of Eq. u_bc: (-U, 0, 0) at k = 0 and (+U, 0, 0) at k = nz."""
    v = v.copy()
    v[:, 0] = 0.0
    v[:, -1] = 0.0
    v[0, 0] = -U
    v[0, -1] = U
    return v


def set_walls(v, lo, hi):
    """Wall planes k = 0 and k = nz of v replaced by the node data lo, hi
    (each [3, ny, nx])."""
    v = v.copy()
    v[:, 0] = lo
    v[:, -1] = hi
    return v


def projection_step(v, sigma, chi, h, dt, lam, mu, p, U, solver, rtol=1e-10, max_cycles=100,
                    walls=None):
    """One quasi-static step n -> n+1 (Sec. 3.3).

    `solver` is an oracle multigrid (`MGOracle`) for the same grid; the solve
    is warm-started from v^n with the new wall values: those of Eq. u_bc with
    speed U, or, when `walls` = (lo, hi) is given, that node data (e.g. the
    spinning discs of Sec. 5).
    """
    sstar, chi_next = stz_step(v, sigma, chi, h, dt, lam, mu, p)
    b = rhs(sstar, h, dt)
    x0 = set_shear_walls(v, U) if walls is None else set_walls(v, *walls)
    v_next, info = solver.solve(b, x0, rtol=rtol, max_cycles=max_cycles)
    s_next = stress_update(sstar, v_next, h, dt, lam, mu)
    return v_next, s_next, chi_next, info
