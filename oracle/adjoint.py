"""Reverse-mode derivative of a sequence of quasi-static projection steps.

The forward map of one step (Sec. 3.3) is
    L     = G_h v^n                                 (Eq. stag_stenc)
    (s*, chi^{n+1}) = stz_pointwise(L, s^n, chi^n)  (Eqs. sig_star_qs, chi_evo)
    v^{n+1}_I = K_II^{-1} (D_h s* / dt - K_IB v_B)  (Eq. proj)
    s^{n+1} = s* + dt C : sym(G_h v^{n+1})          (Eq. sig_n+1)
Its reverse mode needs
  * the Jacobian of the cellwise map, obtained here by the complex-step
    method (one complex evaluation per input component, exact to rounding),
    so no derivative of the STZ formulas is written by hand;
  * the transposes of the linear maps: G_h^T = -D_h on full tensors with
    zero walls (summation by parts), D_h^T likewise, K^T = K.
Cotangents are derivatives with respect to the stored numbers (Euclidean
inner product on the arrays; a Voigt off-diagonal is one entry).
"""
from __future__ import annotations

import numpy as np

from .operators import _node_diff, full_to_voigt, grad_cell, stiffness, voigt_to_full, VOIGT
from .stz import projection_step, stz_pointwise

CS_STEP = 1e-30


def div_node_full(T: np.ndarray, h: float) -> np.ndarray:
    """(D_h T)_a = sum_b d_b T_ab at interior nodes for a full (3, 3, cells) tensor."""
    nz, ny, nx = T.shape[2:]
    out = np.zeros((3, nz + 1, ny, nx))
    for a in range(3):
        out[a, 1:nz] = sum(_node_diff(T[a, b], b, h) for b in range(3))
    return out


def grad_cell_T(gL: np.ndarray, h: float) -> np.ndarray:
    """G_h^T gL on the interior nodes (wall entries zero)."""
    return -div_node_full(gL, h)


def voigt_cotangent_to_tensor(g: np.ndarray) -> np.ndarray:
    """W with W : X = sum_n g_n X_n for every symmetric X stored in Voigt form."""
    W = np.zeros((3, 3) + g.shape[1:])
    for n, (a, b) in enumerate(VOIGT):
        if a == b:
            W[a, a] = g[n]
        else:
            W[a, b] = 0.5 * g[n]
            W[b, a] = 0.5 * g[n]
    return W


def rhs_vjp(g_b: np.ndarray, h: float, dt: float) -> np.ndarray:
    """Cotangent of s* for b = D_h s* / dt (walls of g_b ignored)."""
    g = g_b.copy()
    g[:, 0] = 0.0
    g[:, -1] = 0.0
    G = grad_cell(g, h)  # <g, D_h T> = -<G_h g, T> for any full tensor T
    out = np.empty((6,) + G.shape[2:])
    for n, (a, b) in enumerate(VOIGT):
        out[n] = -(G[a, a] if a == b else G[a, b] + G[b, a]) / dt
    return out


def stress_update_vjp(g_sigma: np.ndarray, h: float, dt: float, lam: float, mu: float) -> np.ndarray:
    """Cotangent of v (interior) for s_out = s* + dt C : sym(G_h v)."""
    W = voigt_cotangent_to_tensor(g_sigma)
    return dt * grad_cell_T(stiffness(W, lam, mu), h)


def stz_pointwise_vjp(L, sigma, chi, dt, lam, mu, p, g_sstar, g_chi1):
    """(g_L, g_sigma, g_chi) = J^T (g_sstar, g_chi1) by complex steps."""
    g_L = np.zeros_like(L)
    g_sigma = np.zeros_like(sigma)

    def contract(out):
        s_out, c_out = out
        return np.sum(g_sstar * s_out.imag, axis=0) / CS_STEP + g_chi1 * c_out.imag / CS_STEP

    for a in range(3):
        for b in range(3):
            Lc = L.astype(np.complex128)
            Lc[a, b] += 1j * CS_STEP
            g_L[a, b] = contract(stz_pointwise(Lc, sigma, chi, dt, lam, mu, p))
    for n in range(6):
        sc = sigma.astype(np.complex128)
        sc[n] += 1j * CS_STEP
        g_sigma[n] = contract(stz_pointwise(L, sc, chi, dt, lam, mu, p))
    g_chi = contract(stz_pointwise(L, sigma, chi + 1j * CS_STEP, dt, lam, mu, p))
    return g_L, g_sigma, g_chi


def mid_shear_loss(sigma: np.ndarray) -> float:
    """Mean of sigma_xz^2 over the two cell layers next to the plane z = 1/2."""
    nz = sigma.shape[1]
    s = sigma[4, nz // 2 - 1: nz // 2 + 1]
    return float(np.mean(s * s))


def mid_shear_loss_grad(sigma: np.ndarray) -> np.ndarray:
    nz = sigma.shape[1]
    g = np.zeros_like(sigma)
    s = sigma[4, nz // 2 - 1: nz // 2 + 1]
    g[4, nz // 2 - 1: nz // 2 + 1] = 2.0 * s / s.size
    return g


def rollout(v0, s0, chi0, h, dt, lam, mu, p, U, solver, nsteps, rtol=1e-13, max_cycles=200):
    """nsteps projection steps; returns the final state and per-step checkpoints.

    rtol <= 0 runs every solve for exactly max_cycles cycles.
    """
    v, s, c = v0.copy(), s0.copy(), chi0.copy()
    ckpt = []
    for _ in range(nsteps):
        ckpt.append((v, s, c))
        v, s, c, _ = projection_step(v, s, c, h, dt, lam, mu, p, U, solver, rtol=rtol,
                                     max_cycles=max_cycles)
    return (v, s, c), ckpt


def rollout_grad_chi0(v0, s0, chi0, h, dt, lam, mu, p, U, solver, nsteps, rtol=1e-13,
                      max_cycles=200):
    """d(mid_shear_loss(s^N)) / d chi^0 by a reverse sweep over the checkpoints."""
    (vN, sN, cN), ckpt = rollout(v0, s0, chi0, h, dt, lam, mu, p, U, solver, nsteps, rtol,
                                 max_cycles)
    g_s = mid_shear_loss_grad(sN)
    g_c = np.zeros_like(chi0)
    g_v = np.zeros_like(v0)  # cotangent of v^{n+1} (interior)
    for n in reversed(range(nsteps)):
        vn, sn, cn = ckpt[n]
        # s^{n+1} = s* + dt C : sym(G_h v^{n+1})
        g_sstar = g_s.copy()
        g_v = g_v + stress_update_vjp(g_s, h, dt, lam, mu)
        # v^{n+1}_I = K_II^{-1}(D_h s*/dt - ...): adjoint solve with K^T = K
        g_v[:, 0] = 0.0
        g_v[:, -1] = 0.0
        lam_v, _ = solver.solve(g_v, np.zeros_like(g_v), rtol=rtol, max_cycles=max_cycles)
        g_sstar = g_sstar + rhs_vjp(lam_v, h, dt)
        # cellwise STZ map
        L = grad_cell(vn, h)
        gL, g_s, g_c = stz_pointwise_vjp(L, sn, cn, dt, lam, mu, p, g_sstar, g_c)
        g_v = grad_cell_T(gL, h)  # cotangent of v^n (its walls are boundary data)
    return mid_shear_loss(sN), g_c
