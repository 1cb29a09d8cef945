"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only *generates* inputs: material constants converted from the
paper's Table 1, random fields, a manufactured velocity with its analytic
source term, and the simple-shear initial state.  It holds none of the
discrete method's arithmetic (no staggered differences, no multigrid, no STZ
update); both the oracle and the GPU path receive what it returns as plain
arrays and numbers.

Array layouts (all float64, C order):
  node vector   (3, nz+1, ny, nx)   components (x, y, z); node k=0 and k=nz
                                    are the two Dirichlet walls
  cell tensor   (6, nz, ny, nx)     Voigt order (xx, yy, zz, yz, xz, xy)
  cell scalar   (nz, ny, nx)
Node (i, j, k) sits at (i h, j h, k h) with h = 1/nz; cell (i, j, k) has its
lower corner at node (i, j, k) (paper Sec. 3.5).  x and y are periodic.
"""
from __future__ import annotations

import math

import numpy as np

VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def lame(E: float = 1.0, nu: float = 0.35) -> tuple[float, float]:
    """Lame parameters of the isotropic stiffness tensor (paper Sec. 2.1, Eq. lnr_elas)."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def stz_constants(E_Pa=101e9, nu=0.35, rho=6125.0, sY_Pa=0.85e9, tau0_s=1e-13,
                  eps0=0.3, c0=0.4, Delta_K=8000.0, Omega_m3=300e-30, T_K=400.0,
                  chi_inf_K=900.0, ez_K=21000.0, L_m=0.01) -> dict:
    """Table 1 constants in units of stress E, time t_s = L/c_s and length L.

    chi is measured in units of e_z/k_B, so exp(-e_z/(k_B chi)) = exp(-1/chi).
    beta multiplies the nondimensional deviatoric stress measure inside cosh
    (Eq. stz_C_form): Omega eps0 E / (k_B T).
    """
    kB = 1.380649e-23
    mu_Pa = E_Pa / (2.0 * (1.0 + nu))
    c_s = math.sqrt(mu_Pa / rho)
    t_s = L_m / c_s
    return dict(
        s_y=sY_Pa / E_Pa,
        tau0=tau0_s / t_s,
        beta=Omega_m3 * eps0 * E_Pa / (kB * T_K),
        delta_over_T=Delta_K / T_K,
        c0=c0,
        chi_inf=chi_inf_K / ez_K,
    )


def _periodic_conv_fft(a: np.ndarray, taps: np.ndarray, axis: int) -> np.ndarray:
    """Circular convolution of `a` along `axis` with centred taps (wrapped)."""
    n = a.shape[axis]
    R = (len(taps) - 1) // 2
    k = np.zeros(n)
    for d in range(-R, R + 1):
        k[d % n] += taps[d + R]
    fa = np.fft.rfft(a, axis=axis)
    shape = [1] * a.ndim
    shape[axis] = fa.shape[axis]
    fk = np.fft.rfft(k).reshape(shape)
    return np.fft.irfft(fa * fk, n=n, axis=axis)


def stress_field(nx: int, ny: int, nz: int, seed: int, jacobi_passes: int = 3) -> np.ndarray:
    """Smoothed random symmetric cell stress (6, nz, ny, nx).

    i.i.d. N(0,1) Voigt components, then `jacobi_passes` passes of
    u <- mean of the 6 face neighbours; x, y wrap periodically and the z
    ghost layers are linear extrapolations of the two nearest layers
    (paper Sec. 4, grid-setup figure).
    """
    if nz < 2:
        raise ValueError("nz must be >= 2")
    s = np.random.default_rng(seed).standard_normal((6, nz, ny, nx))
    for _ in range(jacobi_passes):
        lo = 2.0 * s[:, 0] - s[:, 1]
        hi = 2.0 * s[:, -1] - s[:, -2]
        zp = np.concatenate([s[:, 1:], hi[:, None]], axis=1)
        zm = np.concatenate([lo[:, None], s[:, :-1]], axis=1)
        s = (np.roll(s, 1, -1) + np.roll(s, -1, -1) + np.roll(s, 1, -2)
             + np.roll(s, -1, -2) + zp + zm) / 6.0
    return np.ascontiguousarray(s)


def stress_field_device(nx: int, ny: int, nz: int, seed: int, device, jacobi_passes: int = 3):
    """The recipe of `stress_field` generated on a torch device (for grids where
    the host version takes minutes): i.i.d. N(0,1) Voigt components from a
    seeded torch generator (so other numbers than `stress_field` draws), then
    the same face-mean Jacobi passes, periodic in x and y, with linearly
    extrapolated z ghost layers.  Returns a float64 tensor (6, nz, ny, nx)."""
    import torch
    if nz < 2:
        raise ValueError("nz must be >= 2")
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    s = torch.randn((6, nz, ny, nx), generator=gen, dtype=torch.float64, device=device)
    for _ in range(jacobi_passes):
        acc = torch.roll(s, 1, -1) + torch.roll(s, -1, -1)
        acc += torch.roll(s, 1, -2)
        acc += torch.roll(s, -1, -2)
        acc[:, :-1] += s[:, 1:]
        acc[:, -1] += 2.0 * s[:, -1] - s[:, -2]
        acc[:, 1:] += s[:, :-1]
        acc[:, 0] += 2.0 * s[:, 0] - s[:, 1]
        s = acc / 6.0
        del acc
    return s.contiguous()


def chi_field(nx: int, ny: int, nz: int, seed: int, mean: float = 0.05,
              std: float = 0.003, lc_cells: float = 8.0, cutoff: float = 5.0) -> np.ndarray:
    """Gaussian random effective-temperature field on cells (paper Eq. convolve).

    White noise on the cells plus a ghost shell in z of ceil(cutoff*l_c) layers
    (x, y wrap, so their ghosts are periodic images) is convolved with the
    truncated separable kernel exp(-|r|^2/l_c^2), |r_a| <= ceil(cutoff*l_c),
    and scaled by std/N with N = sqrt(sum of squared kernel weights), which
    keeps the pointwise variance at std^2.
    """
    R = int(math.ceil(cutoff * lc_cells))
    offs = np.arange(-R, R + 1, dtype=np.float64)
    g = np.exp(-offs ** 2 / lc_cells ** 2)
    norm = math.sqrt(float((g ** 2).sum()) ** 3)
    noise = np.random.default_rng(seed).standard_normal((nz + 2 * R, ny, nx))
    w = _periodic_conv_fft(noise, g, axis=2)
    w = _periodic_conv_fft(w, g, axis=1)
    # linear ('valid') convolution in z over the ghost shell
    nzt = nz + 2 * R
    L = nzt + 2 * R + 1
    fz = np.fft.rfft(w, n=L, axis=0)
    fk = np.fft.rfft(g, n=L).reshape(-1, 1, 1)
    full = np.fft.irfft(fz * fk, n=L, axis=0)
    out = full[2 * R: 2 * R + nz]
    return np.ascontiguousarray(mean + std * out / norm)


def defect_chi(nx: int, ny: int, nz: int, base_K: float = 550.0, amp_K: float = 170.0,
               width: float = 200.0, ez_K: float = 21000.0) -> np.ndarray:
    """Single Gaussian defect of higher effective temperature at the centre of
    the sample (paper Sec. 4.4, Eq. case0_chi): base + amp exp(-width |x|^2/L^2)
    in kelvin, converted to units of e_z/k_B.  The sample spans nx h by ny h by
    nz h with h = 1/nz, so L = nz h (the paper's 2L x 2L x L sample on an
    N x N x N/2 grid when nx = ny = 2 nz); |x| is measured from the sample's
    centre to the cell centres."""
    h = 1.0 / nz
    zc = (np.arange(nz) + 0.5 - 0.5 * nz) * h
    yc = (np.arange(ny) + 0.5 - 0.5 * ny) * h
    xc = (np.arange(nx) + 0.5 - 0.5 * nx) * h
    r2 = zc[:, None, None] ** 2 + yc[None, :, None] ** 2 + xc[None, None, :] ** 2
    return (base_K + amp_K * np.exp(-width * r2)) / ez_K


# ---------------------------------------------------------------------------
# Manufactured velocity: periodic sin/cos in x, y, polynomial in z vanishing
# at both walls.  f = -div(C : grad u) is its exact (continuous) source term.
# ---------------------------------------------------------------------------

def _mms_coords(nx, ny, nz):
    if not (nx == ny == nz):
        raise ValueError("manufactured field needs a cubic grid (period 1 in x, y)")
    h = 1.0 / nz
    z = (np.arange(nz + 1) * h)[:, None, None]
    y = (np.arange(ny) * h)[None, :, None]
    x = (np.arange(nx) * h)[None, None, :]
    return x, y, z


def manufactured_velocity(nx: int, ny: int, nz: int) -> np.ndarray:
    x, y, z = _mms_coords(nx, ny, nz)
    tp = 2.0 * np.pi
    u = np.empty((3, nz + 1, ny, nx))
    u[0] = np.sin(tp * x) * np.cos(tp * y) * (z - z ** 2)
    u[1] = np.cos(tp * x) * np.sin(2 * tp * y) * (z - z ** 3)
    u[2] = np.sin(tp * (x + y)) * (z ** 2 - z ** 3)
    return u


def manufactured_source(nx: int, ny: int, nz: int, lam: float, mu: float) -> np.ndarray:
    """Exact f = -[(lam+mu) grad(div u) + mu lap u] at the nodes; walls zero."""
    x, y, z = _mms_coords(nx, ny, nz)
    pi = np.pi
    tp = 2 * pi
    Sx, Cx = np.sin(tp * x), np.cos(tp * x)
    Sy, Cy = np.sin(tp * y), np.cos(tp * y)
    S2y, C2y = np.sin(2 * tp * y), np.cos(2 * tp * y)
    Sxy, Cxy = np.sin(tp * (x + y)), np.cos(tp * (x + y))
    p, dp, ddp = z - z ** 2, 1 - 2 * z, -2.0 + 0 * z
    q, dq, ddq = z - z ** 3, 1 - 3 * z ** 2, -6 * z
    r, dr, ddr = z ** 2 - z ** 3, 2 * z - 3 * z ** 2, 2 - 6 * z
    lap_u = Sx * Cy * (-2 * tp ** 2 * p + ddp)
    lap_v = Cx * S2y * (-(tp ** 2 + (2 * tp) ** 2) * q + ddq)
    lap_w = Sxy * (-2 * tp ** 2 * r + ddr)
    # div u = tp Cx Cy p + 2tp Cx C2y q + Sxy dr
    gdx = -tp ** 2 * Sx * Cy * p - 2 * tp ** 2 * Sx * C2y * q + tp * Cxy * dr
    gdy = -tp ** 2 * Cx * Sy * p - (2 * tp) ** 2 * Cx * S2y * q + tp * Cxy * dr
    gdz = tp * Cx * Cy * dp + 2 * tp * Cx * C2y * dq + Sxy * ddr
    f = np.zeros((3, nz + 1, ny, nx))
    for c, (gd, lp) in enumerate(((gdx, lap_u), (gdy, lap_v), (gdz, lap_w))):
        f[c] = -((lam + mu) * gd + mu * lp)
    f[:, 0] = 0.0
    f[:, nz] = 0.0
    return f


# ---------------------------------------------------------------------------
# Simple-shear initial state (paper Sec. 4, Eq. u_bc): walls at z = 0 and
# z = 1 move with -U and +U in x; linear velocity profile between them.
# ---------------------------------------------------------------------------

def shear_velocity(nx: int, ny: int, nz: int, U: float) -> np.ndarray:
    v = np.zeros((3, nz + 1, ny, nx))
    zk = np.arange(nz + 1) / nz
    v[0] = (U * (2.0 * zk - 1.0))[:, None, None]
    return v


def cylinder_chi(nx: int, ny: int, nz: int, ez_K: float = 21000.0) -> np.ndarray:
    """The finite cylindrical inclusion of the explicit-versus-quasi-static
    comparison (paper Sec. 4.1): 600 K + 200 K exp(-500 (y^2 + z^2)/L^2) where
    |x| < L/2, 600 K elsewhere, in units of e_z/k_B; coordinates of the cell
    centres from the sample's centre, h = 1/nz, L = nz h."""
    h = 1.0 / nz
    zc = (np.arange(nz) + 0.5 - 0.5 * nz) * h
    yc = (np.arange(ny) + 0.5 - 0.5 * ny) * h
    xc = (np.arange(nx) + 0.5 - 0.5 * nx) * h
    r2 = zc[:, None, None] ** 2 + yc[None, :, None] ** 2 + 0.0 * xc[None, None, :]
    inside = np.abs(xc)[None, None, :] < 0.5
    return (600.0 + np.where(inside, 200.0 * np.exp(-500.0 * r2), 0.0)) / ez_K


def helix_chi(nx: int, ny: int, nz: int, ez_K: float = 21000.0) -> np.ndarray:
    """The non-commensurate helix of the weak-scaling runs (paper Sec. 4.3,
    Eq. case12_chi): 550 K + 200 K exp(-750 (dx^2 + dz^2)) with
    dx = x/L - (cos(6 pi (y/L + 1))/8 - 1/16) and
    dz = z/L - (sin(4 pi (y/L + 1))/8 - 1/16), coordinates of the cell centres
    from the sample's centre, h = 1/nz, L = nz h; units of e_z/k_B."""
    h = 1.0 / nz
    zc = (np.arange(nz) + 0.5 - 0.5 * nz) * h
    yc = (np.arange(ny) + 0.5 - 0.5 * ny) * h
    xc = (np.arange(nx) + 0.5 - 0.5 * nx) * h
    dx = xc[None, None, :] - (np.cos(6 * np.pi * (yc + 1)) / 8 - 1.0 / 16)[None, :, None]
    dz = zc[:, None, None] - (np.sin(4 * np.pi * (yc + 1)) / 8 - 1.0 / 16)[None, :, None]
    return (550.0 + 200.0 * np.exp(-750.0 * (dx * dx + dz * dz))) / ez_K


def defect_state(nx: int, ny: int, nz: int, U: float = 1e-7) -> dict:
    """Initial (v, sigma, chi) of the single-defect run (paper Sec. 4.4): the
    sample at rest and free of stress, chi from Eq. case0_chi.  The wall speed
    ramps up over the first t_s (Eq. u_bc), so at t = 0 the walls are still."""
    return dict(v=shear_velocity(nx, ny, nz, 0.0), sigma=np.zeros((6, nz, ny, nx)),
                chi=defect_chi(nx, ny, nz))


def weld_factor(r2: np.ndarray, R: float = 1.0 / 3.0) -> np.ndarray:
    """Radial profile of the spinning disc (paper Sec. 5, Eqs. u_weld and
    v_weld): 1 inside r^2 < R^2, exp(-lambda_w (r^2 - R^2)^2) outside, with
    lambda_w = 16 ln(10) / (1 - R^2)^2."""
    lam_w = 16.0 * math.log(10.0) / (1.0 - R * R) ** 2
    return np.where(r2 < R * R, 1.0, np.exp(-lam_w * (r2 - R * R) ** 2))


def weld_walls(nx: int, ny: int, nz: int, omega: float, h: float, top: bool = True,
               bottom: bool = False, R: float = 1.0 / 3.0) -> tuple[np.ndarray, np.ndarray]:
    """Wall velocities (lo, hi), each (3, ny, nx), of the friction-welding
    runs (paper Sec. 5): a disc spinning about the z axis through the centre
    of the wall at angular speed omega, (u, v, w) = f(r^2) omega (-y, x, 0)
    with (x, y) measured from the centre in units of L = 1 and f the profile
    of `weld_factor`; the welded walls carry it (the same omega on both when
    both are welded), a wall that is not welded stays still.  Nodes sit at
    (i h, j h), so the centre is at (nx h / 2, ny h / 2)."""
    x = np.arange(nx) * h - 0.5 * nx * h
    y = np.arange(ny) * h - 0.5 * ny * h
    X, Y = np.meshgrid(x, y)
    f = weld_factor(X * X + Y * Y, R)
    disc = np.stack([-omega * f * Y, omega * f * X, np.zeros_like(X)])
    still = np.zeros((3, ny, nx))
    return (disc.copy() if bottom else still), (disc if top else still.copy())


def shear_state(nx: int, ny: int, nz: int, seed: int, U: float = 1e-5,
                s0_frac: float = 0.99, chi_mean: float = 0.05, chi_std: float = 0.003,
                lc_cells: float = 8.0) -> dict:
    """Initial (v, sigma, chi) for the simple-shear runs: uniform sigma_xz."""
    c = stz_constants()
    sigma = np.zeros((6, nz, ny, nx))
    sigma[4] = s0_frac * c["s_y"]
    return dict(v=shear_velocity(nx, ny, nz, U), sigma=sigma,
                chi=chi_field(nx, ny, nz, seed, chi_mean, chi_std, lc_cells))
