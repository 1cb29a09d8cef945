"""Input generators: the device version of the smoothed random stress follows
the host recipe exactly when given the same random numbers."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W


def test_device_stress_recipe_matches_host_recipe():
    gen = torch.Generator()
    gen.manual_seed(5)
    draws = torch.randn((6, 6, 8, 10), generator=gen, dtype=torch.float64).numpy()
    dev = W.stress_field_device(10, 8, 6, 5, "cpu").numpy()
    # the host recipe (face-mean Jacobi, periodic x/y, linear z ghosts) on the same draws
    s = draws.copy()
    for _ in range(3):
        lo, hi = 2 * s[:, 0] - s[:, 1], 2 * s[:, -1] - s[:, -2]
        zp = np.concatenate([s[:, 1:], hi[:, None]], axis=1)
        zm = np.concatenate([lo[:, None], s[:, :-1]], axis=1)
        s = (np.roll(s, 1, -1) + np.roll(s, -1, -1) + np.roll(s, 1, -2) + np.roll(s, -1, -2)
             + zp + zm) / 6.0
    assert np.abs(dev - s).max() == 0.0
    # and the host generator is that recipe on numpy's draws
    host = W.stress_field(10, 8, 6, 5)
    assert host.shape == dev.shape and np.isfinite(host).all()
    assert abs(host.std() - dev.std()) < 0.2


def test_defect_chi_follows_eq_case0_chi():
    """Eq. case0_chi on the paper's N x N x N/2 grid shape: the defect sits at
    the sample's centre, so the field is mirror-symmetric in every direction;
    the cells next to the centre (distance h sqrt(3)/2 from it) carry the
    largest value, and far from it the field falls to 550 K."""
    nx, ny, nz = 32, 32, 16
    chi = W.defect_chi(nx, ny, nz) * 21000.0
    assert chi.shape == (nz, ny, nx)
    assert np.array_equal(chi, chi[::-1]) and np.array_equal(chi, chi[:, ::-1])
    assert np.array_equal(chi, chi[:, :, ::-1])
    h = 1.0 / nz
    top = 550.0 + 170.0 * np.exp(-200.0 * 3 * (h / 2) ** 2)
    assert np.isclose(chi.max(), top, rtol=0, atol=1e-12)
    assert np.array_equal(np.argwhere(chi == chi.max()).min(0), [nz // 2 - 1, ny // 2 - 1, nx // 2 - 1])
    # the corner cell: |x|^2 = (L - h/2)^2 + 2 (2L/2 - h/2)^2 with L = 1
    corner = 550.0 + 170.0 * np.exp(-200.0 * ((0.5 - h / 2) ** 2 + 2 * (1.0 - h / 2) ** 2))
    assert np.isclose(chi[0, 0, 0], corner, rtol=1e-14) and chi[0, 0, 0] - 550.0 < 1e-40
    st = W.defect_state(nx, ny, nz)
    assert not st["v"].any() and not st["sigma"].any()


def test_weld_walls_follow_the_spinning_disc():
    """Sec. 5: inside the disc r < R the wall moves as a rigid rotation about
    the centre (tangential, |u| = omega r, no divergence); the profile is
    continuous at r = R and falls to 10 % a quarter of the way, in r^2, from
    the disc's edge to the sample's edge (the property that fixes lambda_w);
    w = 0; only the welded walls move."""
    R = 1.0 / 3.0
    assert np.isclose(W.weld_factor(np.array(R * R + (1 - R * R) / 4), R), 0.1, rtol=1e-14)
    assert np.isclose(W.weld_factor(np.array(R * R * (1 + 1e-12)), R), 1.0, rtol=1e-9)
    nx, ny, nz, omega = 64, 64, 16, 2e-3
    h = 2.0 / nx
    lo, hi = W.weld_walls(nx, ny, nz, omega, h)
    assert not lo.any() and not hi[2].any()
    x = np.arange(nx) * h - 1.0
    X, Y = np.meshgrid(x, x)
    r2 = X * X + Y * Y
    inside = r2 < R * R
    assert inside.sum() > 100
    u, v = hi[0], hi[1]
    assert np.abs(u * X + v * Y)[inside].max() <= 1e-18
    assert np.allclose(np.hypot(u, v)[inside], omega * np.sqrt(r2[inside]), rtol=1e-13)
    # discrete divergence of the rigid rotation (central differences) inside
    du = (np.roll(u, -1, 1) - np.roll(u, 1, 1)) / (2 * h)
    dv = (np.roll(v, -1, 0) - np.roll(v, 1, 0)) / (2 * h)
    core = (r2 < (R - 2 * h) ** 2)
    assert np.abs(du + dv)[core].max() <= 1e-15
    # the profile outside is the same for u and v, and below 1
    f = np.hypot(u, v) / (omega * np.sqrt(np.maximum(r2, 1e-300)))
    assert np.all(f[~inside] < 1.0) and np.all(f[~inside] > 0.0)
    lo2, hi2 = W.weld_walls(nx, ny, nz, omega, h, top=True, bottom=True)
    assert np.array_equal(lo2, hi2) and np.array_equal(hi2, hi)


def test_cylinder_chi_follows_the_inclusion():
    """Sec. 4.1: 800 K on the cylinder's axis (limit at the centre cells),
    600 K outside |x| < L/2 and far from the axis; constant along x inside;
    mirror-symmetric in y and z."""
    nx, ny, nz = 64, 64, 32
    chi = W.cylinder_chi(nx, ny, nz) * 21000.0
    h = 1.0 / nz
    xc = (np.arange(nx) + 0.5 - nx / 2) * h
    inside = np.abs(xc) < 0.5
    assert np.all(chi[:, :, ~inside] == 600.0)
    assert np.all(chi[:, :, inside] == chi[:, :, inside][:, :, :1])
    top = 600.0 + 200.0 * np.exp(-500.0 * 2 * (h / 2) ** 2)
    assert np.isclose(chi.max(), top, rtol=1e-14)
    assert np.array_equal(chi, chi[::-1]) and np.array_equal(chi, chi[:, ::-1])
    assert chi[0, 0, nx // 2] - 600.0 < 1e-9


def test_helix_chi_follows_eq_case12_chi():
    """Eq. case12_chi: in every y-row of cells the field peaks where x and z
    are nearest the helix centre line (cos(6 pi (y+1))/8 - 1/16,
    sin(4 pi (y+1))/8 - 1/16), falls to 550 K far from it, and repeats in y
    with the periods 1/3 (x offset) and 1/2 (z offset), so with period 1 on
    the sample's y range [-1, 1)."""
    nx, ny, nz = 64, 64, 32
    chi = W.helix_chi(nx, ny, nz) * 21000.0
    h = 1.0 / nz
    c = lambda n: (np.arange(n) + 0.5 - n / 2) * h
    xc, yc, zc = c(nx), c(ny), c(nz)
    for jj in (0, 17, 40):
        k, i = np.unravel_index(np.argmax(chi[:, jj, :]), (nz, nx))
        x0 = np.cos(6 * np.pi * (yc[jj] + 1)) / 8 - 1 / 16
        z0 = np.sin(4 * np.pi * (yc[jj] + 1)) / 8 - 1 / 16
        assert abs(xc[i] - x0) <= h / 2 + 1e-12 and abs(zc[k] - z0) <= h / 2 + 1e-12
    assert np.allclose(chi[:, :ny // 2], chi[:, ny // 2:], rtol=1e-13)
    assert chi.min() >= 550.0 and chi.min() - 550.0 < 1e-6 and chi.max() <= 750.0
