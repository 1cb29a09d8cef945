"""Pins of the oracle's reverse mode: dot-product identities and finite differences."""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import stz as ostz
from oracle.multigrid import MGOracle
from oracle.operators import grad_cell, stiffness, sym, voigt_to_full, full_to_voigt
from workloads import chi_field, lame, shear_velocity, stz_constants

LAM, MU = lame()
P = stz_constants()


def _node(rng, n, walls=False):
    v = rng.standard_normal((3, n + 1, n, n))
    if not walls:
        v[:, 0] = 0
        v[:, -1] = 0
    return v


def test_linear_transposes():
    rng = np.random.default_rng(0)
    n, h, dt = 6, 0.3, 0.7
    v = _node(rng, n)
    T = rng.standard_normal((3, 3, n, n, n))
    assert np.isclose(np.sum(grad_cell(v, h) * T), np.sum(v * adj.grad_cell_T(T, h)), rtol=1e-12)
    gb = _node(rng, n)
    s = rng.standard_normal((6, n, n, n))
    assert np.isclose(np.sum(gb * ostz.rhs(s, h, dt)), np.sum(adj.rhs_vjp(gb, h, dt) * s), rtol=1e-12)
    g = rng.standard_normal((6, n, n, n))
    lhs = np.sum(g * (ostz.stress_update(np.zeros_like(g), v, h, dt, LAM, MU)))
    rhs = np.sum(adj.stress_update_vjp(g, h, dt, LAM, MU) * v)
    assert np.isclose(lhs, rhs, rtol=1e-12)


def _active_state(rng, ncell):
    sig = rng.standard_normal((6, ncell))
    S = voigt_to_full(sig)
    S0, sb = ostz.deviator(S)
    sig = sig * (P["s_y"] * rng.uniform(1.02, 1.08, ncell) / sb)
    chi = 0.05 + 0.003 * rng.standard_normal(ncell)
    L = 1e-4 * rng.standard_normal((3, 3, ncell))
    return L, sig, chi


def test_complex_step_vjp_matches_finite_differences():
    rng = np.random.default_rng(1)
    L, sig, chi = _active_state(rng, 50)
    dt = 10.0
    gs = rng.standard_normal((6, 50))
    gc = rng.standard_normal(50)
    gL, gS, gC = adj.stz_pointwise_vjp(L, sig, chi, dt, LAM, MU, P, gs, gc)

    def f(L_, s_, c_):
        a, b = ostz.stz_pointwise(L_, s_, c_, dt, LAM, MU, P)
        return np.sum(gs * a) + np.sum(gc * b)

    for trial in range(3):
        dL = rng.standard_normal(L.shape) * 1e-4
        dS = rng.standard_normal(sig.shape) * P["s_y"]
        dC = rng.standard_normal(chi.shape) * 0.003
        eps = 1e-6
        fd = (f(L + eps * dL, sig + eps * dS, chi + eps * dC)
              - f(L - eps * dL, sig - eps * dS, chi - eps * dC)) / (2 * eps)
        an = np.sum(gL * dL) + np.sum(gS * dS) + np.sum(gC * dC)
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


@pytest.mark.slow
def test_rollout_gradient_matches_finite_differences():
    """Three steps at 8^3 (3 levels) from an actively yielding state."""
    rng = np.random.default_rng(2)
    n, dt, U, steps = 8, 10.0, 1e-5, 3
    h = 1.0 / n
    mg = MGOracle(n, n, n, h, LAM, MU, min_coarse_nz=2)
    v0 = shear_velocity(n, n, n, U)
    s0 = np.zeros((6, n, n, n))
    s0[4] = 1.03 * P["s_y"]
    s0 += 1e-4 * rng.standard_normal(s0.shape)
    c0 = chi_field(n, n, n, 4, lc_cells=2.0)
    loss, g = adj.rollout_grad_chi0(v0, s0, c0, h, dt, LAM, MU, P, U, mg, steps)

    def L(c):
        (v, s, cc), _ = adj.rollout(v0, s0, c, h, dt, LAM, MU, P, U, mg, steps)
        return adj.mid_shear_loss(s)

    for trial in range(2):
        d = rng.standard_normal(c0.shape)
        d /= np.sqrt(np.mean(d * d))
        eps = 1e-6
        fd = (L(c0 + eps * d) - L(c0 - eps * d)) / (2 * eps)
        an = np.sum(g * d)
        assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)
