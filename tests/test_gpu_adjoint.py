"""GPU reverse mode (hand-written VJP kernels + transposed solve) against the oracle."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adjoint as adj
from oracle import stz as ostz
from oracle.multigrid import MGOracle
from oracle.operators import grad_cell
from workloads import lame, shear_state, stz_constants

pytestmark = pytest.mark.gpu
LAM, MU = lame()
P = stz_constants()
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def solver(n, **kw):
    from paper_1904_03808_amd.qsmg import MGSolver
    return MGSolver(n, n, n, 1.0 / n, LAM, MU, **kw)


def active_state(rng, n):
    st = shear_state(n, n, n, seed=5)
    s = st["sigma"].copy()
    s[4] = 1.03 * P["s_y"]
    s += 2e-4 * rng.standard_normal(s.shape)
    v = st["v"] + 1e-5 * rng.standard_normal(st["v"].shape)
    return v, s, st["chi"]


def test_vjp_kernels_match_oracle():
    rng = np.random.default_rng(0)
    n, dt = 16, 10.0
    h = 1.0 / n
    g = solver(n)
    v, s, c = active_state(rng, n)
    gs = rng.standard_normal(s.shape)
    gc = rng.standard_normal(c.shape)
    gv = dev(np.zeros_like(v))
    gS, gC = g.stz_step_vjp(P, dt, dev(v), dev(s), dev(c), dev(gs), dev(gc), gv)
    L = grad_cell(v, h)
    rL, rS, rC = adj.stz_pointwise_vjp(L, s, c, dt, LAM, MU, P, gs, gc)
    assert rel(host(gS), rS) < 1e-10
    assert rel(host(gC), rC) < 1e-10
    assert rel(host(gv), adj.grad_cell_T(rL, h)) < 1e-10
    gb = rng.standard_normal(v.shape)
    out = dev(np.zeros_like(s))
    g.rhs_vjp(dev(gb), 0.7, out)
    assert rel(host(out), adj.rhs_vjp(gb, h, 0.7)) < 1e-13
    gv = dev(np.zeros_like(v))
    g.stress_update_vjp(dev(gs), 0.7, gv)
    assert rel(host(gv), adj.stress_update_vjp(gs, h, 0.7, LAM, MU)) < 1e-13


def test_rollout_gradient_matches_oracle():
    """d loss / d chi0 through 3 steps at 16^3: autograd + GPU kernels vs oracle."""
    from paper_1904_03808_amd.autograd import rollout_loss
    n, dt, U, steps = 16, 10.0, 1e-5, 3
    h = 1.0 / n
    st = shear_state(n, n, n, seed=4, U=U)
    s0 = st["sigma"].copy()
    s0[4] = 1.01 * P["s_y"]
    g = solver(n)
    chi = dev(st["chi"]).requires_grad_(True)
    loss = rollout_loss(chi, dev(st["v"]), dev(s0), g, P, dt, U, steps, rtol=1e-13)
    loss.backward()
    o = MGOracle(n, n, n, h, LAM, MU)
    rloss, rg = adj.rollout_grad_chi0(st["v"], s0, st["chi"], h, dt, LAM, MU, P, U, o, steps)
    assert abs(loss.item() - rloss) <= 1e-12 * rloss
    assert rel(host(chi.grad), rg) < 1e-8


def _config4(n=96, steps=10):
    st = shear_state(n, n, n, seed=4, U=1e-5)
    return st, 10.0, 1e-5, steps


def test_adjoint_config_96_finite_differences_and_oracle():
    """96^3, 10 steps: gradient vs central differences on 16 directions and,
    when its file is present, vs the stored oracle gradient."""
    from paper_1904_03808_amd.autograd import rollout_loss
    n = 96
    st, dt, U, steps = _config4(n)
    g = solver(n)
    v0, s0, c0 = dev(st["v"]), dev(st["sigma"]), dev(st["chi"])
    # fixed 40-cycle solves (converged to rounding): a residual-based stop
    # would add noise of order cond(K) * rtol to every finite difference
    chi = c0.clone().requires_grad_(True)
    loss = rollout_loss(chi, v0, s0, g, P, dt, U, steps, rtol=0.0, max_cycles=40)
    loss.backward()
    grad = host(chi.grad)

    def L(c):
        with torch.no_grad():
            return rollout_loss(c, v0, s0, g, P, dt, U, steps, rtol=0.0, max_cycles=40).item()

    # The map is only piecewise smooth: about 1e-5 of the cells cross the yield
    # surface sbar = s_Y during the 10 steps (hot spots of chi overshoot under
    # forward Euler), so the step must stay below the distance to those kinks.
    # eps = 1e-8 does; rounding then bounds the difference quotient error by
    # about 40 u L / eps (u = 1.1e-16).
    eps = 1e-8
    an, fd = [], []
    for seed in range(100, 116):
        d = np.random.default_rng(seed).standard_normal(grad.shape)
        d /= np.sqrt(np.mean(d * d))
        dd = dev(d)
        fd.append((L(c0 + eps * dd) - L(c0 - eps * dd)) / (2 * eps))
        an.append(float(np.sum(grad * d)))
    an, fd = np.array(an), np.array(fd)
    atol = 40 * 1.1e-16 * loss.item() / eps
    assert np.all(np.abs(fd - an) <= 1e-5 * np.abs(an) + atol), (np.abs(fd - an), np.abs(an), atol)
    path = os.path.join(GOLDEN, "adjoint96.json")
    if os.path.exists(path):
        ref = json.load(open(path))
        assert abs(loss.item() - ref["loss"]) <= 1e-11 * ref["loss"]
        assert np.allclose(an, ref["dir_derivs"], rtol=1e-8, atol=0)
        samp = np.array([grad[tuple(i)] for i in ref["sample_index"]])
        assert np.abs(samp - np.array(ref["sample_grad"])).max() <= 1e-8 * ref["grad_rms"]
