"""GPU parity of the STZ step, RHS, stress correction and projection step."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import stz as ostz
from oracle.multigrid import MGOracle
from oracle.operators import div_node
from workloads import chi_field, lame, shear_state, stz_constants

pytestmark = pytest.mark.gpu
LAM, MU = lame()
P = stz_constants()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def solver(nx, ny, nz, **kw):
    from paper_1904_03808_amd.qsmg import MGSolver
    return MGSolver(nx, ny, nz, 1.0 / nz, LAM, MU, **kw)


def random_state(rng, nx, ny, nz):
    """Stresses around the yield surface, chi around 0.05, small velocity gradients."""
    sig = rng.standard_normal((6, nz, ny, nx))
    S = sig.copy()
    p = (S[0] + S[1] + S[2]) / 3
    dev_ = S.copy()
    dev_[:3] -= p
    sb = np.sqrt(0.5 * (dev_[0] ** 2 + dev_[1] ** 2 + dev_[2] ** 2
                        + 2 * (dev_[3] ** 2 + dev_[4] ** 2 + dev_[5] ** 2)))
    scale = P["s_y"] * rng.uniform(0.9, 1.1, size=sb.shape) / sb
    sig = sig * scale
    chi = 0.05 + 0.003 * rng.standard_normal((nz, ny, nx))
    v = 1e-4 * rng.standard_normal((3, nz + 1, ny, nx))
    return v, sig, chi


@pytest.mark.parametrize("n", [(16, 16, 16), (24, 20, 20)])
def test_stz_step(n):
    rng = np.random.default_rng(0)
    nx, ny, nz = n
    g = solver(nx, ny, nz)
    v, sig, chi = random_state(rng, nx, ny, nz)
    for dt in (0.5, 10.0):
        ss, c1 = g.stz_step(P, dt, dev(v), dev(sig), dev(chi))
        rs, rc = ostz.stz_step(v, sig, chi, 1.0 / nz, dt, LAM, MU, P)
        assert rel(host(ss), rs) < 1e-12
        assert rel(host(c1) - chi, rc - chi) < 1e-11


@pytest.mark.parametrize("n", [(16, 16, 16), (24, 20, 20)])
def test_rhs_and_stress_update(n):
    rng = np.random.default_rng(1)
    nx, ny, nz = n
    g = solver(nx, ny, nz)
    s = rng.standard_normal((6, nz, ny, nx))
    v = rng.standard_normal((3, nz + 1, ny, nx))
    b = host(g.rhs(dev(s), 0.7))
    assert rel(b, ostz.rhs(s, 1.0 / nz, 0.7)) < 1e-13
    assert np.all(b[:, 0] == 0) and np.all(b[:, -1] == 0)
    out = host(g.stress_update(dev(s), dev(v), 0.3))
    assert rel(out, ostz.stress_update(s, v, 1.0 / nz, 0.3, LAM, MU)) < 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32-ir"])
def test_projection_steps(prec):
    """Three simple-shear steps at 16^3 from a random chi field."""
    n, dt, U = 16, 10.0, 1e-5
    st = shear_state(n, n, n, seed=3, U=U)
    v, sig, chi = st["v"], st["sigma"], st["chi"]
    g = solver(n, n, n, precision=prec)
    o = MGOracle(n, n, n, 1.0 / n, LAM, MU)
    vd, sd, cd = dev(v), dev(sig), dev(chi)
    for step in range(3):
        info = g.projection_step(P, dt, U, vd, sd, cd, rtol=1e-12)
        v, sig, chi, oi = ostz.projection_step(v, sig, chi, 1.0 / n, dt, LAM, MU, P, U, o, rtol=1e-12)
        assert info.converged
        tol = 1e-10
        assert rel(host(vd), v) < tol, step
        assert rel(host(sd), sig) < tol, step
        assert rel(host(cd), chi) < 1e-13, step
