"""The allocation-free projection step (qs_projection_step_noalloc) against
qs_projection_step, through the C ABI: same handle state, same inputs, two
calls in a row, the second on a smaller grid; results must be identical
(both run the same kernels, only the step scratch differs)."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1904_03808_amd import _capi  # noqa: E402
from paper_1904_03808_amd.qsmg import MGSolver, _ptr, _stz  # noqa: E402
from workloads import lame, shear_state, stz_constants  # noqa: E402

LAM, MU = lame()
P = stz_constants()


def _step(g, entry, p, dt, U, v, s, c, rtol):
    sp = _stz(p, dt)
    info = _capi.QSSolveInfo()
    args = [g._h, C.byref(sp), C.c_double(U), C.c_void_p(_ptr(v)), C.c_void_p(_ptr(s)),
            C.c_void_p(_ptr(c))]
    if entry == "qs_projection_step":
        args.append(C.c_void_p(g._scratch_buf()))
    args += [C.c_double(rtol), 40, C.byref(info)]
    st = getattr(g._lib, entry)(*args)
    return st, info


@pytest.mark.parametrize("prec", ["fp64", "fp32-ir"])
def test_noalloc_step_matches_projection_step(prec):
    U, dt = 1e-5, 10.0
    for (nx, ny, nz), seed in (((48, 40, 24), 3), ((16, 16, 8), 5)):  # second call smaller
        print("noalloc step", prec, (nx, ny, nz), flush=True)
        g = MGSolver(nx, ny, nz, 1.0 / nz, LAM, MU, precision=prec, device="cuda")
        st = shear_state(nx, ny, nz, seed=seed, U=U)
        p = dict(P, l_diff=1.0 / nz)
        ref = [torch.from_numpy(st[k]).cuda() for k in ("v", "sigma", "chi")]
        new = [t.clone() for t in ref]
        for step in range(2):
            s1, i1 = _step(g, "qs_projection_step", p, dt, U, *ref, 1e-10)
            s2, i2 = _step(g, "qs_projection_step_noalloc", p, dt, U, *new, 1e-10)
            assert s1 == _capi.QS_OK and s2 == _capi.QS_OK, (s1, s2)
            assert i1.cycles == i2.cycles and i1.rel_res == i2.rel_res
            torch.cuda.synchronize()
            for a, b, name in zip(ref, new, ("v", "sigma", "chi")):
                assert torch.equal(a, b), (name, step)
        assert np.isfinite(ref[1].cpu().numpy()).all()
        g.close()


def test_noalloc_step_refuses_grids_beyond_its_buffer():
    n = 128  # 7 n^3 + 3 (n+1) n^2 doubles > 96 MiB
    g = MGSolver(n, n, n, 1.0 / n, LAM, MU, precision="fp32-ir", device="cuda")
    need = C.c_size_t()
    assert g._lib.qs_step_scratch_bytes(g._h, C.byref(need)) == _capi.QS_OK
    assert need.value > _capi.QS_NOALLOC_SCRATCH_BYTES
    v = torch.zeros(g.node_shape(), dtype=torch.float64, device="cuda")
    s = torch.zeros((6, n, n, n), dtype=torch.float64, device="cuda")
    c = torch.full((n, n, n), 0.05, dtype=torch.float64, device="cuda")
    st, _ = _step(g, "qs_projection_step_noalloc", P, 10.0, 1e-5, v, s, c, 1e-10)
    assert st == _capi.QS_ERR_SHAPE
    assert b"static buffer" in g._lib.qs_last_error()
    torch.cuda.synchronize()
    assert not v.any()  # nothing ran
    g.close()
