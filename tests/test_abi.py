"""The C ABI without a GPU: the shared library loads, exports every entry point
that include/qsmg.h declares, the Python binding covers exactly those names,
and the host-only calls (status strings, level planning, workspace sizing,
argument and shape checks) behave as the header states."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qsmg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:qs_status|const char\*)\s+(qs_\w+)\s*\(", text, flags=re.M))


@pytest.fixture(scope="module")
def lib():
    from paper_1904_03808_amd import _capi
    if not os.path.exists(_capi._LIB_PATH):
        from paper_1904_03808_amd.build import build_library
        build_library()
    return _capi.lib()


def params(nx=32, ny=32, nz=32, **kw):
    from paper_1904_03808_amd import _capi
    from workloads import lame
    lam, mu = lame()
    p = _capi.QSParams()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.h = 1.0 / nz
    p.lam, p.mu = lam, mu
    p.min_coarse_nz = kw.get("min_coarse_nz", 8)
    p.n_pre, p.n_post = kw.get("n_pre", 2), kw.get("n_post", 2)
    p.precision = kw.get("precision", _capi.QS_FP64)
    for q, c in enumerate(kw.get("order", (0, 1, 4, 5, 2, 3, 6, 7))):
        p.colour_order[q] = c
    return p


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("qs_setup", "qs_destroy", "qs_apply", "qs_mg_solve", "qs_stz_step", "qs_rhs",
                     "qs_stress_update", "qs_projection_step", "qs_stz_step_vjp", "qs_rhs_vjp",
                     "qs_stress_update_vjp", "qs_workspace_bytes", "qs_status_string",
                     "qs_projection_step_walls", "qs_explicit_step"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in sorted(declared_functions()):
        assert hasattr(lib, name), name


def test_binding_covers_exactly_the_header(lib):
    from paper_1904_03808_amd import _capi
    bound = set(_capi.SIGNATURES) | {"qs_status_string", "qs_last_error"}
    assert bound == declared_functions()


def test_status_strings(lib):
    from paper_1904_03808_amd import _capi
    for code in (_capi.QS_OK, _capi.QS_ERR_ARG, _capi.QS_ERR_SHAPE, _capi.QS_ERR_HIP,
                 _capi.QS_ERR_NOT_CONVERGED, _capi.QS_ERR_NONFINITE, _capi.QS_ERR_WORKSPACE):
        s = lib.qs_status_string(code)
        assert isinstance(s, bytes) and len(s) > 0
    assert lib.qs_status_string(12345) != lib.qs_status_string(_capi.QS_OK)


def test_level_planning_on_the_host(lib):
    from paper_1904_03808_amd import _capi
    n = C.c_int()
    dims = [C.c_int() for _ in range(3)]
    # coarsen while nz > 8: 256 -> 8 is 6 levels, 128 -> 5, 32 -> 3
    for size, levels in ((256, 6), (128, 5), (32, 3), (8, 1)):
        p = params(size, size, size)
        st = lib.qs_level_dims(C.byref(p), 0, C.byref(n), *[C.byref(d) for d in dims])
        assert st == _capi.QS_OK and n.value == levels, size
        st = lib.qs_level_dims(C.byref(p), levels - 1, C.byref(n), *[C.byref(d) for d in dims])
        assert st == _capi.QS_OK
        assert [d.value for d in dims] == [size >> (levels - 1)] * 3
        assert lib.qs_level_dims(C.byref(p), levels, C.byref(n), None, None, None) == _capi.QS_ERR_ARG
    # ragged grid: even in every coarsened level
    p = params(40, 24, 32)
    assert lib.qs_level_dims(C.byref(p), 2, C.byref(n), *[C.byref(d) for d in dims]) == _capi.QS_OK
    assert n.value == 3 and [d.value for d in dims] == [10, 6, 8]
    # 1024-wide rows down to 128 x 2 x 2
    p = params(1024, 16, 16, min_coarse_nz=2)
    got = []
    for lv in range(4):
        assert lib.qs_level_dims(C.byref(p), lv, C.byref(n), *[C.byref(d) for d in dims]) == _capi.QS_OK
        got.append([d.value for d in dims])
    assert n.value == 4 and got == [[1024, 16, 16], [512, 8, 8], [256, 4, 4], [128, 2, 2]]
    # odd sizes: allowed on a level that is not coarsened, refused where one must be
    p = params(7, 5, 6)
    assert lib.qs_level_dims(C.byref(p), 0, C.byref(n), *[C.byref(d) for d in dims]) == _capi.QS_OK
    assert n.value == 1 and [d.value for d in dims] == [7, 5, 6]
    for shape in ((7, 6, 10), (8, 6, 18)):  # odd on the fine level; odd nz = 9 on level 1
        p = params(*shape)
        assert lib.qs_level_dims(C.byref(p), 0, C.byref(n), None, None, None) == _capi.QS_ERR_SHAPE, shape


def test_workspace_sizing_and_argument_errors(lib):
    from paper_1904_03808_amd import _capi
    b64, b32 = C.c_size_t(), C.c_size_t()
    assert lib.qs_workspace_bytes(C.byref(params(64, 64, 64)), C.byref(b64)) == _capi.QS_OK
    p32 = params(64, 64, 64, precision=_capi.QS_FP32_IR)
    assert lib.qs_workspace_bytes(C.byref(p32), C.byref(b32)) == _capi.QS_OK
    vec64 = 3 * 65 * 64 * 64 * 8
    assert b64.value > vec64 and b32.value > vec64 // 2
    # the workspace grows with the grid
    big = C.c_size_t()
    assert lib.qs_workspace_bytes(C.byref(params(128, 128, 128)), C.byref(big)) == _capi.QS_OK
    assert big.value > 4 * b64.value  # the dense coarsest inverse is the same at both sizes
    # invalid parameters
    bad = C.c_size_t()
    assert lib.qs_workspace_bytes(None, C.byref(bad)) == _capi.QS_ERR_ARG
    assert lib.qs_workspace_bytes(C.byref(params(precision=7)), C.byref(bad)) == _capi.QS_ERR_ARG
    assert lib.qs_workspace_bytes(C.byref(params(order=(0, 0, 1, 2, 3, 4, 5, 6))),
                                  C.byref(bad)) == _capi.QS_ERR_ARG
    p = params()
    p.h = 0.0
    assert lib.qs_workspace_bytes(C.byref(p), C.byref(bad)) == _capi.QS_ERR_ARG
    # odd dimension on a level that is coarsened; coarsest level too large for the dense solve
    assert lib.qs_workspace_bytes(C.byref(params(33, 32, 32)), C.byref(bad)) == _capi.QS_ERR_SHAPE
    assert lib.qs_workspace_bytes(C.byref(params(64, 64, 16, min_coarse_nz=16)),
                                  C.byref(bad)) == _capi.QS_ERR_SHAPE
    # 32-bit indexing: a coarsenable grid whose cell tensor has 6 nz ny nx >= 2^31
    # elements is refused, 512^3 is not
    assert lib.qs_workspace_bytes(C.byref(params(640, 640, 1024)), C.byref(bad)) == _capi.QS_ERR_SHAPE
    assert lib.qs_workspace_bytes(C.byref(params(512, 512, 512)), C.byref(bad)) == _capi.QS_OK
    # null handles are refused before anything touches a device
    assert lib.qs_destroy(None) == _capi.QS_ERR_ARG
    assert lib.qs_mg_solve(None, None, None, C.c_double(1e-10), 10, None) == _capi.QS_ERR_ARG
    from workloads import stz_constants
    P = stz_constants()
    sp = _capi.QSStzParams(P["s_y"], P["tau0"], P["beta"], P["delta_over_T"], P["c0"],
                           P["chi_inf"], 1.0, 0.0, 1, 0, 0)
    assert lib.qs_explicit_step(None, C.byref(sp), 0.0, 0.37, 0.1, None, None, None,
                                None) == _capi.QS_ERR_ARG
    assert lib.qs_projection_step_walls(None, C.byref(sp), None, None, None, None, None, None,
                                        C.c_double(1e-10), 10, None) == _capi.QS_ERR_ARG
    assert lib.qs_stz_step(None, C.byref(sp), None, None, None, None, None) == _capi.QS_ERR_ARG
