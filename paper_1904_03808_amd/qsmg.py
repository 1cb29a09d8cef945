"""Torch-facing binding of libqsmg (names follow include/qsmg.h).

Argument marshalling only: shapes and dtypes are checked here, and every
computation runs in the HIP library.  The library's handle is bound to one
HIP stream, torch's current stream when the MGSolver is constructed; every
later call checks that this is still torch's current stream and raises
otherwise, so library work is always ordered with the caller's tensor work.
Tensors are float64, contiguous and on the GPU.

  MGSolver            qs_setup / qs_destroy handle with its device workspace
    .apply            qs_apply
    .solve            qs_mg_solve
    .stz_step         qs_stz_step
    .rhs              qs_rhs
    .stress_update    qs_stress_update
    .projection_step  qs_projection_step
    .projection_step_noalloc  qs_projection_step_noalloc
    .stz_step_vjp / .rhs_vjp / .stress_update_vjp
    .level_*          test-facing pieces of the V-cycle
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Sequence

import torch

from . import _capi
from ._capi import (QS_ERR_NOT_CONVERGED, QS_FP32_IR, QS_FP64, QS_OK, QSParams,
                    QSSolveInfo, QSStzParams, check, lib)


@dataclass
class SolveInfo:
    status: int
    cycles: int
    levels: int
    rel_res: float
    hist: list

    @property
    def converged(self) -> bool:
        return self.status == QS_OK


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _stz(params: dict, dt: float) -> QSStzParams:
    return QSStzParams(params["s_y"], params["tau0"], params["beta"], params["delta_over_T"],
                       params["c0"], params["chi_inf"], dt, params.get("l_diff", 0.0),
                       int(params.get("n_sub", 1)), int(bool(params.get("advect", 0))),
                       int(params.get("chi_wall", 0)))


class MGSolver:
    """Multigrid hierarchy for an nx*ny*nz cell grid (x, y periodic, z walls)."""

    def __init__(self, nx: int, ny: int, nz: int, h: float, lam: float, mu: float,
                 min_coarse_nz: int = 8, n_pre: int = 2, n_post: int = 2,
                 precision: str = "fp64", colour_order: Sequence[int] = (0, 1, 4, 5, 2, 3, 6, 7),
                 device: str | torch.device = "cuda"):
        self.nx, self.ny, self.nz, self.h = nx, ny, nz, h
        self.lam, self.mu = lam, mu
        self.device = torch.device(device)
        prec = {"fp64": QS_FP64, "fp32-ir": QS_FP32_IR}[precision]
        self.precision = precision
        self._params = QSParams(nx, ny, nz, h, lam, mu, min_coarse_nz, n_pre, n_post, prec,
                                (C.c_int * 8)(*colour_order))
        self._lib = lib()
        n = C.c_size_t()
        check(self._lib.qs_workspace_bytes(C.byref(self._params), C.byref(n)), "qs_workspace_bytes")
        self.workspace_bytes = n.value
        self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        base = (self._ws.data_ptr() + 255) & ~255
        self.stream = torch.cuda.current_stream(self.device)
        hd = C.c_void_p()
        check(self._lib.qs_setup(C.byref(self._params), C.c_void_p(base), n.value,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(hd)), "qs_setup")
        self._hd_raw = hd
        nl = C.c_int()
        self._lib.qs_level_dims(C.byref(self._params), 0, C.byref(nl), None, None, None)
        self.levels = nl.value
        self._scratch = None

    # -- helpers ------------------------------------------------------------
    def level_dims(self, level: int):
        nl, a, b, c = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        check(self._lib.qs_level_dims(C.byref(self._params), level, C.byref(nl), C.byref(a),
                                      C.byref(b), C.byref(c)), "qs_level_dims")
        return a.value, b.value, c.value

    def node_shape(self, level: int = 0):
        nx, ny, nz = self.level_dims(level)
        return (3, nz + 1, ny, nx)

    @property
    def cell_shape(self):
        return (self.nz, self.ny, self.nx)

    def _chk(self, t: torch.Tensor, shape, name: str):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
            raise TypeError("%s must be a float64 CUDA tensor" % name)
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError("%s must be contiguous with shape %s, got %s"
                             % (name, tuple(shape), tuple(t.shape)))
        return _ptr(t)

    def _scratch_buf(self) -> int:
        if self._scratch is None:
            n = C.c_size_t()
            check(self._lib.qs_step_scratch_bytes(self._h, C.byref(n)), "qs_step_scratch_bytes")
            self._scratch = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        return (self._scratch.data_ptr() + 255) & ~255

    @property
    def _h(self):
        """The library handle, after checking that torch's current stream is
        the one the handle was set up on."""
        hd = self.__dict__.get("_hd_raw")
        if hd is not None and torch.cuda.current_stream(self.device).cuda_stream != self.stream.cuda_stream:
            raise RuntimeError("MGSolver is bound to the stream that was current at construction; "
                               "call it under that stream (torch.cuda.stream(solver.stream))")
        return hd

    def close(self):
        if self.__dict__.get("_hd_raw"):
            self._lib.qs_destroy(self._hd_raw)
            self._hd_raw = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- operator and solve ---------------------------------------------------
    def apply(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        out = torch.empty_like(x) if out is None else out
        s = self.node_shape()
        check(self._lib.qs_apply(self._h, self._chk(x, s, "x"), self._chk(out, s, "out")),
              "qs_apply")
        return out

    def solve(self, b: torch.Tensor, x: torch.Tensor, rtol: float = 1e-10,
              max_cycles: int = 100, raise_on_failure: bool = True) -> SolveInfo:
        s = self.node_shape()
        info = QSSolveInfo()
        st = self._lib.qs_mg_solve(self._h, self._chk(b, s, "b"), self._chk(x, s, "x"),
                                   float(rtol), int(max_cycles), C.byref(info))
        if raise_on_failure:
            check(st, "qs_mg_solve")
        n = min(info.cycles + 1, _capi.QS_HIST)
        return SolveInfo(st, info.cycles, info.levels, info.rel_res, list(info.rel_res_hist[:n]))

    # -- STZ / projection -------------------------------------------------------
    def stz_step(self, params: dict, dt: float, v, sigma, chi):
        cs = self.cell_shape
        sstar = torch.empty((6,) + cs, dtype=torch.float64, device=self.device)
        chi1 = torch.empty(cs, dtype=torch.float64, device=self.device)
        sp = _stz(params, dt)
        check(self._lib.qs_stz_step(self._h, C.byref(sp), self._chk(v, self.node_shape(), "v"),
                                    self._chk(sigma, (6,) + cs, "sigma"), self._chk(chi, cs, "chi"),
                                    _ptr(sstar), _ptr(chi1)), "qs_stz_step")
        return sstar, chi1

    def rhs(self, sigma_star, dt: float):
        b = torch.empty(self.node_shape(), dtype=torch.float64, device=self.device)
        check(self._lib.qs_rhs(self._h, self._chk(sigma_star, (6,) + self.cell_shape, "sigma_star"),
                               float(dt), _ptr(b)), "qs_rhs")
        return b

    def stress_update(self, sigma_star, v, dt: float, out=None):
        out = torch.empty_like(sigma_star) if out is None else out
        check(self._lib.qs_stress_update(self._h, self._chk(sigma_star, (6,) + self.cell_shape, "sigma_star"),
                                         self._chk(v, self.node_shape(), "v"), float(dt),
                                         self._chk(out, (6,) + self.cell_shape, "out")),
              "qs_stress_update")
        return out

    def projection_step(self, params: dict, dt: float, U: float, v, sigma, chi,
                        rtol: float = 1e-10, max_cycles: int = 100) -> SolveInfo:
        """In-place step n -> n+1 of (v, sigma, chi)."""
        cs = self.cell_shape
        sp = _stz(params, dt)
        info = QSSolveInfo()
        st = self._lib.qs_projection_step(self._h, C.byref(sp), float(U),
                                          self._chk(v, self.node_shape(), "v"),
                                          self._chk(sigma, (6,) + cs, "sigma"),
                                          self._chk(chi, cs, "chi"), C.c_void_p(self._scratch_buf()),
                                          float(rtol), int(max_cycles), C.byref(info))
        check(st, "qs_projection_step")
        n = min(info.cycles + 1, _capi.QS_HIST)
        return SolveInfo(st, info.cycles, info.levels, info.rel_res, list(info.rel_res_hist[:n]))

    def projection_step_noalloc(self, params: dict, dt: float, U: float, v, sigma, chi,
                                rtol: float = 1e-10, max_cycles: int = 100) -> SolveInfo:
        """projection_step with the library's fixed device scratch instead of
        a scratch tensor (qs_projection_step_noalloc: nothing is allocated)."""
        cs = self.cell_shape
        sp = _stz(params, dt)
        info = QSSolveInfo()
        st = self._lib.qs_projection_step_noalloc(self._h, C.byref(sp), float(U),
                                                  self._chk(v, self.node_shape(), "v"),
                                                  self._chk(sigma, (6,) + cs, "sigma"),
                                                  self._chk(chi, cs, "chi"), float(rtol),
                                                  int(max_cycles), C.byref(info))
        check(st, "qs_projection_step_noalloc")
        n = min(info.cycles + 1, _capi.QS_HIST)
        return SolveInfo(st, info.cycles, info.levels, info.rel_res, list(info.rel_res_hist[:n]))

    def projection_step_walls(self, params: dict, dt: float, wall_lo, wall_hi, v, sigma, chi,
                              rtol: float = 1e-10, max_cycles: int = 100) -> SolveInfo:
        """In-place step n -> n+1 with per-node wall velocities of step n+1:
        wall_lo, wall_hi are (3, ny, nx) float64 device tensors for the planes
        k = 0 and k = nz."""
        cs = self.cell_shape
        ws = (3, self.ny, self.nx)
        sp = _stz(params, dt)
        info = QSSolveInfo()
        st = self._lib.qs_projection_step_walls(
            self._h, C.byref(sp), self._chk(wall_lo, ws, "wall_lo"), self._chk(wall_hi, ws, "wall_hi"),
            self._chk(v, self.node_shape(), "v"), self._chk(sigma, (6,) + cs, "sigma"),
            self._chk(chi, cs, "chi"), C.c_void_p(self._scratch_buf()), float(rtol),
            int(max_cycles), C.byref(info))
        check(st, "qs_projection_step_walls")
        n = min(info.cycles + 1, _capi.QS_HIST)
        return SolveInfo(st, info.cycles, info.levels, info.rel_res, list(info.rel_res_hist[:n]))

    def explicit_step(self, params: dict, dt: float, U: float, rho: float, kappa: float, v, sigma,
                      chi) -> None:
        """In-place step n -> n+1 of the explicit method (no solve)."""
        cs = self.cell_shape
        sp = _stz(params, dt)
        check(self._lib.qs_explicit_step(self._h, C.byref(sp), float(U), float(rho), float(kappa),
                                         self._chk(v, self.node_shape(), "v"),
                                         self._chk(sigma, (6,) + cs, "sigma"),
                                         self._chk(chi, cs, "chi"),
                                         C.c_void_p(self._scratch_buf())), "qs_explicit_step")

    # -- reverse mode -------------------------------------------------------------
    def stz_step_vjp(self, params: dict, dt: float, v, sigma, chi, g_sstar, g_chi1, g_v):
        """Returns (g_sigma, g_chi) and adds the velocity cotangent into g_v."""
        cs = self.cell_shape
        g_sigma = torch.empty((6,) + cs, dtype=torch.float64, device=self.device)
        g_chi = torch.empty(cs, dtype=torch.float64, device=self.device)
        sp = _stz(params, dt)
        check(self._lib.qs_stz_step_vjp(
            self._h, C.byref(sp), self._chk(v, self.node_shape(), "v"),
            self._chk(sigma, (6,) + cs, "sigma"), self._chk(chi, cs, "chi"),
            self._chk(g_sstar, (6,) + cs, "g_sstar"), self._chk(g_chi1, cs, "g_chi1"),
            _ptr(g_sigma), _ptr(g_chi), self._chk(g_v, self.node_shape(), "g_v"),
            C.c_void_p(self._scratch_buf())), "qs_stz_step_vjp")
        return g_sigma, g_chi

    def rhs_vjp(self, g_b, dt: float, g_sstar):
        check(self._lib.qs_rhs_vjp(self._h, self._chk(g_b, self.node_shape(), "g_b"), float(dt),
                                   self._chk(g_sstar, (6,) + self.cell_shape, "g_sstar")),
              "qs_rhs_vjp")
        return g_sstar

    def stress_update_vjp(self, g_sigma, dt: float, g_v):
        check(self._lib.qs_stress_update_vjp(self._h, self._chk(g_sigma, (6,) + self.cell_shape, "g_sigma"),
                                             float(dt), self._chk(g_v, self.node_shape(), "g_v")),
              "qs_stress_update_vjp")
        return g_v

    # -- test-facing V-cycle pieces -----------------------------------------------
    def level_colour_pass(self, level: int, x, b, colour: int):
        s = self.node_shape(level)
        check(self._lib.qs_level_colour_pass(self._h, level, self._chk(x, s, "x"),
                                             self._chk(b, s, "b"), colour), "qs_level_colour_pass")

    def level_residual(self, level: int, x, b):
        s = self.node_shape(level)
        r = torch.zeros(s, dtype=torch.float64, device=self.device)
        check(self._lib.qs_level_residual(self._h, level, self._chk(x, s, "x"),
                                          self._chk(b, s, "b"), _ptr(r)), "qs_level_residual")
        return r

    def level_restrict(self, level: int, r):
        bc = torch.zeros(self.node_shape(level + 1), dtype=torch.float64, device=self.device)
        check(self._lib.qs_level_restrict(self._h, level, self._chk(r, self.node_shape(level), "r"),
                                          _ptr(bc)), "qs_level_restrict")
        return bc

    def level_prolong_add(self, level: int, x, ec):
        check(self._lib.qs_level_prolong_add(self._h, level, self._chk(x, self.node_shape(level), "x"),
                                             self._chk(ec, self.node_shape(level + 1), "ec")),
              "qs_level_prolong_add")

    def coarse_solve(self, x, b):
        s = self.node_shape(self.levels - 1)
        check(self._lib.qs_coarse_solve(self._h, self._chk(x, s, "x"), self._chk(b, s, "b")),
              "qs_coarse_solve")

    def smooth(self, level: int, x, b, sweeps: int):
        s = self.node_shape(level)
        dt = torch.float32 if self.precision == "fp32-ir" else torch.float64
        for t, name in ((x, "x"), (b, "b")):
            if t.dtype != dt or tuple(t.shape) != s or not t.is_contiguous() or t.device.type != "cuda":
                raise ValueError("%s must be a contiguous %s CUDA tensor of shape %s" % (name, dt, s))
        check(self._lib.qs_smooth(self._h, level, _ptr(x), _ptr(b), int(sweeps)), "qs_smooth")

    def level_stencil(self, level: int):
        import numpy as np
        nx, ny, nz = self.level_dims(level)
        out = np.zeros((nz + 1, 27, 3, 3))
        check(self._lib.qs_level_stencil(self._h, level, out.ctypes.data_as(C.c_void_p)),
              "qs_level_stencil")
        return out.reshape(nz + 1, 3, 3, 3, 3, 3)
