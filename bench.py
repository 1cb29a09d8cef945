"""Benchmark: multigrid solves of the projection system at 256^3 on one MI355X.

One step = one full solve K x = b from x = 0 to a relative residual of 1e-10
(V(2,2) cycles, 6 levels, FP32 V-cycles inside FP64 iterative refinement),
with b = D_h sigma for a smoothed random cell stress (seed 2), all inputs
resident in HBM.  The same workload is also timed with plain FP64 V-cycles.

Prints one JSON line.  Besides the contract fields it carries
  roofline      the fine-level smoother (dominant kernel) against HBM peak,
                timed with HIP events on the library's stream
  cpu_baseline  the FP64 oracle on the host cores over a bounded sample
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "V-cycle solves/s + smoother HBM GB/s, 256^3 to 1e-10 rel resid, FP32-IR vs FP64"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the fine FP32 half sweep at 256^3, from two rocprofv3
# counter runs of `bench.py --profile-smoother` (FETCH_SIZE, then WRITE_SIZE; KiB
# per dispatch, mean of 6 launches).  A 512 MiB device copy reads as
# FETCH_SIZE = 262,166 KiB and WRITE_SIZE = 524,288 KiB: on this chip every read
# request (TCC_EA0_RDREQ, 4,194,593 for the copy) carries 128 bytes but the
# derived FETCH_SIZE prices it at 64, so reads scale by 2.0 and writes by 1.0.
# Valid only for the kernel source these counters were taken on.
SWEEP_COUNTERS = {
    "kernel_source": "paper_1904_03808_amd/csrc/kernels_sweep.hip",
    "source_sha256_16": "dea4244a5a0518a8",
    "n": 256,
    "fetch_kib": 177898.6,
    "write_kib": 97920.0,
    "fetch_scale": 2.0,
    "write_scale": 1.0,
}


def _block(fn):
    """Run one of the secondary measurement blocks; if it raises, report the
    error in its place so that the main line still prints."""
    try:
        return fn()
    except Exception as e:  # noqa: BLE001 - reported in the JSON line
        import torch
        torch.cuda.empty_cache()
        return {"error": "%s: %s" % (type(e).__name__, e)}


def _events_ms(fn, reps: int) -> float:
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def sweep_traffic(n: int):
    """HBM bytes per FP32 fine half-sweep launch from the stored counters, or
    None when the workload or the kernel source differs from the measured one."""
    import hashlib
    sc = SWEEP_COUNTERS
    with open(os.path.join(ROOT, sc["kernel_source"]), "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    if h != sc["source_sha256_16"] or n != sc["n"]:
        return None
    return 1024.0 * (sc["fetch_kib"] * sc["fetch_scale"] + sc["write_kib"] * sc["write_scale"])


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sig_host, n: int, cycles_full: int) -> dict:
    """Oracle (NumPy/SciPy FP64) timed on the host at the bench size itself:
    one V(2,2) cycle plus the residual norm the solve loop takes after it, on
    the same n^3 workload (b = D_h sigma from the same host stress), scaled
    by the measured number of cycles of one solve to 1e-10.  `cores` is the
    process CPU time over the wall time of that sample (the matrix-free
    cycle runs single-threaded NumPy)."""
    import numpy as np
    import psutil

    from oracle.multigrid import MGOracle
    from oracle.operators import div_node
    from workloads import lame
    lam, mu = lame()
    o = MGOracle(n, n, n, 1.0 / n, lam, mu)
    b = div_node(sig_host, 1.0 / n)
    x = np.zeros_like(b)
    proc = psutil.Process()
    c0 = proc.cpu_times()
    t0 = time.perf_counter()
    o.vcycle(x, b)
    float(np.linalg.norm(o.residual(x, b)[:, 1:-1]))
    wall = time.perf_counter() - t0
    c1 = proc.cpu_times()
    cpu = (c1.user - c0.user) + (c1.system - c0.system)
    t_solve = wall * cycles_full
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": max(1, int(round(cpu / wall))),
            "kind": "oracle",
            "sample": "one oracle V(2,2) cycle and residual norm measured at %d^3 (%.1f s wall, "
                      "%.1f s CPU), times %d cycles per solve to 1e-10 (the FP64 solve's count)"
                      % (n, wall, cpu, cycles_full),
            "host_cpu": _cpu_model(), "host_cpus": os.cpu_count()}


def error_vs_oracle(n: int, sols: dict) -> dict:
    """Relative L2 difference of each GPU solution from the FP64 oracle's
    solution of the same system (solved to 1e-12), over the 4096 interior
    nodes stored in tests/golden/solve256.json by an oracle-only script."""
    import torch
    path = os.path.join(ROOT, "tests", "golden", "solve%d.json" % n)
    if not os.path.exists(path):
        return {"error": "no stored oracle solution for n = %d" % n}
    with open(path) as f:
        ref = json.load(f)
    out = {"oracle_rtol": ref["rtol"], "oracle_cycles": ref["cycles"], "nodes_sampled": len(ref["sample_index"])}
    for name, x in sols.items():
        idx = torch.tensor(ref["sample_index"], device=x.device)
        got = x[:, idx[:, 0], idx[:, 1], idx[:, 2]].T
        want = torch.tensor(ref["sample_x"], dtype=torch.float64, device=x.device)
        out[name] = (torch.linalg.vector_norm(got - want) / torch.linalg.vector_norm(want)).item()
    return out


def smoother_timing(g, b, dtype, bytes_per_node: float) -> dict:
    """Fine-level full sweeps of solver g on its own: HIP events on the
    library's stream; the difference of a 5-sweep and a 1-sweep call leaves 4
    sweeps of the kernel alone (one call also moves the wall planes of the
    ping-pong buffer).  One sweep = two row-parity half sweeps (k_sweep_rows),
    each updating half of the nodes."""
    import torch
    n3 = g.node_shape(0)
    nodes = n3[3] * n3[2] * (n3[1] - 2)
    xs = torch.zeros(n3, dtype=dtype, device=b.device)
    bs = b.to(dtype)
    g.smooth(0, xs, bs, 1)
    t5 = _events_ms(lambda: g.smooth(0, xs, bs, 5), 5)
    t1 = _events_ms(lambda: g.smooth(0, xs, bs, 1), 5)
    ms = (t5 - t1) / 4
    del xs, bs
    return {"ms_per_sweep": ms, "launches_per_sweep": 2, "avg_launch_us": ms * 1e3 / 2,
            "effective_GBs": bytes_per_node * nodes / (ms * 1e-3) / 1e9}


def solve_pair(n: int, b, steps: int, warmup: int, smoother: bool = False) -> dict:
    """FP32-IR and FP64 solves of K x = b from x = 0 to 1e-10 at n^3; wall time
    per solve between device synchronisations, and the two solutions' relative
    L2 difference (with `smoother`, also the fine-level sweep timing)."""
    import torch

    from paper_1904_03808_amd.qsmg import MGSolver
    from workloads import lame
    lam, mu = lame()
    out, sols = {}, {}
    for name, prec in (("fp32_ir", "fp32-ir"), ("fp64", "fp64")):
        g = MGSolver(n, n, n, 1.0 / n, lam, mu, precision=prec, device=b.device)
        x = torch.zeros_like(b)
        for _ in range(warmup):
            x.zero_()
            g.solve(b, x, rtol=1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            info = g.solve(b, x, rtol=1e-10)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[name] = {"ms_per_solve": dt * 1e3, "solves_per_s": 1.0 / dt, "cycles": info.cycles,
                     "rel_res": info.rel_res, "levels": g.levels,
                     "ms_per_cycle": dt * 1e3 / max(info.cycles, 1)}
        if smoother:
            fp32 = prec == "fp32-ir"
            out[name]["smoother"] = smoother_timing(g, b, torch.float32 if fp32 else torch.float64,
                                                    36.0 if fp32 else 72.0)
        sols[name] = x
        g.close()
    out["fp32ir_vs_fp64_rel_l2"] = (torch.linalg.vector_norm(sols["fp32_ir"] - sols["fp64"])
                                    / torch.linalg.vector_norm(sols["fp64"])).item()
    out["speedup_fp32ir_vs_fp64"] = out["fp64"]["ms_per_solve"] / out["fp32_ir"]["ms_per_solve"]
    return out


def config_512(steps: int = 3, warmup: int = 1) -> dict:
    """The 512^3 case of the mixed-precision comparison (7 levels); the RHS is
    the same recipe (D_h of the smoothed random stress, seed 2) generated on the
    device."""
    import torch

    from paper_1904_03808_amd.qsmg import MGSolver
    from workloads import lame, stress_field_device
    lam, mu = lame()
    n = 512
    dev = torch.device("cuda:0")
    g = MGSolver(n, n, n, 1.0 / n, lam, mu, precision="fp64", device=dev)
    sig = stress_field_device(n, n, n, 2, dev)
    b = g.rhs(sig, 1.0)
    del sig
    g.close()
    out = solve_pair(n, b, steps, warmup, smoother=True)
    out["grid"] = [n, n, n]
    out["steps"] = steps
    out["rhs"] = "D_h sigma, sigma smoothed N(0,1) generated on the device (seed 2)"
    del b
    torch.cuda.empty_cache()
    return out


def config3_shear(n: int = 256, steps: int = 20) -> dict:
    """Quasi-static steps under simple shear: `steps` FP32-IR projection steps at
    n^3 from the shear initial state (chi seed 3), warm-started from the
    previous velocity, timed between device synchronisations; then the phases
    of one more step (STZ update, right-hand side, solve, stress correction)
    timed one by one with HIP events on the library's stream."""
    import torch

    from paper_1904_03808_amd.qsmg import MGSolver
    from workloads import lame, shear_state, stz_constants
    lam, mu = lame()
    dev = torch.device("cuda:0")
    P, dt, U = stz_constants(), 10.0, 1e-5
    st = shear_state(n, n, n, seed=3, U=U)
    g = MGSolver(n, n, n, 1.0 / n, lam, mu, precision="fp32-ir", device=dev)
    v0, s0, c0 = (torch.from_numpy(st[k]).to(dev) for k in ("v", "sigma", "chi"))
    del st
    v, s, c = v0.clone(), s0.clone(), c0.clone()
    g.projection_step(P, dt, U, v, s, c, rtol=1e-10)  # warm-up (state discarded)
    v.copy_(v0), s.copy_(s0), c.copy_(c0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles = [g.projection_step(P, dt, U, v, s, c, rtol=1e-10).cycles for _ in range(steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ph = {}
    ph["stz_ms"] = _events_ms(lambda: g.stz_step(P, dt, v, s, c), 3)
    # the same step with the ENO advection of the stress (not in Eq. sig_star_qs)
    ph["stz_with_advection_ms"] = _events_ms(lambda: g.stz_step(dict(P, advect=1), dt, v, s, c), 3)
    sstar, _ = g.stz_step(P, dt, v, s, c)
    ph["rhs_ms"] = _events_ms(lambda: g.rhs(sstar, dt), 3)
    b = g.rhs(sstar, dt)
    x = v.clone()
    ph["solve_ms"] = _events_ms(lambda: (x.copy_(v), g.solve(b, x, rtol=1e-10)), 1)
    ph["stress_update_ms"] = _events_ms(lambda: g.stress_update(sstar, x, dt), 3)
    g.close()
    del v0, s0, c0, v, s, c, sstar, b, x
    torch.cuda.empty_cache()
    return {"grid": [n, n, n], "steps": steps, "ms_per_step": ms, "steps_per_s": 1e3 / ms,
            "cycles_per_step": cycles, "phase_ms_one_step": ph, "solver": "fp32-ir",
            "inputs": "shear state: sigma_xz = 0.99 s_Y, linear v, chi Gaussian field (seed 3)"}


def config4_adjoint(n: int = 96, steps: int = 10) -> dict:
    """Reverse mode of a `steps`-step FP64 rollout at n^3 (chi seed 4): time of
    the forward pass with per-step checkpoints and of the backward pass (the
    transposed solves and the step VJPs), solves to 1e-10."""
    import torch

    from paper_1904_03808_amd.autograd import rollout_loss
    from paper_1904_03808_amd.qsmg import MGSolver
    from workloads import lame, shear_state, stz_constants
    lam, mu = lame()
    dev = torch.device("cuda:0")
    P, dt, U = stz_constants(), 10.0, 1e-5
    st = shear_state(n, n, n, seed=4, U=U)
    g = MGSolver(n, n, n, 1.0 / n, lam, mu, precision="fp64", device=dev)
    v0, s0, c0 = (torch.from_numpy(st[k]).to(dev) for k in ("v", "sigma", "chi"))
    times = []
    for _ in range(2):  # the first pass is a warm-up
        chi = c0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = rollout_loss(chi, v0, s0, g, P, dt, U, steps, rtol=1e-10)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append(((t1 - t0) * 1e3, (t2 - t1) * 1e3))
    g.close()
    return {"grid": [n, n, n], "steps": steps, "forward_ms": times[-1][0],
            "backward_ms": times[-1][1], "gradient_ms": sum(times[-1]),
            "loss": loss.item(), "solver": "fp64, rtol 1e-10 forward and transposed"}


# The paper's simple-shear runs on N x N x N/2 grids (dt = 200 t_s, U = 1e-7
# L/t_s, 5000 steps to 1e6 t_s, 32 CPU processes): chi0, diffusion length in
# cells, and the reported (total hours, V-cycle hours, V-cycles) per N.
PAPER_RUNS = {
    "defect": {"chi": "Eq. case0_chi (550 K + 170 K Gaussian)", "l_cells": 1.0,
               "paper": {256: (7.52, 5.852, 17586)}},
    "random": {"chi": "Eq. convolve, 550 K mean, 15 K std, l_c = 10 h, cutoff 5 (seed 7)",
               "l_cells": 1.5,
               "paper": {128: (1.61, 1.27, 20480), 256: (6.12, 3.89, 18367),
                         384: (22.44, 14.28, 24675), 512: (42.86, 30.23, 28175),
                         768: (105.97, 75.90, 19689)}},
    "helix": {"chi": "Eq. case12_chi (550 K + 200 K along the helix)", "l_cells": 1.5,
              "paper": {80: (1.52, 1.00, 15073), 128: (1.94, 1.37, 16511),
                        256: (3.69, 2.75, 17939)}},
}


def paper_chi(kind: str, nx: int, ny: int, nz: int):
    from workloads import chi_field, defect_chi, helix_chi
    if kind == "defect":
        return defect_chi(nx, ny, nz)
    if kind == "helix":
        return helix_chi(nx, ny, nz)
    return chi_field(nx, ny, nz, 7, 550.0 / 21000, 15.0 / 21000, 10.0)


def defect_run(N: int = 256, steps: int = 5000, min_coarse_nz: int = 4, n_sub: int = -1,
               per_vcycle: bool = True, kind: str = "defect", chi_wall: int = 0) -> dict:
    """The single-defect run of Sec. 4.4 on its N x N x N/2 grid (h = L/(N/2)):
    chi from Eq. case0_chi, l = h, dt = 200 t_s, U = 1e-7 L/t_s, the sample at
    rest and free of stress at t = 0.  `steps` FP32-IR projection steps
    (rtol 1e-10, warm-started) are timed between device synchronisations, with
    a split every 500 steps: elastic loading (to t = 1e5 t_s), yield, then
    plastic flow concentrating in the defect and a band forming.  The default
    is the paper's whole run (5000 steps to t = 1e6 t_s) with the plastic terms
    sub-stepped per cell (n_sub = -1): with the single forward-Euler step of
    Eq. sig_star_qs (n_sub = 1) the run loses stability near t = 3.7e5 t_s,
    so at most about 1850 steps can be run that way.  Then the time per V-cycle at this
    shape, FP32-IR and FP64, from solves from zero of a D_h sigma right-hand
    side (seed 2): the figure the paper tabulates (Tables 2 and 3, and the
    single-defect run's V-cycle total).  `kind` = "random" or "helix" runs the
    Table 3 or Table 2 workload instead (l = 1.5 h)."""
    import torch

    from paper_1904_03808_amd.qsmg import MGSolver
    from workloads import defect_state, lame, stress_field_device, stz_constants
    lam, mu = lame()
    dev = torch.device("cuda:0")
    nx, ny, nz = N, N, N // 2
    h = 1.0 / nz
    run = PAPER_RUNS[kind]
    P, dt, U = (dict(stz_constants(), l_diff=run["l_cells"] * h, n_sub=n_sub, chi_wall=chi_wall),
                200.0, 1e-7)
    st = defect_state(nx, ny, nz, U)
    st["chi"] = paper_chi(kind, nx, ny, nz)
    g = MGSolver(nx, ny, nz, h, lam, mu, min_coarse_nz=min_coarse_nz, precision="fp32-ir",
                 device=dev)
    v0, s0, c0 = (torch.from_numpy(st[k]).to(dev) for k in ("v", "sigma", "chi"))
    del st
    v, s, c = v0.clone(), s0.clone(), c0.clone()
    g.projection_step(P, dt, U, v, s, c, rtol=1e-10)  # warm-up (state discarded)
    v.copy_(v0), s.copy_(s0), c.copy_(c0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks, cycles, failed = [t0], [], None
    # U(t) ramps to U_B over the first t_s < dt, so every step sees U_B
    from paper_1904_03808_amd._capi import QSError
    for i in range(steps):
        try:
            cycles.append(g.projection_step(P, dt, U, v, s, c, rtol=1e-10).cycles)
        except QSError as e:  # a non-finite state: report the steps that ran
            failed = {"step": i, "status": str(e)}
            torch.cuda.synchronize()
            marks.append(time.perf_counter())
            break
        if (i + 1) % 500 == 0 or i + 1 == steps:
            torch.cuda.synchronize()
            marks.append(time.perf_counter())
            if steps > 1500:
                print("%s run: %d steps, %.1f s" % (kind, i + 1, marks[-1] - t0), file=sys.stderr,
                      flush=True)
    steps = max(len(cycles), 1)
    ms = (marks[-1] - t0) * 1e3 / steps
    phases = []
    for m in range(len(marks) - 1):
        a, b = 500 * m, min(500 * (m + 1), steps)
        if b <= a:
            continue
        phases.append({"steps": [a, b], "ms_per_step": (marks[m + 1] - marks[m]) * 1e3 / (b - a),
                       "vcycles_per_step": sum(cycles[a:b]) / (b - a)})
    p_ = (s[0] + s[1] + s[2]) / 3
    sbar = torch.sqrt(0.5 * ((s[0] - p_) ** 2 + (s[1] - p_) ** 2 + (s[2] - p_) ** 2)
                      + s[3] ** 2 + s[4] ** 2 + s[5] ** 2)
    state = {"t_end": steps * dt, "sbar_max_over_sY": (sbar.max() / P["s_y"]).item(),
             "sbar_mean_over_sY": (sbar.mean() / P["s_y"]).item(),
             "chi_max_K": c.max().item() * 21000.0, "chi_min_K": c.min().item() * 21000.0}
    levels = g.levels
    g.close()
    del v0, s0, c0, v, s, c, sbar, p_
    res = {"grid": [nx, ny, nz], "levels": levels, "min_coarse_nz": min_coarse_nz,
           "steps": steps, "ms_per_step": ms, "steps_per_s": 1e3 / ms,
           "vcycles": sum(cycles), "vcycles_per_step": sum(cycles) / steps,
           "max_vcycles_in_a_step": max(cycles), "phases": phases, "state_at_end": state,
           "plastic_substeps": ("single step (Eq. sig_star_qs)" if n_sub == 1 else
                                "per cell from the stability bound" if n_sub == -1 else n_sub),
           "solver": "fp32-ir, rtol 1e-10",
           "workload": kind, "failed": failed, "chi_wall": chi_wall,
           "inputs": "chi %s, sigma = 0, v = 0 at t = 0; l = %g h, dt = 200 t_s, U = 1e-7 L/t_s"
                     % (run["chi"], run["l_cells"]),
           "seconds": ms * steps / 1e3}
    if N in run["paper"]:
        hours, vc_hours, vcycles = run["paper"][N]
        res["paper_context_32_cpu_processes"] = {
            "steps": 5000, "hours": hours, "vcycle_hours": vc_hours, "vcycles": vcycles,
            "s_per_vcycle": vc_hours * 3600 / vcycles}
        if steps == 5000:
            res["paper_hours_over_ours"] = hours * 3600 / res["seconds"]
    if not per_vcycle:
        torch.cuda.empty_cache()
        return res
    sig = stress_field_device(nx, ny, nz, 2, dev)
    gr = MGSolver(nx, ny, nz, h, lam, mu, min_coarse_nz=min_coarse_nz, precision="fp64",
                  device=dev)
    b = gr.rhs(sig, 1.0)
    gr.close()
    del sig
    per_cycle = {}
    for name, prec in (("fp32_ir", "fp32-ir"), ("fp64", "fp64")):
        gs = MGSolver(nx, ny, nz, h, lam, mu, min_coarse_nz=min_coarse_nz, precision=prec,
                      device=dev)
        x = torch.zeros_like(b)
        gs.solve(b, x, rtol=1e-10)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            x.zero_()
            info = gs.solve(b, x, rtol=1e-10)
        torch.cuda.synchronize()
        dts = (time.perf_counter() - t1) / reps
        per_cycle[name] = {"ms_per_solve": dts * 1e3, "cycles": info.cycles,
                           "ms_per_vcycle": dts * 1e3 / max(info.cycles, 1)}
        gs.close()
    del b, x
    torch.cuda.empty_cache()
    res["per_vcycle_from_zero"] = per_cycle
    return res


def weld_run(N: int = 256, steps: int = 500, both: bool = True, n_sub: int = -2) -> dict:
    """Friction welding (Sec. 5) on the slender N x N x N/4 sample (h = 2L/N):
    spinning-disc wall data of Eqs. u_weld and v_weld on both walls
    (omega = 2 pi / 1e8 t_s, R = 1/3), chi from Eq. convolve with mean 450 K,
    std 15 K, l_c = 5h, l = h, dt = 2e4 t_s, the sample at rest at t = 0.
    `steps` FP32-IR projection steps (rtol 1e-10, warm-started) timed between
    device synchronisations, the plastic terms by backward Euler (n_sub = -2;
    500 steps, a tenth of the paper's run).  The explicit forms cannot take
    this dt once the sample flows: with per-cell sub-steps (n_sub = -1) the chi
    diffusion number (dt/c0) 6 D^pl l^2/h^2 passes 1 near step 15, and
    without diffusion the local relaxation near step 38 needs more than 65536
    sub-steps; backward Euler keeps D^pl near the loading rate, which keeps the
    diffusion number small."""
    import math

    import torch

    from paper_1904_03808_amd.qsmg import MGSolver
    from workloads import chi_field, lame, stz_constants, weld_walls
    lam, mu = lame()
    dev = torch.device("cuda:0")
    nx, ny, nz = N, N, N // 4
    h = 2.0 / N
    P, dt, omega = dict(stz_constants(), l_diff=h, n_sub=n_sub), 2e4, 2 * math.pi / 1e8
    lo, hi = (torch.from_numpy(w).to(dev) for w in weld_walls(nx, ny, nz, omega, h, True, both))
    c0 = torch.from_numpy(chi_field(nx, ny, nz, 5, 450.0 / 21000, 15.0 / 21000, 5.0)).to(dev)
    g = MGSolver(nx, ny, nz, h, lam, mu, min_coarse_nz=4, precision="fp32-ir", device=dev)
    v = torch.zeros(g.node_shape(), dtype=torch.float64, device=dev)
    s = torch.zeros((6, nz, ny, nx), dtype=torch.float64, device=dev)
    c = c0.clone()
    g.projection_step_walls(P, dt, lo, hi, v, s, c, rtol=1e-10)  # warm-up (state discarded)
    v.zero_(), s.zero_(), c.copy_(c0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles = [g.projection_step_walls(P, dt, lo, hi, v, s, c, rtol=1e-10).cycles
              for _ in range(steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    p_ = (s[0] + s[1] + s[2]) / 3
    sbar = torch.sqrt(0.5 * ((s[0] - p_) ** 2 + (s[1] - p_) ** 2 + (s[2] - p_) ** 2)
                      + s[3] ** 2 + s[4] ** 2 + s[5] ** 2)
    out = {"grid": [nx, ny, nz], "levels": g.levels, "steps": steps, "ms_per_step": ms,
           "steps_per_s": 1e3 / ms, "vcycles_per_step": sum(cycles) / steps,
           "max_vcycles_in_a_step": max(cycles), "walls": "both" if both else "top",
           "state_at_end": {"t_end": steps * dt,
                            "sbar_max_over_sY": (sbar.max() / P["s_y"]).item()},
           "solver": "fp32-ir, rtol 1e-10",
           "plastic_update": ("backward Euler" if n_sub == -2 else
                              "per-cell sub-steps" if n_sub == -1 else "n_sub = %d" % n_sub),
           "inputs": "chi Eq. convolve (450 K, 15 K, l_c = 5h, seed 5), sigma = 0, v = 0 at t = 0; "
                     "l = h, dt = 2e4 t_s, omega = 2 pi / 1e8 t_s, R = 1/3"}
    g.close()
    del v, s, c, c0, lo, hi, sbar, p_
    torch.cuda.empty_cache()
    return out


def explicit_vs_qs(steps_e: int = 20000, steps_qs: int = 200, zeta: float = 1e4) -> dict:
    """The explicit-versus-quasi-static comparison of Secs. 4.1-4.2 on its
    64 x 64 x 32 grid (h = L/32): chi0 the cylindrical inclusion, tau0 scaled
    to tau0/zeta and U_B = 1e-7 zeta L/t_s, ramped as U_B t/t_s over the first
    t_s (Eq. u_bc), the sample at rest and free of stress at t = 0.
    `steps_e` explicit steps (kappa = 4.8 h, dt = h^2/20, rho = mu/E) and
    `steps_qs` quasi-static steps (dt = 200/zeta t_s, FP32-IR, rtol 1e-10)
    are each timed between device synchronisations from t = 0, and scaled to
    the paper's t_f = 2e6/zeta t_s."""
    import torch

    from paper_1904_03808_amd.qsmg import MGSolver
    from workloads import cylinder_chi, lame, shear_velocity, stz_constants
    lam, mu = lame()
    dev = torch.device("cuda:0")
    nx, ny, nz = 64, 64, 32
    h = 1.0 / nz
    P = stz_constants()
    P = dict(P, tau0=P["tau0"] / zeta)
    UB, tf = 1e-7 * zeta, 2e6 / zeta
    chi0 = torch.from_numpy(cylinder_chi(nx, ny, nz)).to(dev)
    out = {"grid": [nx, ny, nz], "zeta": zeta, "t_f": tf}
    for method in ("explicit", "quasi_static"):
        g = MGSolver(nx, ny, nz, h, lam, mu, min_coarse_nz=4, precision="fp32-ir", device=dev)
        v = torch.from_numpy(shear_velocity(nx, ny, nz, 0.0)).to(dev)
        s = torch.zeros((6, nz, ny, nx), dtype=torch.float64, device=dev)
        c = chi0.clone()
        if method == "explicit":
            dt, n = h * h / 20.0, steps_e
            kappa, rho = 4.8 * h, mu
            g.explicit_step(P, dt, UB * min(dt, 1.0), rho, kappa, v, s, c)  # warm-up step
            v.zero_(), s.zero_(), c.copy_(chi0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(n):
                g.explicit_step(P, dt, UB * min((i + 1) * dt, 1.0), rho, kappa, v, s, c)
            torch.cuda.synchronize()
            cycles = None
        else:
            dt, n = 200.0 / zeta, steps_qs
            g.projection_step(P, dt, UB * min(dt, 1.0), v, s, c, rtol=1e-10)  # warm-up step
            v.zero_(), s.zero_(), c.copy_(chi0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cycles = [g.projection_step(P, dt, UB * min((i + 1) * dt, 1.0), v, s, c,
                                        rtol=1e-10).cycles for i in range(n)]
            torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[method] = {"dt": dt, "steps": n, "t_end": n * dt, "ms_per_step": sec * 1e3 / n,
                       "steps_to_t_f": tf / dt, "projected_s_to_t_f": sec / n * tf / dt,
                       "sigma_xz_mean_at_end": s[4].mean().item()}
        if cycles is not None:
            out[method]["vcycles_per_step"] = sum(cycles) / n
        g.close()
        del v, s, c
    torch.cuda.empty_cache()
    return out


TABLE3_S_PER_VCYCLE = {128: 0.22, 256: 0.76, 384: 2.08, 512: 3.87, 768: 13.88}


def table3_shapes(Ns=(128, 256, 384, 512, 768), reps: int = 3) -> dict:
    """Time per V-cycle on the paper's N x N x N/2 grids (Table 3: N = 128 to
    768, h = L/(N/2)), FP32-IR and FP64: solves from zero of b = D_h sigma
    (smoothed random stress generated on the device, seed 2) to 1e-10, `reps`
    timed after one warm-up, divided by the cycles taken.  Coarsening stops at
    nz <= 4 (8 x 8 x 4 or 6 x 6 x 3 coarsest)."""
    import torch

    from paper_1904_03808_amd.qsmg import MGSolver
    from workloads import lame, stress_field_device
    lam, mu = lame()
    dev = torch.device("cuda:0")
    out = {}
    for N in Ns:
        nx, ny, nz = N, N, N // 2
        h = 1.0 / nz
        sig = stress_field_device(nx, ny, nz, 2, dev)
        g64 = MGSolver(nx, ny, nz, h, lam, mu, min_coarse_nz=4, precision="fp64", device=dev)
        b = g64.rhs(sig, 1.0)
        del sig
        row = {"grid": [nx, ny, nz], "levels": g64.levels,
               "paper_s_per_vcycle_32_cpu_processes": TABLE3_S_PER_VCYCLE.get(N)}
        for name, prec in (("fp32_ir", "fp32-ir"), ("fp64", "fp64")):
            g = g64 if prec == "fp64" else MGSolver(nx, ny, nz, h, lam, mu, min_coarse_nz=4,
                                                    precision=prec, device=dev)
            x = torch.zeros_like(b)
            g.solve(b, x, rtol=1e-10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                x.zero_()
                info = g.solve(b, x, rtol=1e-10)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            row[name] = {"ms_per_solve": ms, "cycles": info.cycles, "rel_res": info.rel_res,
                         "ms_per_vcycle": ms / max(info.cycles, 1)}
            if g is not g64:
                g.close()
            del x
        g64.close()
        del b
        torch.cuda.empty_cache()
        p = row["paper_s_per_vcycle_32_cpu_processes"]
        if p:
            row["paper_over_fp64"] = p * 1e3 / row["fp64"]["ms_per_vcycle"]
        out["N%d" % N] = row
        print("table3 shape N=%d done" % N, file=sys.stderr, flush=True)
    return out


def profile_solve(n: int, precision: str = "fp32-ir") -> None:
    """Kernels for hardware-counter runs of a whole V-cycle: two cycles (fixed
    count, no convergence test) of the n^3 bench system, FP32-IR or FP64."""
    import torch

    from paper_1904_03808_amd.qsmg import MGSolver
    from workloads import lame, stress_field
    lam, mu = lame()
    dev = torch.device("cuda:0")
    g = MGSolver(n, n, n, 1.0 / n, lam, mu, precision=precision, device=dev)
    sig_host = stress_field(n, n, n, 2)
    sig = torch.from_numpy(sig_host).to(dev)
    b = g.rhs(sig, 1.0)
    del sig
    x = torch.zeros_like(b)
    g.solve(b, x, rtol=0.0, max_cycles=2, raise_on_failure=False)
    torch.cuda.synchronize()
    print(json.dumps({"profiled": precision + " solve", "cycles": 2}), flush=True)


def profile_step(n: int) -> None:
    """Kernels for hardware-counter runs of the projection step's cell kernels
    at n^3 (shear state, chi seed 3, dt = 10 t_s): the STZ step plain, with
    the stress advection, and with advection and chi diffusion (l = h), then
    the right-hand side and the stress correction, each called twice."""
    import torch

    from paper_1904_03808_amd.qsmg import MGSolver
    from workloads import lame, shear_state, stz_constants
    lam, mu = lame()
    P = stz_constants()
    st = shear_state(n, n, n, seed=3, U=1e-5)
    g = MGSolver(n, n, n, 1.0 / n, lam, mu, precision="fp32-ir", device="cuda:0")
    v, s, c = (torch.from_numpy(st[k]).to("cuda:0") for k in ("v", "sigma", "chi"))
    del st
    for name, p in (("plain", P), ("advect", dict(P, advect=1)),
                    ("advect+diffusion", dict(P, advect=1, l_diff=1.0 / n))):
        for _ in range(2):
            sstar, _ = g.stz_step(p, 10.0, v, s, c)
        torch.cuda.synchronize()
        print(json.dumps({"profiled": "stz_step " + name}), flush=True)
    for _ in range(2):
        b = g.rhs(sstar, 10.0)
        g.stress_update(sstar, v, 10.0)
    torch.cuda.synchronize()
    print(json.dumps({"profiled": "rhs, stress_update"}), flush=True)


def profile_smoother(n: int) -> None:
    """Kernels for hardware-counter runs: one device-to-device copy of a known
    size (calibrates FETCH_SIZE / WRITE_SIZE), then 3 fine-level sweeps in FP32
    and in FP64 (6 half-sweep launches each) on the 256^3 bench input."""
    import torch

    from paper_1904_03808_amd.qsmg import MGSolver
    from workloads import lame, stress_field
    lam, mu = lame()
    dev = torch.device("cuda:0")
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)  # 512 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    sig_host = stress_field(n, n, n, 2)
    sig = torch.from_numpy(sig_host).to(dev)
    for prec, dt_ in (("fp32-ir", torch.float32), ("fp64", torch.float64)):
        g = MGSolver(n, n, n, 1.0 / n, lam, mu, precision="fp64", device=dev)
        b = g.rhs(sig, 1.0)
        g.close()
        g = MGSolver(n, n, n, 1.0 / n, lam, mu, precision=prec, device=dev)
        xs = torch.zeros(g.node_shape(0), dtype=dt_, device=dev)
        g.smooth(0, xs, b.to(dt_), 3)
        torch.cuda.synchronize()
        print(json.dumps({"profiled": prec, "sweeps": 3, "copy_bytes": 512 * 1024 * 1024}),
              flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-512", action="store_true", help="skip the 512^3 comparison block")
    ap.add_argument("--no-steps", action="store_true",
                    help="skip the shear-step (256^3) and adjoint (96^3) blocks")
    ap.add_argument("--no-defect", action="store_true",
                    help="skip the single-defect (256 x 256 x 128) and welding (256 x 256 x 64) blocks")
    ap.add_argument("--defect-steps", type=int, default=5000,
                    help="projection steps of the single-defect block (the paper's whole run)")
    ap.add_argument("--defect-only", action="store_true",
                    help="only run the single-defect and welding blocks and print them")
    ap.add_argument("--no-table3", action="store_true",
                    help="skip the V-cycle timing on the paper's N x N x N/2 grids (N = 128..768)")
    ap.add_argument("--paper-run", choices=sorted(PAPER_RUNS),
                    help="only run one of the paper's simple-shear runs (see --paper-n, "
                         "--defect-steps) and print it")
    ap.add_argument("--paper-n", type=int, default=256, help="N of the N x N x N/2 grid")
    ap.add_argument("--min-coarse-nz", type=int, default=4,
                    help="coarsening limit of the paper runs (8 for N = 80: 80 x 80 x 40 halves to nz = 5)")
    ap.add_argument("--chi-wall", type=int, default=0, choices=(0, 1),
                    help="chi diffusion at the walls: 0 ghost-state D^pl, 1 the wall cell's own")
    ap.add_argument("--explicit-only", action="store_true",
                    help="only run the explicit-versus-quasi-static block (64 x 64 x 32)")
    ap.add_argument("--table3-only", action="store_true",
                    help="only time V-cycles on the paper's N x N x N/2 grids and print them")
    ap.add_argument("--profile-solve", action="store_true",
                    help="only run two FP32-IR V-cycles (for rocprofv3 counters)")
    ap.add_argument("--profile-solve-fp64", action="store_true",
                    help="only run two FP64 V-cycles (for rocprofv3 counters)")
    ap.add_argument("--profile-smoother", action="store_true",
                    help="only run a calibration copy and fine-level sweeps (for rocprofv3 counters)")
    ap.add_argument("--profile-step", action="store_true",
                    help="only run the projection step's cell kernels (for rocprofv3 counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1904_03808_amd.qsmg import MGSolver
    from workloads import lame, stress_field

    if args.profile_smoother:
        profile_smoother(args.n)
        return
    if args.profile_solve or args.profile_solve_fp64:
        profile_solve(args.n, "fp64" if args.profile_solve_fp64 else "fp32-ir")
        return
    if args.profile_step:
        profile_step(args.n)
        return
    if args.paper_run:
        print(json.dumps({"paper_run": defect_run(N=args.paper_n, steps=args.defect_steps,
                                                  kind=args.paper_run, per_vcycle=False,
                                                  chi_wall=args.chi_wall,
                                                  min_coarse_nz=args.min_coarse_nz)}))
        return
    if args.explicit_only:
        print(json.dumps({"explicit_vs_qs_64x64x32": explicit_vs_qs()}))
        return
    if args.table3_only:
        print(json.dumps({"table3_shapes": table3_shapes()}))
        return
    if args.defect_only:
        print(json.dumps({"defect_256x256x128": defect_run(steps=args.defect_steps),
                          "weld_256x256x64": weld_run(),
                          "explicit_vs_qs_64x64x32": explicit_vs_qs()}))
        return
    n = args.n
    h = 1.0 / n
    lam, mu = lame()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sig_host = stress_field(n, n, n, 2)
    sig = torch.from_numpy(sig_host).to(dev)
    g64 = MGSolver(n, n, n, h, lam, mu, precision="fp64", device=dev)
    g32 = MGSolver(n, n, n, h, lam, mu, precision="fp32-ir", device=dev)
    b = g64.rhs(sig, 1.0)
    del sig
    x = torch.zeros_like(b)
    nodes = n * n * (n - 1)  # interior nodes

    def run(g):
        x.zero_()
        return g.solve(b, x, rtol=1e-10)

    results = {}
    for name, g in (("fp32_ir", g32), ("fp64", g64)):
        for _ in range(args.warmup):
            run(g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [run(g) for _ in range(args.steps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        results[name] = {"ms_per_solve": dt * 1e3, "solves_per_s": 1.0 / dt,
                         "cycles": infos[-1].cycles, "rel_res": infos[-1].rel_res,
                         "ms_per_cycle": dt * 1e3 / max(infos[-1].cycles, 1)}
        results[name + "_x"] = x.clone()
    err = (torch.linalg.vector_norm(results["fp32_ir_x"] - results["fp64_x"])
           / torch.linalg.vector_norm(results["fp64_x"])).item()
    vs_oracle = _block(lambda: error_vs_oracle(n, {k: results[k + "_x"] for k in ("fp32_ir", "fp64")}))
    del results["fp32_ir_x"], results["fp64_x"]

    # smoother on its own: fine level, full sweeps, HIP events on the same stream
    sm = {"fp32": smoother_timing(g32, b, torch.float32, 36.0),
          "fp64": smoother_timing(g64, b, torch.float64, 72.0)}
    # roofline kernel: one FP32 half sweep; algorithmic bytes per launch =
    # 36 B x (interior nodes / 2), over the average launch time from HIP events
    algo_bytes = 36.0 * nodes / 2
    achieved = algo_bytes / (sm["fp32"]["avg_launch_us"] * 1e-6) / 1e9
    traffic = sweep_traffic(n)
    # measured streaming reference: a 1 GiB device-to-device tensor copy
    # (read + write bytes over its event time)
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    copy_ms = _events_ms(lambda: dst.copy_(src), 10)
    copy_gbs = 2.0 * src.numel() * 4 / (copy_ms * 1e-3) / 1e9
    del src, dst
    out = {
        "metric": METRIC,
        "value": results["fp32_ir"]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": results["fp32_ir"]["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "projection-system solve %d^3 cells, x,y periodic, z Dirichlet; "
                               "b = D_h sigma, sigma smoothed N(0,1) (seed 2); x0 = 0; "
                               "rtol 1e-10; V(2,2), %d levels" % (n, g32.levels),
                   "grid": [n, n, n], "levels": g32.levels, "rtol": 1e-10,
                   "solver": "FP32 V-cycles in FP64 iterative refinement",
                   "parallelism": "single GPU"},
        "fp32_ir": results["fp32_ir"],
        "fp64": results["fp64"],
        "speedup_fp32ir_vs_fp64": results["fp64"]["ms_per_solve"] / results["fp32_ir"]["ms_per_solve"],
        "fp32ir_vs_fp64_rel_l2": err,
        "error_vs_fp64_oracle": vs_oracle,
        "smoother": sm,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_sweep_rows<float, 256, 0, 0>: fine-level FP32 half sweep",
                     "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "algorithmic_bytes_per_launch": algo_bytes,
                     "bytes_per_node_update": 36,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE)",
                     "traffic_GBs": (traffic / (sm["fp32"]["avg_launch_us"] * 1e-6) / 1e9
                                     if traffic else None)},
    }
    if not args.no_512 and n == 256:
        out["config2_512"] = _block(config_512)
    if not args.no_steps and n == 256:
        out["config3_shear_256"] = _block(config3_shear)
        out["config4_adjoint_96"] = _block(config4_adjoint)
    if not args.no_defect and n == 256:
        out["defect_256x256x128"] = _block(lambda: defect_run(steps=args.defect_steps))
    if not args.no_defect and n == 256:
        out["weld_256x256x64"] = _block(weld_run)
        out["explicit_vs_qs_64x64x32"] = _block(explicit_vs_qs)
    if not args.no_table3 and n == 256:
        out["table3_shapes"] = _block(table3_shapes)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _block(lambda: cpu_baseline(sig_host, n, results["fp64"]["cycles"]))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
