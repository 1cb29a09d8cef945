"""Pins of the STZ magnitudes in SI units (paper Sec. 3.1, Eqs. stz_dpl,
stz_R, stz_C_form, chi_evo; Table 1; t_s = L/c_s of Sec. 4).

The oracle works in units of E (stress), t_s (time), L (length) and e_z/k_B
(chi).  These tests restate the model in SI units straight from the printed
Table 1 values (`tests/golden/table1.json`), with the rates of Eq. stz_R in
their exponential form and the stiffness as the fourth-order isotropic tensor,
and compare the oracle with the result after converting units.  A mistake in
the exponent of chi, in where tau0 enters, in the cosh argument, in the
conversion of beta or in the factor of the dissipation D^pl : sigma_0 changes
the answer by far more than the tolerance; `test_pins_reject_mutants` applies
each such mistake to the oracle's own source and checks that the pin fails.
"""
import inspect
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import stz

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
KB = 1.380649e-23  # J/K, exact by the SI definition
L_M = 0.01  # sample length L = 1 cm (Sec. 4)


def _table1():
    g = json.load(open(os.path.join(GOLDEN, "table1.json")))
    E = g["E_GPa"] * 1e9
    mu = E / (2.0 * (1.0 + g["nu"]))
    lam = E * g["nu"] / ((1.0 + g["nu"]) * (1.0 - 2.0 * g["nu"]))
    t_s = L_M / math.sqrt(mu / g["rho_kg_m3"])
    return dict(E=E, mu=mu, lam=lam, t_s=t_s, s_y=g["s_Y_GPa"] * 1e9, tau0=g["tau0_s"],
                eps0=g["eps0"], c0=g["c0"], Delta=g["Delta_over_kB_K"] * KB,
                Omega=g["Omega_A3"] * 1e-30, T=g["T_K"], chi_inf=g["chi_inf_K"],
                ez=g["ez_over_kB_K"] * KB, t_s_printed=g["t_s_us_printed"] * 1e-6)


T1 = _table1()


def dpl_si(sbar_pa, chi_k):
    """D^pl in 1/s: Eq. stz_dpl with C = (R(+s) + R(-s))/2 and the rates of
    Eq. stz_R, R(+-s) = exp(-(Delta -+ Omega eps0 s)/(k_B T))."""
    kT = KB * T1["T"]
    Rp = math.exp(-(T1["Delta"] - T1["Omega"] * T1["eps0"] * sbar_pa) / kT)
    Rm = math.exp(-(T1["Delta"] + T1["Omega"] * T1["eps0"] * sbar_pa) / kT)
    C = 0.5 * (Rp + Rm)
    if sbar_pa <= T1["s_y"]:
        return 0.0
    return math.exp(-T1["ez"] / (KB * chi_k)) * C * (1.0 - T1["s_y"] / sbar_pa) / T1["tau0"]


def si_step(sig_pa, chi_k, dt_s):
    """One forward-Euler step of the plastic terms with L = 0 in SI units:
    sigma* = sigma - dt C : D^pl (Eq. sig_star_qs), and
    chi' = chi + (dt/c0) (D^pl : sigma_0 / s_Y)(chi_inf - chi) (Eq. chi_evo, l = 0),
    D^pl = D^pl sigma_0 / sbar, with the full contractions written out."""
    S = np.asarray(sig_pa, dtype=float)
    S0 = S - np.trace(S) / 3.0 * np.eye(3)
    sbar = math.sqrt(0.5 * sum(S0[i, j] ** 2 for i in range(3) for j in range(3)))
    Dt = dpl_si(sbar, chi_k) * S0 / sbar
    d = np.eye(3)
    Cijkl = (T1["lam"] * np.einsum("ij,kl->ijkl", d, d)
             + T1["mu"] * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))
    CD = np.einsum("ijkl,kl->ij", Cijkl, Dt)
    diss = sum(Dt[i, j] * S0[i, j] for i in range(3) for j in range(3))
    chi1 = chi_k + dt_s / T1["c0"] * (diss / T1["s_y"]) * (T1["chi_inf"] - chi_k)
    return S - dt_s * CD, chi1


# states: (sbar / s_Y, chi in K)
STATES = [(1.05, 800.0), (1.05, 1050.0), (1.2, 950.0), (1.6, 700.0), (1.01, 550.0)]


def _anisotropic(ratio):
    """A symmetric stress (Pa) with all six components non-zero, a pressure,
    and sbar = ratio * s_Y."""
    A = np.array([[0.3, 0.5, -0.2], [0.5, -0.4, 0.6], [-0.2, 0.6, 0.9]])
    A0 = A - np.trace(A) / 3.0 * np.eye(3)
    sb = math.sqrt(0.5 * np.sum(A0 * A0))
    return A0 * (ratio * T1["s_y"] / sb) + 0.37 * T1["s_y"] * np.eye(3)


def _voigt(S):
    return np.array([S[0, 0], S[1, 1], S[2, 2], S[1, 2], S[0, 2], S[0, 1]])


def pin_beta(P):
    beta_si = T1["Omega"] * T1["eps0"] * T1["E"] / (KB * T1["T"])
    return abs(P["beta"] - beta_si) / beta_si


def pin_dpl(plastic_rate, P):
    """Largest relative difference of the oracle's D^pl (nondimensional) and
    the SI value times t_s over STATES."""
    err = 0.0
    for ratio, chi_k in STATES:
        ref = dpl_si(ratio * T1["s_y"], chi_k) * T1["t_s"]
        got = float(plastic_rate(np.array([ratio * T1["s_y"] / T1["E"]]),
                                 np.array([chi_k / 21000.0]), P)[0])
        err = max(err, abs(got - ref) / ref)
    return err


def pin_step(stz_pointwise, P):
    """Relative errors of the stress and chi increments of one step with
    L = 0 on an anisotropic stress, oracle against the SI restatement."""
    es, ec = 0.0, 0.0
    for ratio, chi_k in STATES:
        S = _anisotropic(ratio)
        ref_rate = dpl_si(ratio * T1["s_y"], chi_k)
        dt_s = 0.02 * ratio * T1["s_y"] / (2.0 * T1["mu"] * ref_rate)  # sbar drops by ~2 %
        S1, chi1 = si_step(S, chi_k, dt_s)
        sig = (_voigt(S) / T1["E"])[:, None]
        L = np.zeros((3, 3, 1))
        sstar, chin = stz_pointwise(L, sig, np.array([chi_k / 21000.0]), dt_s / T1["t_s"],
                                    T1["lam"] / T1["E"], T1["mu"] / T1["E"], P)
        d_ref = (_voigt(S1) - _voigt(S)) / T1["E"]
        d_got = sstar[:, 0] - sig[:, 0]
        es = max(es, np.abs(d_got - d_ref).max() / np.abs(d_ref).max())
        c_ref = (chi1 - chi_k) / 21000.0
        assert c_ref != 0.0  # every state lies off chi_inf
        ec = max(ec, abs((chin[0] - chi_k / 21000.0) - c_ref) / abs(c_ref))
    return es, ec


def test_time_unit_matches_printed():
    """t_s = L/c_s from Table 1's E, nu, rho agrees with the printed 4.05 us."""
    assert abs(T1["t_s"] - T1["t_s_printed"]) < 0.005e-6


def test_beta_from_table1():
    """beta = Omega eps0 E/(k_B T) from the printed Omega = 300 A^3, eps0 = 0.3,
    E = 101 GPa, T = 400 K; about 1645.97."""
    P = workloads.stz_constants()
    assert pin_beta(P) < 1e-13
    assert abs(P["beta"] - 1645.97) < 0.005


def test_plastic_rate_matches_si_rates():
    """D^pl of Eq. stz_dpl with the two stress-biased rates of Eq. stz_R, in
    SI units from Table 1, converted by t_s, equals the oracle's D^pl."""
    assert pin_dpl(stz.plastic_rate, workloads.stz_constants()) < 1e-12


def test_plastic_rate_literal_values():
    """The SI restatement itself at two states, against values worked out by
    hand from Table 1 (s = 1.05 s_Y; chi = 1050 K and 800 K):
    tau0 D^pl = exp(-21000/chi) exp(-20) cosh(beta s/E) (1 - 1/1.05)."""
    s = 1.05 * 0.85e9
    x = 300e-30 * 0.3 * s / (KB * 400.0)
    for chi_k in (1050.0, 800.0):
        by_hand = math.exp(-21000.0 / chi_k) * math.exp(-20.0) * math.cosh(x) * (1 - 1 / 1.05) / 1e-13
        assert dpl_si(s, chi_k) == pytest.approx(by_hand, rel=1e-13)
    # orders of magnitude: about 2.2 / s at 1050 K and 4.3e-3 / s at 800 K
    assert 2.0 < dpl_si(s, 1050.0) < 2.5
    assert 3.5e-3 < dpl_si(s, 800.0) < 5.0e-3


def test_step_increments_match_si_contraction():
    """sigma* - sigma = -dt C : D^pl and the chi increment with the full
    contraction D^pl : sigma_0 of Eq. chi_evo (not its shortcut 2 sbar D^pl),
    on an anisotropic stress with pressure, agree with the oracle's step."""
    es, ec = pin_step(stz.stz_pointwise, workloads.stz_constants())
    assert es < 1e-11 and ec < 1e-11, (es, ec)


def _mutant(module, name, old, new):
    src = inspect.getsource(getattr(module, name))
    assert src.count(old) == 1, (name, old)
    ns = dict(vars(module))
    exec(compile(src.replace(old, new), "<mutant %s>" % name, "exec"), ns)
    return ns[name]


def test_pins_reject_mutants():
    """Each plausible mistake, applied to the oracle's own source, fails a pin."""
    P = workloads.stz_constants()
    mutants = {
        "exp(-chi) for exp(-1/chi)": _mutant(stz, "plastic_rate", "np.exp(-1.0 / chi)", "np.exp(-chi)"),
        "tau0 multiplied": _mutant(stz, "plastic_rate", '/ p["tau0"]', '* p["tau0"]'),
        "1 + s_Y/sbar": _mutant(stz, "plastic_rate", '(1.0 - p["s_y"] / sb)', '(1.0 + p["s_y"] / sb)'),
    }
    for what, fn in mutants.items():
        assert pin_dpl(fn, P) > 1e-3, what
    # a beta converted with mu instead of E, or with k_B dropped to k_B T / 2
    const_mutants = {
        "beta with mu": ("beta=Omega_m3 * eps0 * E_Pa / (kB * T_K)",
                         "beta=Omega_m3 * eps0 * mu_Pa / (kB * T_K)"),
        "beta halved": ("beta=Omega_m3 * eps0 * E_Pa / (kB * T_K)",
                        "beta=Omega_m3 * eps0 * E_Pa / (2 * kB * T_K)"),
    }
    for what, (old, new) in const_mutants.items():
        Pm = _mutant(workloads, "stz_constants", old, new)()
        assert pin_beta(Pm) > 1e-3 and pin_dpl(stz.plastic_rate, Pm) > 1e-3, what
    # the cosh argument and the dissipation's factor 2
    rate_m = _mutant(stz, "transition_rate", 'p["beta"] * sbar', 'p["beta"] * sbar * 0.5')
    pr = _mutant(stz, "plastic_rate", "transition_rate(sb, p)", "rate_m(sb, p)")
    pr.__globals__["rate_m"] = rate_m
    assert pin_dpl(pr, P) > 1e-3
    step_m = _mutant(stz, "stz_pointwise", "2.0 * sbar * Dpl", "sbar * Dpl")
    es, ec = pin_step(step_m, P)
    assert ec > 1e-3 and es < 1e-11
    step_m2 = _mutant(stz, "stz_pointwise", "stiffness(ratio * S0, lam, mu)",
                      "stiffness(ratio * S0, lam, 0.5 * mu)")
    es, ec = pin_step(step_m2, P)
    assert es > 1e-3
