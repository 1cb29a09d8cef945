"""Pins of the oracle's discrete operators against closed forms and invariants.

Operator: paper Sec. 3.3 (Eq. proj) discretised with Eq. col_snd_deriv and the
mixed-derivative stencil of Sec. 3.4; staggered differences: Eq. stag_stenc.
"""
import numpy as np
import pytest

from oracle.operators import (apply_elastic, assemble_elastic, div_node, grad_cell,
                              interior_mask, voigt_to_full)
from workloads import lame, manufactured_source, manufactured_velocity

LAM, MU = lame()


@pytest.mark.parametrize("n", [(8, 8, 8), (6, 10, 4)])
def test_fourier_symbol(n):
    """K applied to a Fourier mode equals the closed-form 3x3 symbol times the mode.

    h^2 (K v)_c = sum_d S_cd a_d e^{i theta.p},
    S_cc = sum_a kappa_ca 4 sin^2(theta_a/2),  S_cd = (lam+mu) sin(theta_c) sin(theta_d).
    """
    nx, ny, nz = n
    h = 0.37
    rng = np.random.default_rng(1)
    for trial in range(4):
        th = np.array([2 * np.pi * rng.integers(0, nx) / nx,
                       2 * np.pi * rng.integers(0, ny) / ny,
                       rng.uniform(-np.pi, np.pi)])
        a = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny), np.arange(nx), indexing="ij")
        phase = np.exp(1j * (th[0] * i + th[1] * j + th[2] * k))
        v = a[:, None, None, None] * phase[None]
        Kv = apply_elastic(v, h, LAM, MU)
        kap = np.array([[LAM + 2 * MU if c == d else MU for d in range(3)] for c in range(3)])
        S = np.empty((3, 3))
        for c in range(3):
            for d in range(3):
                if c == d:
                    S[c, d] = sum(kap[c, q] * 4 * np.sin(th[q] / 2) ** 2 for q in range(3))
                else:
                    S[c, d] = (LAM + MU) * np.sin(th[c]) * np.sin(th[d])
        expect = (S @ a)[:, None, None, None] * phase[None] / h ** 2
        err = np.abs(Kv[:, 1:nz] - expect[:, 1:nz]).max()
        assert err <= 1e-12 * np.abs(expect).max() + 1e-12


@pytest.mark.parametrize("n", [4, 8])
def test_symmetric_positive_definite_not_dominant(n):
    """Sec. 3.3: the system is symmetric positive definite but not diagonally dominant."""
    h = 1.0 / n
    K = assemble_elastic(n, n, n, h, LAM, MU)
    m = interior_mask(n, n, n)
    A = K[m][:, m].toarray()
    assert np.abs(A - A.T).max() == 0.0
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > 0.0
    off = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
    assert (off > np.abs(np.diag(A))).sum() > 0.5 * A.shape[0]
    # 15 scalar couplings per row away from the walls (45 per node)
    full = K[m]
    nnz = np.diff(full.indptr)
    assert nnz.max() == 15


def test_sparse_matches_matrix_free():
    rng = np.random.default_rng(2)
    for (nx, ny, nz) in [(4, 6, 4), (8, 8, 6), (2, 4, 4)]:
        h = 1.0 / nz
        v = rng.standard_normal((3, nz + 1, ny, nx))
        K = assemble_elastic(nx, ny, nz, h, LAM, MU)
        a = (K @ v.ravel()).reshape(v.shape)
        b = apply_elastic(v, h, LAM, MU)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def test_summation_by_parts():
    """<G_h v, tau>_cells = -<v, D_h tau>_nodes for v vanishing on the walls."""
    rng = np.random.default_rng(3)
    nx, ny, nz = 6, 4, 5
    h = 0.3
    v = rng.standard_normal((3, nz + 1, ny, nx))
    v[:, 0] = 0
    v[:, -1] = 0
    tau = rng.standard_normal((6, nz, ny, nx))
    L = grad_cell(v, h)
    T = voigt_to_full(tau)
    lhs = np.sum(L * T)
    rhs = -np.sum(v * div_node(tau, h))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_special_cases():
    """D_h of a uniform stress vanishes; G_h of a linear velocity is exact."""
    rng = np.random.default_rng(4)
    nx, ny, nz = 6, 6, 6
    h = 1.0 / nz
    s = np.ones((6, nz, ny, nx)) * rng.standard_normal(6)[:, None, None, None]
    assert np.abs(div_node(s, h)).max() < 1e-12
    # a linear field that is periodic in x, y can only vary in z
    g = rng.standard_normal(3)
    c0 = rng.standard_normal(3)
    zk = np.arange(nz + 1) * h
    v = np.zeros((3, nz + 1, ny, nx))
    for a in range(3):
        v[a] = (c0[a] + g[a] * zk)[:, None, None]
    L = grad_cell(v, h)
    for a in range(3):
        for b in range(3):
            expect = g[a] if b == 2 else 0.0
            assert np.abs(L[a, b] - expect).max() < 1e-12
    # K annihilates a z-linear velocity (the simple-shear profile)
    assert np.abs(apply_elastic(v, h, LAM, MU)).max() < 1e-9


def test_manufactured_consistency():
    """K u_exact - f = O(h^2) for the manufactured velocity (Eq. col_snd_deriv is 2nd order)."""
    errs = []
    for n in (16, 32):
        h = 1.0 / n
        u = manufactured_velocity(n, n, n)
        f = manufactured_source(n, n, n, LAM, MU)
        d = apply_elastic(u, h, LAM, MU) - f
        errs.append(np.sqrt(np.mean(d[:, 1:n] ** 2)) / np.sqrt(np.mean(f[:, 1:n] ** 2)))
    order = np.log2(errs[0] / errs[1])
    assert 1.8 < order < 2.2, errs
