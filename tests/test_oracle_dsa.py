"""Pins of the oracle's thick-region diffusion operator (eq. SIP, Sec. 3.1; Sec. 3.2).

P13 the assembled D_ff equals a pointwise-quadrature evaluation of the SIP
    bilinear form (principal submatrix semantics), is symmetric and SPD, and
    satisfies D 1 = sigma_a M 1 on thick cells whose faces are all thick.
P14 the CG correction equals a dense solve.
P15 heterogeneous DSA is not a global DSA solve restricted to the thick DOFs
    (Section 2.3).
"""
import math

import numpy as np
import pytest

import bruteforce as bf
import oracle
import sninputs
from sninputs import Problem


def _mixed(dim, n, seed):
    rng = np.random.default_rng(seed)
    nc = n ** dim
    kind = rng.integers(0, 3, nc)           # 0 void, 1 thin, 2 thick
    st = np.where(kind == 2, rng.uniform(20, 300, nc), np.where(kind == 1, rng.uniform(0.5, 2, nc), 0.0))
    ss = np.where(kind == 2, st * rng.uniform(0.95, 0.999, nc), np.where(kind == 1, 0.5 * st, 0.0))
    om, w = sninputs.level_symmetric(4, dim)
    nz = n if dim == 3 else 1
    h = (1.0, 0.8, 1.2) if dim == 3 else (1.0, 0.8, 1.0)
    return Problem("mix", dim, n, n, nz, h, st, ss, np.ones(nc), om, w)


@pytest.mark.parametrize("dim,n,seed", [(2, 4, 0), (2, 5, 1), (3, 3, 2)])
def test_p13_matrix_vs_quadrature(dim, n, seed):
    p = _mixed(dim, n, seed)
    D, cells = oracle.dsa_dense(p)
    Dq, cq = bf.sip_matrix(p, p.eta)
    assert np.array_equal(cells, cq)
    assert np.allclose(D, Dq, rtol=1e-12, atol=1e-14 * np.max(np.abs(Dq)))
    assert np.allclose(D, D.T, atol=1e-15 * np.max(np.abs(D)))
    ev = np.linalg.eigvalsh(0.5 * (D + D.T))
    assert ev.min() > 0


def test_p13_interior_row_sums():
    n = 6
    p = _mixed(2, n, 5)
    st = np.full(p.ncells, 200.0)
    ss = np.full(p.ncells, 199.9)
    ss[0] = 0.5                      # one thin corner cell
    p = Problem("rs", 2, n, n, 1, p.h, st, ss, np.ones(p.ncells), p.omega, p.w)
    D, cells = oracle.dsa_dense(p)
    ones = np.ones(len(cells) * p.nn)
    y = D @ ones
    Ma = bf.mass_matrix(p, p.sigma_t - p.sigma_s)
    ref = Ma @ np.ones(p.ncells * p.nn)
    for s, c in enumerate(cells):
        i, j = c % n, c // n
        if 1 <= i <= n - 2 and 1 <= j <= n - 2 and not (i == 1 and j == 1) and c not in (1, n):
            assert np.allclose(y[s * 4:(s + 1) * 4], ref[c * 4:(c + 1) * 4], rtol=1e-12)


@pytest.mark.parametrize("mass_kind", [0, 1])
def test_p14_cg_vs_dense(mass_kind):
    p = _mixed(2, 6, 3)
    rng = np.random.default_rng(9)
    phi_old = rng.uniform(0, 1, (p.ncells, p.nn))
    phi_si = rng.uniform(0, 1, (p.ncells, p.nn))
    out, it, rr = oracle.dsa_correct(p, phi_old, phi_si, mass_kind=mass_kind, cg_rtol=1e-14)
    D, cells = oracle.dsa_dense(p)
    coef = p.sigma_t if mass_kind == 1 else p.sigma_s
    M = bf.mass_matrix(p, coef)
    b = (M @ (phi_si - phi_old).ravel()).reshape(p.ncells, p.nn)[cells].ravel()
    delta = np.linalg.solve(D, b)
    ref = phi_si.copy()
    ref[cells] += delta.reshape(-1, p.nn)
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))
    thin = np.setdiff1d(np.arange(p.ncells), cells)
    assert np.array_equal(out[thin], phi_si[thin])


def test_p15_het_differs_from_restricted_global():
    n = 8
    st = np.full(n * n, 1.0)
    ss = np.full(n * n, 0.5)
    for j in range(2, 6):
        for i in range(2, 6):
            st[j * n + i], ss[j * n + i] = 100.0, 99.9
    om, w = sninputs.level_symmetric(4, 2)
    p = Problem("p15", 2, n, n, 1, (1.0, 1.0, 1.0), st, ss, np.ones(n * n), om, w)
    rng = np.random.default_rng(2)
    r = rng.uniform(0, 1, (p.ncells, p.nn))
    z = np.zeros_like(r)
    het, _, _ = oracle.dsa_correct(p, z, r, eta=1.0)
    glob, _, _ = oracle.dsa_correct(p, z, r, eta=0.0)
    thick = p.sigma_s >= 1.0
    dh = het[thick] - r[thick]
    dg = glob[thick] - r[thick]
    assert np.linalg.norm(dh - dg) > 1e-3 * np.linalg.norm(dg)
