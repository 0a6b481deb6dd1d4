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


# ---------------------------------------------------------------------------
# the nonsymmetric forms of Sec. 3.1: NIP (eq. NIP) and mNIP (eq. ModifiedF0)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("form,op", [("nip", oracle.DSA_NIP), ("mnip", oracle.DSA_MNIP)])
@pytest.mark.parametrize("dim,n,seed", [(2, 4, 0), (3, 3, 2)])
def test_n1_nonsymmetric_forms_vs_quadrature(form, op, dim, n, seed):
    """NIP and mNIP against a pointwise-quadrature assembly with the term
    -int [[u]]{D dv/dn} left out (void cells made thin: eq. ModifiedF0 needs
    sigma_t > 0)."""
    p = _mixed(dim, n, seed)
    p.sigma_t[p.sigma_t == 0.0] = 0.05
    D, cells = oracle.dsa_dense(p, dsa_op=op)
    Dq, cq = bf.sip_matrix(p, p.eta, form=form)
    assert np.array_equal(cells, cq)
    assert np.allclose(D, Dq, rtol=1e-12, atol=1e-14 * np.max(np.abs(Dq)))
    assert not np.allclose(D, D.T, atol=1e-6 * np.max(np.abs(D)))       # really nonsymmetric


@pytest.mark.parametrize("dim,n,seed", [(2, 5, 1), (3, 3, 2)])
def test_n1_structure_of_the_dropped_term(dim, n, seed):
    """Structure that fixes which term NIP leaves out.  With one and the same
    penalty kappa_0, SIP = A0 + C + C^T and NIP = A0 + C, with A0 symmetric
    (volume, mass and penalty terms) and C the consistency term
    -int {D du/dn}[[v]]; so X = SIP - NIP is C^T and NIP - X^T = A0 must be
    symmetric, while X itself is not (a dropped term of the wrong sign, or
    the consistency term dropped in place of the symmetry term, breaks one of
    the two).  The mNIP and NIP matrices differ by a penalty, which is
    symmetric."""
    p = _mixed(dim, n, seed)
    p.sigma_t[p.sigma_t == 0.0] = 0.05
    Dn, _ = oracle.dsa_dense(p, dsa_op=oracle.DSA_NIP)
    Ds0, _ = bf.sip_matrix(p, p.eta, form="sip", ckappa=0.0)
    sc = np.max(np.abs(Dn))
    X = Ds0 - Dn
    assert np.max(np.abs(X)) > 1e-3 * sc
    assert not np.allclose(X, X.T, atol=1e-6 * sc)
    A0 = Dn - X.T
    assert np.allclose(A0, A0.T, rtol=0, atol=1e-13 * sc)
    Dm, _ = oracle.dsa_dense(p, dsa_op=oracle.DSA_MNIP)
    P = Dm - Dn
    assert np.max(np.abs(P)) > 0
    assert np.allclose(P, P.T, rtol=0, atol=1e-13 * sc)


def test_n1_mnip_refuses_voids():
    """eq. ModifiedF0 divides by sigma_t: a void next to a thick cell is an error."""
    p = _mixed(2, 5, 1)
    assert np.any(p.sigma_t == 0.0)
    with pytest.raises(RuntimeError):
        oracle.dsa_dense(p, dsa_op=oracle.DSA_MNIP)


def test_n2_mnip_equals_nip_when_thick_enough():
    """The modified penalty's factor max(0.2 / (sigma_t h), 1) is 1 wherever
    sigma_t h >= 0.2, so there mNIP is NIP exactly; with thin cells next to
    thick ones the two differ on those faces only."""
    p = _mixed(2, 5, 1)
    keep = p.sigma_t.copy()
    p.sigma_t[:] = np.maximum(keep, 0.3)
    p.sigma_s[:] = np.minimum(p.sigma_s, p.sigma_t)
    Dn, _ = oracle.dsa_dense(p, dsa_op=oracle.DSA_NIP)
    Dm, _ = oracle.dsa_dense(p, dsa_op=oracle.DSA_MNIP)
    assert np.array_equal(Dn, Dm)
    p.sigma_t[:] = keep
    p.sigma_t[p.sigma_t == 0.0] = 0.05                 # no voids (eq. ModifiedF0 needs sigma_t > 0)
    Dn, _ = oracle.dsa_dense(p, dsa_op=oracle.DSA_NIP)
    Dm, _ = oracle.dsa_dense(p, dsa_op=oracle.DSA_MNIP)
    assert not np.array_equal(Dn, Dm)


@pytest.mark.parametrize("op", [oracle.DSA_NIP, oracle.DSA_MNIP])
def test_n3_gmres_correction_vs_dense(op):
    """The DSA correction with a nonsymmetric form (band LU solve) against a
    dense solve of the same assembled operator, both mass kinds."""
    p = _mixed(2, 6, 3)
    p.sigma_t[p.sigma_t == 0.0] = 0.05
    rng = np.random.default_rng(4)
    phi_old = rng.uniform(0, 1, (p.ncells, p.nn))
    phi_si = rng.uniform(0, 1, (p.ncells, p.nn))
    D, cells = oracle.dsa_dense(p, dsa_op=op)
    M = oracle.cell_mass(p.dim, p.h)
    for mass_kind in (0, 1):
        out, it, rr = oracle.dsa_correct(p, phi_old, phi_si, mass_kind=mass_kind, dsa_op=op, cg_rtol=1e-14)
        coef = p.sigma_t if mass_kind == 1 else p.sigma_s
        b = np.concatenate([coef[c] * (M @ (phi_si[c] - phi_old[c])) for c in cells])
        x = np.linalg.solve(D, b)
        ref = phi_si.copy()
        for s, c in enumerate(cells):
            ref[c] += x[s * p.nn:(s + 1) * p.nn]
        assert rr <= 1e-13 and it == 0
        assert np.max(np.abs(out - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_n4_nonsymmetric_dsa_keeps_fixed_point():
    """SI accelerated by het-NIP and het-mNIP DSA reaches the fixed point of
    unaccelerated SI (eq. DSA_fp: the DSA changes only the path), on C1 with
    its void block replaced by a thin cell so that mNIP is defined."""
    p = sninputs.config("c1")
    st = p.sigma_t.copy()
    st[st == 0.0] = 0.05
    ref = oracle.source_iterate(p, tol=1e-13, max_it=200000, use_dsa=False, sigma_t=st)
    assert ref["rc"] == 0
    for op in (oracle.DSA_NIP, oracle.DSA_MNIP):
        r = oracle.source_iterate(p, tol=1e-13, max_it=3000, use_dsa=True, dsa_op=op, cg_rtol=1e-13, sigma_t=st)
        assert r["rc"] == 0 and r["iters"] < ref["iters"] / 20
        assert np.linalg.norm(r["phi"] - ref["phi"]) <= 1e-10 * np.linalg.norm(ref["phi"])
