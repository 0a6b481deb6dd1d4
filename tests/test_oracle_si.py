"""Pins of the oracle's source iteration and heterogeneous DSA.

P7  closed form: infinite-medium limit phi = q / sigma_a.
P8  brute force: converged phi against the dense block system (eq. system).
P9  symmetry: mirror- and diagonal-symmetric problems give symmetric phi.
P10 textbook: unaccelerated SI contracts at most at rate c = sigma_s/sigma_t.
P11 invariant: DSA changes the path, not the fixed point (eq. DSA_fp).
P12 special cases: eta = inf reproduces plain SI bitwise; eta below every
    sigma_s on a void-free problem makes every cell thick (full DSA).
"""
import math

import numpy as np
import pytest

import bruteforce as bf
import oracle
import sninputs
from sninputs import Problem


def _prob(dim, nx, st, ss, q, order=4, h=(1.0, 1.0, 1.0), eta=1.0):
    om, w = sninputs.level_symmetric(order, dim)
    ny = nx
    nz = nx if dim == 3 else 1
    nc = nx * ny * nz
    f = lambda v: np.full(nc, v, dtype=np.float64) if np.isscalar(v) else np.asarray(v, dtype=np.float64)
    return Problem("t", dim, nx, ny, nz, h, f(st), f(ss), f(q), om, w, eta=eta)


def test_p7_infinite_medium():
    p = _prob(2, 64, 1.0, 0.5, 1.0)
    r = oracle.source_iterate(p, tol=1e-14, max_it=200, use_dsa=False)
    assert r["rc"] == 0
    phi = r["phi"].reshape(64, 64, 4)
    centre = phi[28:36, 28:36, :]
    assert np.max(np.abs(centre - 2.0)) <= 1e-12 * 2.0


@pytest.mark.parametrize("dim,n,dsa", [(2, 3, False), (2, 3, True), (3, 2, True)])
def test_p8_fixed_point_vs_block_system(dim, n, dsa):
    rng = np.random.default_rng(3 + n)
    nc = n ** dim
    st = rng.uniform(0.5, 30.0, nc)
    ss = st * rng.uniform(0.0, 0.99, nc)
    st[0], ss[0] = 0.0, 0.0          # one void cell
    q = rng.uniform(0.0, 1.0, nc)
    p = _prob(dim, n, st, ss, q)
    A, rhs = bf.block_system(p)
    x = np.linalg.solve(A, rhs)
    N = p.ncells * p.nn
    phi_ref = x[p.ndirs * N:]
    r = oracle.source_iterate(p, tol=1e-15, max_it=5000, use_dsa=dsa)
    err = np.linalg.norm(r["phi"].ravel() - phi_ref) / np.linalg.norm(phi_ref)
    assert err <= 1e-12, err


def test_p9_symmetry():
    n = 16
    st = np.ones(n * n)
    ss = np.full(n * n, 0.9)
    q = np.zeros(n * n)
    for j in range(n):
        for i in range(n):
            c = j * n + i
            if 5 <= i <= 10 and 5 <= j <= 10:
                st[c], ss[c] = 100.0, 99.9
            if (i in (0, 15)) and (j in (0, 15)):
                st[c], ss[c] = 0.0, 0.0
            if 7 <= i <= 8 and 7 <= j <= 8:
                q[c] = 1.0
    p = _prob(2, n, st, ss, q)
    r = oracle.source_iterate(p, tol=1e-14, max_it=2000, use_dsa=True)
    phi = r["phi"].reshape(n, n, 2, 2)        # [j, i, b, a]
    mirror_x = phi[:, ::-1, :, ::-1]
    diag = np.transpose(phi, (1, 0, 3, 2))
    scale = np.max(np.abs(phi))
    assert np.max(np.abs(phi - mirror_x)) <= 1e-12 * scale
    assert np.max(np.abs(phi - diag)) <= 1e-12 * scale


def test_p10_si_rate_bounded_by_c():
    c = 0.9
    p = _prob(2, 32, 10.0, 10.0 * c, 1.0)
    r = oracle.source_iterate(p, tol=1e-300, max_it=40, use_dsa=False)
    res = r["res_hist"]
    ratios = res[10:] / res[9:-1]
    assert np.all(ratios <= c + 1e-12)
    assert ratios[-1] > 0.8 * c      # thick, large domain: close to c


def test_p11_dsa_does_not_move_fixed_point():
    """C1 (S4, 16x16, thick block + void): accelerated and unaccelerated converge
    to the same phi (eq. DSA_fp)."""
    p = sninputs.config("c1")
    a = oracle.source_iterate(p, tol=1e-14, max_it=2000, use_dsa=True)
    b = oracle.source_iterate(p, tol=1e-14, max_it=60000, use_dsa=False)
    assert a["rc"] == 0 and b["rc"] == 0
    err = np.linalg.norm(a["phi"] - b["phi"]) / np.linalg.norm(b["phi"])
    # the unaccelerated error is about res / (1 - rho) with rho ~ 0.999
    assert err <= 2e-10, err
    assert a["iters"] < b["iters"] / 50


def test_p11_mass_kind_same_fixed_point():
    p = sninputs.config("c1")
    a = oracle.source_iterate(p, tol=1e-13, max_it=2000, use_dsa=True, mass_kind=0)
    b = oracle.source_iterate(p, tol=1e-13, max_it=2000, use_dsa=True, mass_kind=1)
    err = np.linalg.norm(a["phi"] - b["phi"]) / np.linalg.norm(b["phi"])
    assert err <= 1e-11


def test_p12_eta_infinite_is_plain_si():
    p = sninputs.config("c1")
    a = oracle.source_iterate(p, tol=1e-8, max_it=30, use_dsa=True, eta=math.inf)
    b = oracle.source_iterate(p, tol=1e-8, max_it=30, use_dsa=False)
    assert np.array_equal(a["phi"], b["phi"])
    assert np.array_equal(a["res_hist"], b["res_hist"])


def test_p12_all_thick_is_full_dsa():
    n = 6
    p = _prob(2, n, 50.0, 49.5, 1.0)
    D, cells = oracle.dsa_dense(p, eta=0.0)
    assert len(cells) == p.ncells
    # full-domain operator: D 1 = sigma_a M 1 on interior cells, plus
    # kappa_0 * face mass on domain faces
    ones = np.ones(p.ncells * p.nn)
    Ma = bf.mass_matrix(p, p.sigma_t - p.sigma_s)
    k0 = [np.sum(p.w * np.abs(p.omega[:, ax])) / (8 * math.pi) for ax in range(2)]
    ref = Ma @ ones
    for c, ijk in bf._cells(p):
        for ax in range(2):
            for side in (0, 1):
                if bf._neighbour(p, ijk, ax, 1 if side else -1) is None:
                    for x, wq in bf._face_points(p, ijk, ax, side):
                        for m in range(p.nn):
                            ref[c * p.nn + m] += wq * k0[ax] * bf._basis(p, ijk, m, x)[0]
    assert np.allclose(D @ ones, ref, rtol=1e-12, atol=1e-14)
    # and the accelerated solve converges far faster than plain SI
    a = oracle.source_iterate(p, tol=1e-10, max_it=3000, use_dsa=True, eta=0.0)
    b = oracle.source_iterate(p, tol=1e-10, max_it=3000, use_dsa=False)
    assert a["iters"] * 5 < b["iters"]
