"""Pins of the oracle's triangular heterogeneous DSA (Alg. 1, Sec. 2.3) and of
its Krylov solve of the scalar-flux Schur system (Sec. 2.2, eq. schur).

Everything is checked against dense matrices assembled independently of the
oracle by brute-force quadrature (tests/bruteforce.py):

T1  one Alg. 1 step equals phi + D_T^{-1} (phi_SI - phi), with D_T^{-1} built
    from the paper's block form (eq. approxS): the Schur complement
    S_ff = L_ff - L_fs L_ss^{-1} L_sf of every L_d, the off-diagonal block
    X = sum_d w_d L_ss^{-1} L_sf S_ff^{-1} Sigma_s,f and the thick-region
    diffusion inverse.  The oracle instead applies it as Alg. 1 states: a
    zero-source transport update accumulated into the thin DOFs only.  The two
    agree only if that rewriting (the identity below eq. approxS) holds and the
    code follows it.
T2  Alg. 1 does not move the fixed point (eq. DSA_fp): converged Alg. 1,
    Alg. 2 and plain SI agree with the dense block system.
T3  special cases: eta = infinity gives plain SI bitwise; with every cell
    thick there is no thin DOF and Alg. 1 gives Alg. 2 bitwise.
G1  GMRES with a restart at least the system size solves S phi = b exactly
    (finite termination) and matches the dense solve.
G2  minimal residual: after k iterations the residual equals
    min ||r0 - S M^{-1} y|| over the Krylov space K_k(S M^{-1}, r0), computed
    by dense least squares, for M^{-1} = I, Alg. 2 and Alg. 1.
G3  restarted GMRES and source iteration reach the same fixed point.
"""
import math

import numpy as np
import pytest

import bruteforce as bf
import oracle
import sninputs
from sninputs import Problem


def _mixed(dim, shape, seed, order=4):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    nc = nx * ny * nz
    kind = rng.integers(0, 3, nc)           # 0 void, 1 thin, 2 thick
    kind[:3] = [0, 1, 2][:min(3, nc)]
    st = np.where(kind == 2, rng.uniform(5, 40, nc), np.where(kind == 1, rng.uniform(0.5, 2, nc), 0.0))
    ss = np.where(kind == 2, st * rng.uniform(0.9, 0.99, nc), np.where(kind == 1, st * rng.uniform(0.3, 0.9, nc),
                                                                       0.0))
    q = np.where(kind == 1, rng.uniform(0.2, 1.0, nc), 0.0)
    om, w = sninputs.level_symmetric(order, dim)
    h = (1.0, 0.8, 1.2) if dim == 3 else (1.0, 0.8, 1.0)
    return Problem("mix", dim, nx, ny, nz, h, st, ss, q, om, w)


_CACHE = {}


def _assembled(p):
    """The brute-force pieces that do not depend on the mass kind (cached per
    problem: the quadrature assembly is slow)."""
    key = (p.dim, p.nx, p.ny, p.nz, p.sigma_t.tobytes(), p.sigma_s.tobytes(), p.q.tobytes())
    if key not in _CACHE:
        Ss = bf.mass_matrix(p, p.sigma_s / (4 * math.pi))
        qd = bf.cell_load(p, p.q / (4 * math.pi))
        Ls = [bf.transport_matrix(p, d) for d in range(p.ndirs)]
        K = sum(p.w[d] * np.linalg.solve(Ls[d], Ss) for d in range(p.ndirs))
        b = sum(p.w[d] * np.linalg.solve(Ls[d], qd) for d in range(p.ndirs))
        Dff, cells = bf.sip_matrix(p, p.eta)
        _CACHE[key] = (Ss, Ls, K, b, Dff, cells)
    return _CACHE[key]


def _dense(p, mass_kind=0):
    """K = sum_d w_d L_d^{-1} Sigma_s, b, the L_d, the thick DOFs and the
    dense Alg. 2 preconditioner I + P D_ff^{-1} Sigma_f R."""
    N = p.ncells * p.nn
    Ss, Ls, K, b, Dff, cells = _assembled(p)
    F = np.array([c * p.nn + n for c in cells for n in range(p.nn)], dtype=np.int64)
    coef = p.sigma_t if mass_kind == 1 else p.sigma_s
    Sf = bf.mass_matrix(p, coef)[np.ix_(F, F)]
    P = np.zeros((N, F.size))
    P[F, np.arange(F.size)] = 1.0
    Mdiag = np.eye(N) + P @ np.linalg.solve(Dff, Sf) @ P.T
    return K, b, Ls, F, Ss, Dff, Sf, Mdiag


def _triangular_dense(p, Ls, F, Ss, Dff, Sf):
    """D_T^{-1} of eq. approxS from the block Schur complements."""
    N = p.ncells * p.nn
    S = np.setdiff1d(np.arange(N), F)
    X = np.zeros((S.size, F.size))
    Ssf = Ss[np.ix_(F, F)]
    for d in range(p.ndirs):
        L = Ls[d]
        Lss, Lsf, Lfs, Lff = L[np.ix_(S, S)], L[np.ix_(S, F)], L[np.ix_(F, S)], L[np.ix_(F, F)]
        Sff = Lff - Lfs @ np.linalg.solve(Lss, Lsf)
        X += p.w[d] * np.linalg.solve(Lss, Lsf @ np.linalg.solve(Sff, Ssf))
    upper = np.eye(N)
    upper[np.ix_(S, F)] = -X
    diag = np.eye(N)
    diag[np.ix_(F, F)] += np.linalg.solve(Dff, Sf)
    return upper @ diag


@pytest.mark.parametrize("dim,shape,seed", [(2, (4, 3, 1), 1), (2, (3, 3, 1), 2), (3, (2, 2, 1), 3)])
@pytest.mark.parametrize("mass_kind", [0, 1])
def test_t1_triangular_step_vs_block_form(dim, shape, seed, mass_kind):
    p = _mixed(dim, shape, seed)
    K, b, Ls, F, Ss, Dff, Sf, _ = _dense(p, mass_kind)
    assert 0 < F.size < p.ncells * p.nn
    DT = _triangular_dense(p, Ls, F, Ss, Dff, Sf)
    phi0 = np.random.default_rng(seed + 7).uniform(0.0, 1.0, p.ncells * p.nn)
    ref = phi0 + DT @ (K @ phi0 + b - phi0)
    got = oracle.source_iterate(p, tol=0.0, max_it=1, use_dsa=True, mass_kind=mass_kind, cg_rtol=1e-15,
                                phi0=phi0, dsa_form=1)["phi"].ravel()
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))
    # and it is not the diagonal form: the thin correction is non-zero
    diag = oracle.source_iterate(p, tol=0.0, max_it=1, use_dsa=True, mass_kind=mass_kind, cg_rtol=1e-15,
                                 phi0=phi0, dsa_form=0)["phi"].ravel()
    assert np.max(np.abs(got - diag)) > 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("dim,shape,seed", [(2, (3, 3, 1), 4), (3, (2, 2, 2), 5)])
def test_t2_fixed_point(dim, shape, seed):
    p = _mixed(dim, shape, seed)
    A, rhs = bf.block_system(p)
    N = p.ncells * p.nn
    ref = np.linalg.solve(A, rhs)[p.ndirs * N:]
    for form in (0, 1):
        r = oracle.source_iterate(p, tol=1e-15, max_it=5000, use_dsa=True, dsa_form=form)
        err = np.linalg.norm(r["phi"].ravel() - ref) / np.linalg.norm(ref)
        assert err <= 1e-12, (form, err)


def test_t3_special_cases():
    p = sninputs.config("c1")
    a = oracle.source_iterate(p, tol=1e-8, max_it=25, use_dsa=True, eta=math.inf, dsa_form=1)
    b = oracle.source_iterate(p, tol=1e-8, max_it=25, use_dsa=False)
    assert np.array_equal(a["phi"], b["phi"])
    om, w = sninputs.level_symmetric(4, 2)
    n = 6
    rng = np.random.default_rng(9)
    st = rng.uniform(20, 60, n * n)
    ss = st * rng.uniform(0.95, 0.99, n * n)
    q = rng.uniform(0, 1, n * n)
    p2 = Problem("allthick", 2, n, n, 1, (1.0, 1.0, 1.0), st, ss, q, om, w, eta=1.0)
    assert np.all(p2.sigma_s >= p2.eta)
    a = oracle.source_iterate(p2, tol=0.0, max_it=6, use_dsa=True, dsa_form=1)
    b = oracle.source_iterate(p2, tol=0.0, max_it=6, use_dsa=True, dsa_form=0)
    assert np.array_equal(a["phi"], b["phi"])


@pytest.mark.parametrize("dim,shape,seed,use_dsa", [(2, (3, 2, 1), 6, False), (2, (3, 2, 1), 6, True),
                                                    (3, (3, 1, 1), 7, True)])
def test_g1_finite_termination(dim, shape, seed, use_dsa):
    p = _mixed(dim, shape, seed)
    K, b, *_ = _dense(p)
    N = p.ncells * p.nn
    ref = np.linalg.solve(np.eye(N) - K, b)
    r = oracle.gmres(p, tol=1e-14, max_it=N + 2, restart=N + 2, use_dsa=use_dsa, cg_rtol=1e-15)
    assert r["rc"] == 0 and r["iters"] <= N
    err = np.linalg.norm(r["phi"].ravel() - ref) / np.linalg.norm(ref)
    assert err <= 1e-11, err


@pytest.mark.parametrize("precond", ["none", "alg2", "alg1"])
def test_g2_minimal_residual(precond):
    p = _mixed(2, (4, 3, 1), 8)
    K, b, Ls, F, Ss, Dff, Sf, Mdiag = _dense(p)
    N = p.ncells * p.nn
    S = np.eye(N) - K
    Minv = {"none": np.eye(N), "alg2": Mdiag, "alg1": _triangular_dense(p, Ls, F, Ss, Dff, Sf)}[precond]
    A = S @ Minv
    k = 5
    r = oracle.gmres(p, tol=0.0, max_it=k, restart=30, use_dsa=precond != "none", dsa_form=int(precond == "alg1"),
                     cg_rtol=1e-15)
    assert r["iters"] == k
    bn = np.linalg.norm(b)
    for j in range(1, k + 1):
        kry = np.empty((N, j))
        v = b / bn
        for i in range(j):
            kry[:, i] = v
            v = A @ v
            v /= np.linalg.norm(v)
        Q, _ = np.linalg.qr(kry)
        c, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
        res = np.linalg.norm(b - A @ Q @ c) / bn
        assert abs(r["res_hist"][j - 1] - res) <= 1e-8 * res, (j, r["res_hist"][j - 1], res)
    # the history of a minimal-residual method does not increase
    assert np.all(np.diff(r["res_hist"]) <= 1e-14)


def test_g3_restarted_gmres_same_fixed_point():
    p = _mixed(2, (12, 10, 1), 10)
    si = oracle.source_iterate(p, tol=1e-13, max_it=3000, use_dsa=True)
    assert si["rc"] == 0
    for restart, form in ((30, 0), (4, 0), (30, 1)):
        g = oracle.gmres(p, tol=1e-13, max_it=3000, restart=restart, use_dsa=True, dsa_form=form)
        assert g["rc"] == 0
        err = np.linalg.norm(g["phi"] - si["phi"]) / np.linalg.norm(si["phi"])
        assert err <= 1e-10, (restart, form, err)
