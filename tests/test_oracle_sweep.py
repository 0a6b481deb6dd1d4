"""Pins of the oracle's transport sweep (Section 2.2, eq. psi; Section 3.1, eq. Tmat1).

P1 brute force: dense L_d^{-1} (and L_d^{-T}) from the quadrature-assembled weak form.
P2 closed form: pure absorber, outflow factor of the upwind Q1 scheme per cell.
P3 textbook convergence: O(h^3) outflow error for the pure absorber.
P4 exact invariant: per-direction particle balance.
P5 exact identity: A(Omega)^T = A(-Omega), <L^{-1} a, b> = <a, L^{-T} b>.
"""
import math

import numpy as np
import pytest

import bruteforce as bf
import oracle
import sninputs
from sninputs import Problem


def _tiny(dim, n, order=4, seed=0, void=False, hs=(1.0, 0.7, 1.3)):
    rng = np.random.default_rng(seed)
    nz = n if dim == 3 else 1
    nc = n * n * nz
    om, w = sninputs.level_symmetric(order, dim)
    st = rng.uniform(0.3, 5.0, nc)
    if void:
        st[rng.integers(0, nc)] = 0.0
    ss = st * rng.uniform(0.0, 0.95, nc)
    q = rng.uniform(0.0, 2.0, nc)
    h = hs if dim == 3 else (hs[0], hs[1], 1.0)
    return Problem("tiny", dim, n, n, nz, h, st, ss, q, om, w)


def _rand_inflow(p, seed):
    nbf = sninputs.inflow_size(p.dim, p.nx, p.ny, p.nz)
    return np.random.default_rng(seed).uniform(0, 1, (p.ndirs, nbf))


@pytest.mark.parametrize("dim,n", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
@pytest.mark.parametrize("transpose", [False, True])
def test_p1_sweep_vs_dense(dim, n, transpose):
    p = _tiny(dim, n, seed=n + 10 * dim, void=(n == 3))
    rng = np.random.default_rng(7)
    phi = rng.uniform(-1, 1, (p.ncells, p.nn))
    inflow = _rand_inflow(p, 3)
    psi = oracle.sweep(p, phi, p.q, inflow=inflow, transpose=transpose)
    Ss = bf.mass_matrix(p, p.sigma_s / (4 * math.pi))
    vol = Ss @ phi.ravel() + bf.cell_load(p, p.q / (4 * math.pi))
    for d in range(p.ndirs):
        L = bf.transport_matrix(p, d)
        if not transpose:
            ref = np.linalg.solve(L, vol + bf.inflow_load(p, d, inflow))
        else:
            # boundary data of the transposed sweep enters through the faces
            # with Omega.n > 0, in the layout of the reversed direction
            # (L_d^T = L_{-d}): its load is the inflow load of -Omega_d.
            pr = Problem(p.name, p.dim, p.nx, p.ny, p.nz, p.h, p.sigma_t, p.sigma_s, p.q,
                         -p.omega, p.w)
            ref = np.linalg.solve(L.T, vol + bf.inflow_load(pr, d, inflow))
        got = psi[:, d, :].ravel()
        assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def _absorber_profile(tau, ncell):
    R = (1 - tau / 3) / (1 + 2 * tau / 3 + tau * tau / 6)
    P = (1 + 2 * tau / 3) / (1 + 2 * tau / 3 + tau * tau / 6)
    # node 0 (inflow end) and node 1 (outflow end) of cell i
    return np.array([[R ** i * P, R ** (i + 1)] for i in range(ncell)]), R


@pytest.mark.parametrize("sig,h", [(0.5, 1.0), (2.0, 1.0), (10.0, 0.5), (1e3, 1.0)])
def test_p2_pure_absorber_closed_form(sig, h):
    """psi_inc = 1 on x = 0; y inflow carries the 1D profile, so psi is
    y-independent and every row equals the 1D upwind-Q1 solution:
    outflow of cell i = R(tau)^(i+1), R = (1 - tau/3)/(1 + 2tau/3 + tau^2/6)
    (the [1/2] Pade approximant of exp(-tau)), tau = sigma h / |mu|."""
    nx, ny = 12, 3
    om, w = sninputs.level_symmetric(4, 2)
    p = Problem("abs", 2, nx, ny, 1, (h, 0.8, 1.0), np.full(nx * ny, sig), np.zeros(nx * ny),
                np.zeros(nx * ny), om, w)
    nbf = sninputs.inflow_size(2, nx, ny, 1)
    inflow = np.zeros((p.ndirs, nbf))
    prof = {}
    for d in range(p.ndirs):
        mu, eta_ = om[d, 0], om[d, 1]
        if mu <= 0:
            continue
        tau = sig * h / mu
        pr, R = _absorber_profile(tau, nx)
        prof[d] = pr
        inflow[d, :2 * ny] = 1.0                      # x = 0 face, both nodes of each cell
        inflow[d, 2 * ny:] = pr.ravel()                # y inflow face: (i*2 + a)
    psi = oracle.sweep(p, None, None, inflow=inflow)
    for d, pr in prof.items():
        for j in range(ny):
            for i in range(nx):
                c = j * nx + i
                for b in range(2):
                    got = psi[c, d, 2 * b:2 * b + 2]
                    assert np.allclose(got, pr[i], rtol=1e-12, atol=1e-300)


def test_p2_pure_absorber_3d():
    nx, n = 6, 2
    om, w = sninputs.level_symmetric(4, 3)
    sig, h = 3.0, 0.6
    nc = nx * n * n
    p = Problem("abs3", 3, nx, n, n, (h, 1.0, 1.0), np.full(nc, sig), np.zeros(nc), np.zeros(nc), om, w)
    nbf = sninputs.inflow_size(3, nx, n, n)
    inflow = np.zeros((p.ndirs, nbf))
    offy, offz = n * n * 4, n * n * 4 + nx * n * 4
    prof = {}
    for d in range(p.ndirs):
        if om[d, 0] <= 0:
            continue
        pr, _ = _absorber_profile(sig * h / om[d, 0], nx)
        prof[d] = pr
        inflow[d, :offy] = 1.0
        for k in range(n):
            for i in range(nx):
                for c2 in range(2):
                    for a in range(2):
                        inflow[d, offy + (k * nx + i) * 4 + a + 2 * c2] = pr[i, a]
        for j in range(n):
            for i in range(nx):
                for b in range(2):
                    for a in range(2):
                        inflow[d, offz + (j * nx + i) * 4 + a + 2 * b] = pr[i, a]
    psi = oracle.sweep(p, None, None, inflow=inflow)
    for d, pr in prof.items():
        for c in range(nc):
            i = c % nx
            for node in range(8):
                assert abs(psi[c, d, node] - pr[i, node & 1]) <= 1e-12 * abs(pr[i, node & 1])


def test_p3_third_order_outflow():
    """Outflow error against exp(-sigma L / mu) falls as h^3."""
    om, w = sninputs.level_symmetric(4, 2)
    d = 0
    mu = om[d, 0]
    L, sig = 2.0, 1.5
    errs = []
    for nx in (16, 32, 64, 128):
        h = L / nx
        p = Problem("cv", 2, nx, 1, 1, (h, 1.0, 1.0), np.full(nx, sig), np.zeros(nx), np.zeros(nx), om, w)
        pr, _ = _absorber_profile(sig * h / mu, nx)
        inflow = np.zeros((p.ndirs, sninputs.inflow_size(2, nx, 1, 1)))
        inflow[d, :2] = 1.0
        inflow[d, 2:] = pr.ravel()
        psi = oracle.sweep(p, None, None, inflow=inflow)
        errs.append(abs(psi[nx - 1, d, 1] - math.exp(-sig * L / mu)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(2.85 < r < 3.15 for r in rates), rates


@pytest.mark.parametrize("dim", [2, 3])
def test_p4_particle_balance(dim):
    """sum_K int sigma_t psi + outflow - inflow = sum_K int s, per direction."""
    n = 5 if dim == 2 else 3
    p = _tiny(dim, n, order=4, seed=11, void=True)
    rng = np.random.default_rng(5)
    phi = rng.uniform(0, 1, (p.ncells, p.nn))
    inflow = _rand_inflow(p, 9)
    psi = oracle.sweep(p, phi, p.q, inflow=inflow)
    Mt = bf.mass_matrix(p, p.sigma_t)
    Ss = bf.mass_matrix(p, p.sigma_s / (4 * math.pi))
    src = Ss @ phi.ravel() + bf.cell_load(p, p.q / (4 * math.pi))
    ones = np.ones(p.ncells * p.nn)
    for d in range(p.ndirs):
        om = p.omega[d]
        absorb = ones @ (Mt @ psi[:, d, :].ravel())
        # boundary currents via the Q1 face traces (trapezoid-exact face mass)
        out, inc = 0.0, bf.inflow_load(p, d, inflow).sum()
        for c, ijk in bf._cells(p):
            for ax in range(dim):
                for side in (0, 1):
                    if bf._neighbour(p, ijk, ax, 1 if side else -1) is not None:
                        continue
                    on = om[ax] * (1 if side else -1)
                    if on <= 0:
                        continue
                    for x, wq in bf._face_points(p, ijk, ax, side):
                        val = sum(psi[c, d, m] * bf._basis(p, ijk, m, x)[0] for m in range(p.nn))
                        out += wq * on * val
        total = src.sum()
        assert abs(absorb + out - inc - total) <= 1e-12 * (abs(total) + inc + 1.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_p5_transpose_identities(dim):
    om, w = sninputs.level_symmetric(4, dim)
    h = (0.9, 1.1, 1.3)
    for d in range(len(w)):
        A = oracle.cell_matrix(dim, h, om[d], 2.5)
        Am = oracle.cell_matrix(dim, h, -om[d], 2.5)
        assert np.allclose(A.T, Am, atol=1e-15, rtol=0)
    p = _tiny(dim, 3 if dim == 2 else 2, seed=4)
    rng = np.random.default_rng(1)
    a = rng.standard_normal((p.ncells, p.nn))
    b = rng.standard_normal((p.ncells, p.nn))
    # sweep with a pure volume density field: use q = 0 and phi with sigma_s = 4pi
    pa = Problem(p.name, p.dim, p.nx, p.ny, p.nz, p.h, p.sigma_t, np.full(p.ncells, 4 * math.pi),
                 np.zeros(p.ncells), p.omega, p.w)
    fa = oracle.sweep(pa, a, None)           # L^{-1} M a
    gb = oracle.sweep(pa, b, None, transpose=True)   # L^{-T} M b
    M = bf.mass_matrix(p, np.ones(p.ncells))
    for d in range(p.ndirs):
        lhs = fa[:, d, :].ravel() @ (M @ b.ravel())
        rhs = (M @ a.ravel()) @ gb[:, d, :].ravel()
        assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1e-300) + 1e-15
