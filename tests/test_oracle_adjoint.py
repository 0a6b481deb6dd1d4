"""Pins of the oracle's adjoint (derived from the block system, eq. system).

For J = g^T phi with A x = b the discrete adjoint gives
  chi = sum_d w_d L_d^{-T}(g + Sigma_s chi),  psi~_d = L_d^{-T}(g + Sigma_s chi),
  dJ/dlog sigma_t,K = -sigma_t,K sum_d w_d psi~_d,K^T M_K psi_d,K,
  dJ/dlog sigma_s,K =  sigma_s,K chi_K^T M_K phi_K / 4pi.
P16 reciprocity: g^T phi[q] = (M q / 4pi)^T chi[g].
P17 brute force: gradients against central differences of dense solves.
"""
import math

import numpy as np
import pytest

import bruteforce as bf
import oracle
import sninputs
from sninputs import Problem


def _prob(dim, n, seed):
    rng = np.random.default_rng(seed)
    nc = n ** dim
    st = rng.uniform(0.5, 20.0, nc)
    ss = st * rng.uniform(0.1, 0.99, nc)
    q = rng.uniform(0.0, 1.0, nc)
    om, w = sninputs.level_symmetric(4, dim)
    nz = n if dim == 3 else 1
    return Problem("adj", dim, n, n, nz, (1.0, 0.9, 1.1), st, ss, q, om, w, eta=5.0)


def _adjoint(p, qadj, inflow=None):
    fwd = oracle.source_iterate(p, tol=1e-15, max_it=5000, use_dsa=True)
    adj = oracle.source_iterate(p, tol=1e-15, max_it=5000, use_dsa=True, transpose=True, q=qadj,
                                inflow=inflow)
    phi, chi = fwd["phi"], adj["phi"]
    psi = oracle.sweep(p, phi, p.q)
    psia = oracle.sweep(p, chi, qadj, inflow=inflow, transpose=True)
    gt, gs = oracle.gradient(p, psi, psia, phi, chi)
    return phi, chi, gt, gs


def test_p16_reciprocity_volume():
    p = _prob(2, 8, 1)
    qadj = sninputs.patch_source(p, (5, 5), (8, 8))
    phi, chi, _, _ = _adjoint(p, qadj)
    M = bf.mass_matrix(p, np.ones(p.ncells))
    J = (M @ (qadj / (4 * math.pi)).repeat(p.nn)) @ phi.ravel()     # g = M q_adj / 4pi
    Jr = (M @ (p.q / (4 * math.pi)).repeat(p.nn)) @ chi.ravel()
    assert abs(J - Jr) <= 1e-13 * abs(J)


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_p17_gradient_vs_dense_fd(dim, n):
    p = _prob(dim, n, 4 + dim)
    qadj = np.zeros(p.ncells)
    qadj[-1] = 4 * math.pi
    _, _, gt, gs = _adjoint(p, qadj)
    M1 = bf.mass_matrix(p, np.ones(p.ncells))
    g = M1 @ (qadj / (4 * math.pi)).repeat(p.nn)
    N = p.ncells * p.nn

    def J(st, ss):
        A, rhs = bf.block_system(p, sigma_t=st, sigma_s=ss)
        x = np.linalg.solve(A, rhs)
        return g @ x[p.ndirs * N:]

    eps = 1e-5
    for c in range(p.ncells):
        for which, grad in ((0, gt), (1, gs)):
            st, ss = p.sigma_t.copy(), p.sigma_s.copy()
            arr = st if which == 0 else ss
            base = arr[c]
            arr[c] = base * math.exp(eps)
            jp = J(st, ss)
            arr[c] = base * math.exp(-eps)
            jm = J(st, ss)
            fd = (jp - jm) / (2 * eps)
            assert abs(fd - grad[c]) <= 1e-7 * max(abs(fd), 1e-3 * np.max(np.abs(grad))), (c, which, fd, grad[c])


def test_p16_reciprocity_outflow():
    """Outflow partial current through x = L: adjoint source = unit boundary
    data on x = L for the directions with mu > 0 (transposed sweep)."""
    p = _prob(2, 6, 8)
    inflow_adj = sninputs.unit_inflow_on_face(
        Problem(p.name, p.dim, p.nx, p.ny, p.nz, p.h, p.sigma_t, p.sigma_s, p.q, -p.omega, p.w),
        axis=0, high=True, directions_sign=-1)
    fwd = oracle.source_iterate(p, tol=1e-15, max_it=5000, use_dsa=True)
    adj = oracle.source_iterate(p, tol=1e-15, max_it=5000, use_dsa=True, transpose=True,
                                q=np.zeros(p.ncells), inflow=inflow_adj)
    psi = oracle.sweep(p, fwd["phi"], p.q)
    # J = sum_{mu>0} w mu int_{x=L} psi
    J = 0.0
    for d in range(p.ndirs):
        mu = p.omega[d, 0]
        if mu <= 0:
            continue
        for j in range(p.ny):
            c = j * p.nx + p.nx - 1
            ijk = (p.nx - 1, j, 0)
            for x, wq in bf._face_points(p, ijk, 0, 1):
                val = sum(psi[c, d, m] * bf._basis(p, ijk, m, x)[0] for m in range(p.nn))
                J += p.w[d] * mu * wq * val
    M = bf.mass_matrix(p, np.ones(p.ncells))
    Jr = (M @ (p.q / (4 * math.pi)).repeat(p.nn)) @ adj["phi"].ravel()
    assert abs(J - Jr) <= 1e-12 * abs(J)
