"""Pins of the oracle's scalar-flux moment (eq. phi: phi = sum_d w_d psi_d)
in the [cell][direction][node] layout of psi.

P6a closed form: an isotropic psi = 1 gives phi = 4 pi (the weights sum to
    4 pi) at every node of every cell.
P6b quadrature moments: psi[c, d, n] = f[c, n] (1 + 2 mu_d + 3 eta_d + 3 mu_d^2)
    gives phi = 8 pi f, because the odd moments of a level-symmetric set
    vanish and its second moment is 4 pi / 3.  A wrong stride (direction-major
    indexing, a transposed cell/node index) mixes the values of f across cells
    or nodes, and a dropped or misplaced weight breaks the moments, so each
    fails this check.
P6c consistency with the source iteration: the moment of a sweep equals the
    unaccelerated source-iteration update from the same flux (eq. psi and
    eq. phi), which the oracle forms by a separate accumulation that is
    itself pinned against the dense block system (P8).
"""
import math

import numpy as np
import pytest

import oracle
import sninputs
from sninputs import Problem


def _problem(dim, shape, order, seed=0):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    nc = nx * ny * nz
    om, w = sninputs.level_symmetric(order, dim)
    st = rng.uniform(0.5, 4.0, nc)
    ss = st * rng.uniform(0.0, 0.9, nc)
    q = rng.uniform(0.0, 1.0, nc)
    h = (1.0, 0.8, 1.3) if dim == 3 else (1.0, 0.8, 1.0)
    return Problem("moment", dim, nx, ny, nz, h, st, ss, q, om, w)


CASES = [(2, (5, 3, 1), 4), (2, (7, 4, 1), 8), (3, (3, 4, 2), 4), (3, (2, 3, 4), 8), (3, (3, 2, 2), 12)]


@pytest.mark.parametrize("dim,shape,order", CASES)
def test_p6a_isotropic_flux(dim, shape, order):
    p = _problem(dim, shape, order)
    psi = np.ones((p.ncells, p.ndirs, p.nn))
    phi = oracle.moment(p, psi)
    assert phi.shape == (p.ncells, p.nn)
    assert np.max(np.abs(phi - 4 * math.pi)) <= 1e-14 * 4 * math.pi


@pytest.mark.parametrize("dim,shape,order", CASES)
def test_p6b_direction_moments_and_layout(dim, shape, order):
    p = _problem(dim, shape, order, seed=1)
    rng = np.random.default_rng(2)
    f = rng.uniform(-1.0, 2.0, (p.ncells, p.nn))
    mu, eta = p.omega[:, 0], p.omega[:, 1]
    g = 1.0 + 2.0 * mu + 3.0 * eta + 3.0 * mu * mu
    psi = f[:, None, :] * g[None, :, None]
    phi = oracle.moment(p, psi)
    ref = 8.0 * math.pi * f
    assert np.max(np.abs(phi - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_p6b_detects_direction_major_layout():
    """The layout check above is not vacuous: reading the same numbers in
    direction-major order (psi[d][c][n]) gives a different flux."""
    p = _problem(3, (3, 2, 2), 8, seed=3)
    rng = np.random.default_rng(4)
    f = rng.uniform(-1.0, 2.0, (p.ncells, p.nn))
    g = 1.0 + 2.0 * p.omega[:, 0] + 3.0 * p.omega[:, 1] + 3.0 * p.omega[:, 0] ** 2
    psi = f[:, None, :] * g[None, :, None]
    wrong = np.ascontiguousarray(np.transpose(psi, (1, 0, 2))).reshape(p.ncells, p.ndirs, p.nn)
    assert np.max(np.abs(oracle.moment(p, wrong) - 8 * math.pi * f)) > 1e-3


@pytest.mark.parametrize("dim,shape,order", [(2, (6, 5, 1), 4), (3, (4, 3, 3), 4), (3, (3, 3, 2), 12)])
def test_p6c_moment_of_sweep_is_si_update(dim, shape, order):
    p = _problem(dim, shape, order, seed=5)
    phi0 = np.random.default_rng(6).uniform(0.0, 1.0, (p.ncells, p.nn))
    psi = oracle.sweep(p, phi0, p.q)
    via_moment = oracle.moment(p, psi)
    r = oracle.source_iterate(p, tol=0.0, max_it=1, use_dsa=False, phi0=phi0)
    assert r["iters"] == 1
    assert np.max(np.abs(via_moment - r["phi"])) <= 1e-13 * np.max(np.abs(r["phi"]))
