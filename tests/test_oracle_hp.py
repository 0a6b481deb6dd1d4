"""Pins of the order-p oracle (oracle/hp.py, 2D Q_p, p = 1..4).

H1 p = 1 is the Q1 oracle: sweeps and the SIP / NIP / mNIP diffusion matrices
   equal those of the independently pinned C oracle.
H2 polynomial reproduction: when the exact transport solution is a Q_p
   polynomial (its source Omega.grad psi + sigma_t psi is then in Q_p too,
   and the inflow is its trace), the sweep returns it exactly, for every
   direction sign pattern.
H3 p = 2, 3, 4 sweeps against the dense solve of a brute-force quadrature
   assembly (tests/bruteforce_hp.py) with boundary inflow.
H4 particle balance per direction: absorption + net outflow = source + inflow.
H5 the diffusion matrices (SIP, NIP, mNIP) against the brute-force pointwise
   assembly; interior rows annihilate constants up to sigma_a; SIP symmetric
   positive definite.
H6 source iteration reaches the fixed point of the dense block system
   (eq. system), with and without DSA (the DSA does not move it, eq. DSA_fp).
H7 the Gauss-Lobatto nodes (closed forms for p = 1..4) and the 1D matrices
   (closed forms for p = 1, 2; mass, derivative and integration-by-parts
   identities for p = 1..4).
"""
import math

import numpy as np
import pytest

import bruteforce_hp as bfh
import oracle
from oracle import hp
import sninputs
from sninputs import Problem


def _prob(nx, ny, order, seed=0, voids=False, h=(0.9, 1.2), sn=4):
    rng = np.random.default_rng(seed)
    nc = nx * ny
    kind = rng.integers(0 if voids else 1, 3, nc)
    st = np.where(kind == 2, rng.uniform(20, 200, nc), np.where(kind == 1, rng.uniform(0.3, 2, nc), 0.0))
    ss = np.where(kind == 2, st * rng.uniform(0.95, 0.999, nc), np.where(kind == 1, 0.5 * st, 0.0))
    q = rng.uniform(0, 1, nc)
    om, w = sninputs.level_symmetric(sn, 2)
    return Problem(f"hp{order}", 2, nx, ny, 1, (h[0], h[1], 1.0), st, ss, q, om, w, order=order)


def test_h7_nodes_and_reference_matrices():
    assert np.allclose(hp.gll_nodes(1), [0, 1])
    assert np.allclose(hp.gll_nodes(2), [0, 0.5, 1])
    assert np.allclose(hp.gll_nodes(3), [0, (1 - 1 / math.sqrt(5)) / 2, (1 + 1 / math.sqrt(5)) / 2, 1])
    # p = 4: the interior points of [-1, 1] are 0 and +-sqrt(3/7)
    assert np.allclose(hp.gll_nodes(4), [0, (1 - math.sqrt(3 / 7)) / 2, 0.5, (1 + math.sqrt(3 / 7)) / 2, 1])
    r1 = hp.Ref1D(1)
    assert np.allclose(r1.M, [[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    assert np.allclose(r1.D, [[-0.5, 0.5], [-0.5, 0.5]])
    assert np.allclose(r1.K, [[1, -1], [-1, 1]])
    r2 = hp.Ref1D(2)                      # quadratic Lagrange on 0, 1/2, 1 (Simpson-type masses)
    assert np.allclose(r2.M, np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30)
    assert np.allclose(r2.K, np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3)
    for p in (1, 2, 3, 4):
        r = hp.Ref1D(p)
        assert np.allclose(r.M.sum(), 1.0) and np.allclose(r.D.sum(axis=1), 0.0)
        assert np.allclose(r.D + r.D.T, np.outer(np.eye(p + 1)[-1], np.eye(p + 1)[-1]) -
                           np.outer(np.eye(p + 1)[0], np.eye(p + 1)[0]))   # integration by parts


def test_h1_order1_is_the_q1_oracle():
    p = _prob(5, 4, 1, seed=1, voids=True)
    rng = np.random.default_rng(2)
    phi = rng.uniform(0, 1, (p.ncells, 4))
    a = hp.sweep(p, phi, p.q)
    b = oracle.sweep(p, phi, p.q)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))
    p.sigma_t[p.sigma_t == 0.0] = 0.05
    for form, op in ((hp.SIP, oracle.DSA_SIP), (hp.NIP, oracle.DSA_NIP), (hp.MNIP, oracle.DSA_MNIP)):
        A, ca = hp.dsa_dense(p, form=form)
        B, cb = oracle.dsa_dense(p, dsa_op=op)
        assert np.array_equal(ca, cb)
        assert np.allclose(A, B, rtol=0, atol=1e-13 * np.max(np.abs(B))), form


def _poly_case(order, om_signs):
    """Exact solution psi(x, y) = P(x) Q(y), degree `order` in each variable."""
    nx, ny = 3, 2
    h = (0.7, 1.1)
    rng = np.random.default_rng(order)
    cx = rng.uniform(-1, 1, order + 1)
    cy = rng.uniform(-1, 1, order + 1)
    P = np.polynomial.Polynomial(cx)
    Q = np.polynomial.Polynomial(cy)
    om = np.array([[om_signs[0] * 0.6, om_signs[1] * 0.48, 0.64]])
    st = rng.uniform(0.5, 3.0, nx * ny)
    prob = Problem("poly", 2, nx, ny, 1, (h[0], h[1], 1.0), st, np.zeros(nx * ny), np.zeros(nx * ny), om,
                   np.array([4 * math.pi]), order=order)
    nodes = hp.gll_nodes(order)
    n = order + 1
    src = np.zeros((prob.ncells, n * n))
    exact = np.zeros((prob.ncells, n * n))
    for j in range(ny):
        for i in range(nx):
            c = j * nx + i
            for b in range(n):
                for a in range(n):
                    x, y = (i + nodes[a]) * h[0], (j + nodes[b]) * h[1]
                    exact[c, b * n + a] = P(x) * Q(y)
                    src[c, b * n + a] = om[0, 0] * P.deriv()(x) * Q(y) + om[0, 1] * P(x) * Q.deriv()(y) + st[c] * P(x) * Q(y)
    inflow = np.zeros((1, hp.inflow_size(order, nx, ny)))
    xb = 0.0 if om[0, 0] > 0 else nx * h[0]
    yb = 0.0 if om[0, 1] > 0 else ny * h[1]
    for j in range(ny):
        for b in range(n):
            inflow[0, j * n + b] = P(xb) * Q((j + nodes[b]) * h[1])
    for i in range(nx):
        for a in range(n):
            inflow[0, ny * n + i * n + a] = P((i + nodes[a]) * h[0]) * Q(yb)
    return prob, src, inflow, exact


@pytest.mark.parametrize("order", [1, 2, 3, 4])
@pytest.mark.parametrize("signs", [(1, 1), (-1, 1), (1, -1), (-1, -1)])
def test_h2_polynomial_reproduction(order, signs):
    prob, src, inflow, exact = _poly_case(order, signs)
    psi = hp.sweep_src(prob, src, inflow)
    assert np.max(np.abs(psi[:, 0, :] - exact)) <= 1e-12 * np.max(np.abs(exact))


@pytest.mark.parametrize("order", [2, 3, 4])
def test_h3_sweep_vs_bruteforce(order):
    prob = _prob(3, 2, order, seed=3 + order, voids=True)
    rng = np.random.default_rng(7)
    inflow = rng.uniform(0, 1, (prob.ndirs, hp.inflow_size(order, prob.nx, prob.ny)))
    psi = hp.sweep(prob, None, prob.q, inflow=inflow)
    dirs = range(prob.ndirs)
    if order == 4:
        # the brute-force assembly takes about a second per direction at
        # order 4: the first direction of each quadrant
        sig = [tuple(np.sign(prob.omega[d][:2])) for d in dirs]
        dirs = [sig.index(sg) for sg in sorted(set(sig))]
        assert len(dirs) == 4
    for d in dirs:
        L = bfh.transport_matrix(prob, d)
        f = bfh.load(prob, d, dens=prob.q / (4 * math.pi), inflow=inflow)
        ref = np.linalg.solve(L, f).reshape(prob.ncells, prob.nn)
        assert np.max(np.abs(psi[:, d] - ref)) <= 1e-12 * np.max(np.abs(ref)), d


@pytest.mark.parametrize("order", [2, 3, 4])
def test_h4_balance(order):
    prob = _prob(4, 3, order, seed=11, voids=True)
    psi = hp.sweep(prob, None, prob.q)
    r = hp.Ref1D(order)
    n = order + 1
    w1 = r.M.sum(axis=0)                                  # int of each 1D basis function
    for d in range(prob.ndirs):
        om = prob.omega[d]
        ab = src = 0.0
        for c in range(prob.ncells):
            u = psi[c, d].reshape(n, n)
            ab += prob.sigma_t[c] * prob.h[0] * prob.h[1] * (w1 @ u @ w1)
            src += prob.q[c] / (4 * math.pi) * prob.h[0] * prob.h[1]
        out = 0.0
        for j in range(prob.ny):
            for i in range(prob.nx):
                u = psi[j * prob.nx + i, d].reshape(n, n)
                if (om[0] > 0 and i == prob.nx - 1) or (om[0] < 0 and i == 0):
                    col = u[:, n - 1] if om[0] > 0 else u[:, 0]
                    out += abs(om[0]) * prob.h[1] * (w1 @ col)
                if (om[1] > 0 and j == prob.ny - 1) or (om[1] < 0 and j == 0):
                    row = u[n - 1, :] if om[1] > 0 else u[0, :]
                    out += abs(om[1]) * prob.h[0] * (w1 @ row)
        assert abs(ab + out - src) <= 1e-12 * src, d


@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("form,fname", [(hp.SIP, "sip"), (hp.NIP, "nip"), (hp.MNIP, "mnip")])
def test_h5_diffusion_vs_bruteforce(order, form, fname):
    prob = _prob(3, 3, order, seed=5, voids=False)
    A, cells = hp.dsa_dense(prob, form=form)
    B, cb = bfh.diffusion_matrix(prob, prob.eta, fname)
    assert np.array_equal(cells, cb) and len(cells) > 0
    assert np.allclose(A, B, rtol=0, atol=1e-12 * np.max(np.abs(B)))
    if form == hp.SIP:
        assert np.allclose(A, A.T, atol=1e-14 * np.max(np.abs(A)))
        assert np.linalg.eigvalsh(A).min() > 0


def test_h5_interior_rows_annihilate_constants():
    order = 3
    prob = _prob(6, 6, order, seed=2, voids=False)
    prob.sigma_t[:] = 150.0
    prob.sigma_s[:] = 149.5
    for form in (hp.SIP, hp.NIP, hp.MNIP):
        A, cells = hp.dsa_dense(prob, form=form)
        y = A @ np.ones(A.shape[0])
        Mc = hp.cell_mass(order, prob.h)
        ref = 0.5 * (Mc @ np.ones(prob.nn))
        for s, c in enumerate(cells):
            i, j = c % prob.nx, c // prob.nx
            if 1 <= i <= prob.nx - 2 and 1 <= j <= prob.ny - 2:
                assert np.allclose(y[s * prob.nn:(s + 1) * prob.nn], ref, rtol=1e-11, atol=0), form


@pytest.mark.parametrize("order", [2, 3, 4])
def test_h6_si_fixed_point(order):
    prob = _prob(2, 2, order, seed=9, voids=False) if order == 4 else _prob(3, 2, order, seed=9, voids=False)
    thick = prob.sigma_s >= prob.eta
    prob.sigma_t[thick] = 5.0                    # thick (sigma_s >= 1) at scattering ratio 0.8, so that
    prob.sigma_s[thick] = 4.0                    # plain SI converges in about a hundred iterations
    assert thick.any() and not thick.all()
    A, rhs = bfh.block_system(prob)
    x = np.linalg.solve(A, rhs)
    N = prob.ncells * prob.nn
    ref = x[prob.ndirs * N:].reshape(prob.ncells, prob.nn)
    plain = hp.source_iterate(prob, tol=1e-13, max_it=20000, use_dsa=False)
    assert np.max(np.abs(plain["phi"] - ref)) <= 1e-10 * np.max(np.abs(ref))
    for form in (hp.SIP, hp.NIP, hp.MNIP):
        acc = hp.source_iterate(prob, tol=1e-13, max_it=2000, use_dsa=True, form=form, mass_kind=1)
        assert np.max(np.abs(acc["phi"] - ref)) <= 1e-10 * np.max(np.abs(ref)), form
        assert acc["iters"] < plain["iters"], form


def test_h8_gmres_order1_is_the_q1_oracle():
    """The order-p flexible GMRES at p = 1 against the C oracle's (pinned by
    G1-G3): the same residual history and iterates, with the SIP DSA."""
    prob = _prob(6, 5, 1, seed=4, voids=True)
    for use_dsa in (False, True):
        a = hp.gmres(prob, tol=0.0, max_it=12, restart=5, use_dsa=use_dsa, mass_kind=1)
        b = oracle.gmres(prob, tol=0.0, max_it=12, restart=5, use_dsa=use_dsa, mass_kind=1, cg_rtol=1e-15)
        assert np.allclose(a["res_hist"], b["res_hist"], rtol=1e-8, atol=1e-15)
        assert np.max(np.abs(a["phi"] - b["phi"])) <= 1e-10 * np.max(np.abs(b["phi"]))


@pytest.mark.parametrize("form", [hp.SIP, hp.NIP])
def test_h8_gmres_fixed_point(form):
    prob = _prob(3, 2, 2, seed=9, voids=False)
    A, rhs = bfh.block_system(prob)
    x = np.linalg.solve(A, rhs)
    N = prob.ncells * prob.nn
    ref = x[prob.ndirs * N:].reshape(prob.ncells, prob.nn)
    r = hp.gmres(prob, tol=1e-13, max_it=200, restart=30, use_dsa=True, mass_kind=1, form=form)
    assert r["iters"] < 200
    assert np.max(np.abs(r["phi"] - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert np.all(np.diff(r["res_hist"]) <= 1e-15)            # GMRES residuals never grow within a cycle
