"""Brute-force dense assembly of the order-p (Q_p) 2D discrete problem for
tiny meshes: the weak forms evaluated with Gauss-Legendre quadrature at
global coordinates, cell by cell and face by face, with the basis built from
monomial coefficients (Vandermonde solves on the Gauss-Lobatto nodes), and
the global matrices solved densely.  Independent of oracle/hp.py (which uses
1D reference matrices, Kronecker products and sweeps).

Weak forms as in the oracle's header: transport with upwind inflow faces,
the block system of eq. system, and the SIP / NIP / mNIP diffusion forms on
the thick cells with thin neighbours contributing zero values.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _gll(p):
    """Gauss-Lobatto points of [0, 1] from the roots of (1 - x^2) P_p'(x)."""
    c = np.zeros(p + 1)
    c[p] = 1.0
    d = np.polynomial.legendre.legder(c)
    inner = np.polynomial.legendre.legroots(d) if p > 1 else np.array([])
    return 0.5 * (np.concatenate(([-1.0], np.sort(inner), [1.0])) + 1.0)


class Basis:
    """Q_p basis of a uniform 2D grid: 1D monomial coefficients per node."""

    def __init__(self, prob):
        self.p = prob.order
        self.n = self.p + 1
        self.h = prob.h
        nodes = _gll(self.p)
        V = np.vander(nodes, self.n, increasing=True)        # V[k, m] = x_k^m
        self.C = np.linalg.solve(V, np.eye(self.n))           # column k: monomial coefficients of l_k
        gx, gw = np.polynomial.legendre.leggauss(self.p + 3)
        self.gx, self.gw = 0.5 * (gx + 1.0), 0.5 * gw

    def l1(self, k, t):
        return sum(self.C[m, k] * t ** m for m in range(self.n))

    def dl1(self, k, t):
        return sum(m * self.C[m, k] * t ** (m - 1) for m in range(1, self.n))

    def val_grad(self, ij, node, x):
        """Value and gradient of the cell's node basis at global point x."""
        a, b = node % self.n, node // self.n
        tx = (x[0] - ij[0] * self.h[0]) / self.h[0]
        ty = (x[1] - ij[1] * self.h[1]) / self.h[1]
        vx, vy = self.l1(a, tx), self.l1(b, ty)
        return vx * vy, np.array([self.dl1(a, tx) / self.h[0] * vy, vx * self.dl1(b, ty) / self.h[1]])

    def cell_points(self, ij):
        for a, b in itertools.product(range(len(self.gx)), repeat=2):
            x = np.array([(ij[0] + self.gx[a]) * self.h[0], (ij[1] + self.gx[b]) * self.h[1]])
            yield x, self.gw[a] * self.gw[b] * self.h[0] * self.h[1]

    def face_points(self, ij, axis, side):
        o = 1 - axis
        for a in range(len(self.gx)):
            x = np.zeros(2)
            x[axis] = (ij[axis] + side) * self.h[axis]
            x[o] = (ij[o] + self.gx[a]) * self.h[o]
            yield x, self.gw[a] * self.h[o]


def _cells(prob):
    for j in range(prob.ny):
        for i in range(prob.nx):
            yield j * prob.nx + i, (i, j)


def _nb(prob, ij, axis, step):
    q = list(ij)
    q[axis] += step
    if q[axis] < 0 or q[axis] >= (prob.nx, prob.ny)[axis]:
        return None
    return q[1] * prob.nx + q[0], tuple(q)


def _inflow_value(prob, B, inflow, d, axis, ij, x):
    """The boundary data's face interpolant at x (face nodes = the GLL nodes)."""
    n = B.n
    o = 1 - axis
    base = ij[1] * n if axis == 0 else prob.ny * n + ij[0] * n
    t = (x[o] - ij[o] * B.h[o]) / B.h[o]
    return sum(inflow[d, base + k] * B.l1(k, t) for k in range(n))


def transport_matrix(prob, d):
    B = Basis(prob)
    nn = prob.nn
    N = prob.ncells * nn
    om = prob.omega[d][:2]
    L = np.zeros((N, N))
    for c, ij in _cells(prob):
        for x, wq in B.cell_points(ij):
            vg = [B.val_grad(ij, k, x) for k in range(nn)]
            for m in range(nn):
                for k in range(nn):
                    L[c * nn + m, c * nn + k] += wq * ((om @ vg[k][1]) * vg[m][0] + prob.sigma_t[c] * vg[k][0] * vg[m][0])
        for axis in range(2):
            for side in (0, 1):
                on = om[axis] * (1.0 if side else -1.0)
                if on >= 0:
                    continue
                nb = _nb(prob, ij, axis, 1 if side else -1)
                for x, wq in B.face_points(ij, axis, side):
                    for m in range(nn):
                        vm = B.val_grad(ij, m, x)[0]
                        for k in range(nn):
                            L[c * nn + m, c * nn + k] += wq * abs(on) * B.val_grad(ij, k, x)[0] * vm
                            if nb is not None:
                                L[c * nn + m, nb[0] * nn + k] -= wq * abs(on) * B.val_grad(nb[1], k, x)[0] * vm
    return L


def load(prob, d, src_fn=None, dens=None, inflow=None):
    """int s v over cells (s from a callable of global x, or a per-cell constant
    density) plus the inflow boundary load of direction d."""
    B = Basis(prob)
    nn = prob.nn
    om = prob.omega[d][:2]
    f = np.zeros(prob.ncells * nn)
    for c, ij in _cells(prob):
        for x, wq in B.cell_points(ij):
            s = src_fn(x) if src_fn is not None else (dens[c] if dens is not None else 0.0)
            for m in range(nn):
                f[c * nn + m] += wq * s * B.val_grad(ij, m, x)[0]
        if inflow is None:
            continue
        for axis in range(2):
            for side in (0, 1):
                on = om[axis] * (1.0 if side else -1.0)
                if on >= 0 or _nb(prob, ij, axis, 1 if side else -1) is not None:
                    continue
                for x, wq in B.face_points(ij, axis, side):
                    g = _inflow_value(prob, B, inflow, d, axis, ij, x)
                    for m in range(nn):
                        f[c * nn + m] += wq * abs(on) * g * B.val_grad(ij, m, x)[0]
    return f


def mass_matrix(prob, coef):
    B = Basis(prob)
    nn = prob.nn
    Mg = np.zeros((prob.ncells * nn, prob.ncells * nn))
    for c, ij in _cells(prob):
        for x, wq in B.cell_points(ij):
            v = [B.val_grad(ij, k, x)[0] for k in range(nn)]
            for m in range(nn):
                for k in range(nn):
                    Mg[c * nn + m, c * nn + k] += wq * coef[c] * v[k] * v[m]
    return Mg


def block_system(prob):
    """Dense eq. system: unknowns [psi_1..psi_D, phi], vacuum boundaries."""
    N = prob.ncells * prob.nn
    D = prob.ndirs
    A = np.zeros(((D + 1) * N, (D + 1) * N))
    rhs = np.zeros((D + 1) * N)
    Ss = mass_matrix(prob, prob.sigma_s / (4 * math.pi))
    for d in range(D):
        A[d * N:(d + 1) * N, d * N:(d + 1) * N] = transport_matrix(prob, d)
        A[d * N:(d + 1) * N, D * N:] = -Ss
        A[D * N:, d * N:(d + 1) * N] = -prob.w[d] * np.eye(N)
        rhs[d * N:(d + 1) * N] = load(prob, d, dens=prob.q / (4 * math.pi))
    A[D * N:, D * N:] = np.eye(N)
    return A, rhs


def diffusion_matrix(prob, eta, form="sip"):
    """Dense thick-cell diffusion matrix evaluated pointwise (forms as in the oracle's header)."""
    B = Basis(prob)
    p = prob.order
    nn = prob.nn
    st, ss = prob.sigma_t, prob.sigma_s
    thick = np.flatnonzero(ss >= eta)
    slot = {c: s for s, c in enumerate(thick)}
    N = len(thick) * nn
    A = np.zeros((N, N))
    k0 = [float(np.sum(prob.w * np.abs(prob.omega[:, a]))) / (8 * math.pi) for a in range(2)]
    cp = 0.1 * p * (p + 1)
    f = lambda c, a: max(cp / (st[c] * prob.h[a]), 1.0)
    for c, ij in _cells(prob):
        if c not in slot:
            continue
        s = slot[c]
        D = 1.0 / (3.0 * st[c])
        for x, wq in B.cell_points(ij):
            vg = [B.val_grad(ij, k, x) for k in range(nn)]
            for m in range(nn):
                for k in range(nn):
                    A[s * nn + m, s * nn + k] += wq * (D * vg[k][1] @ vg[m][1] + (st[c] - ss[c]) * vg[k][0] * vg[m][0])
    for c, ij in _cells(prob):
        for axis in range(2):
            # faces on the low side of c (interior) and every domain face of a thick cell
            for side in (0, 1):
                nb = _nb(prob, ij, axis, 1 if side else -1)
                if nb is None:
                    if c not in slot:
                        continue
                    s = slot[c]
                    kb = k0[axis] * (f(c, axis) if form == "mnip" else 1.0)
                    for x, wq in B.face_points(ij, axis, side):
                        v = [B.val_grad(ij, k, x)[0] for k in range(nn)]
                        for m in range(nn):
                            for k in range(nn):
                                A[s * nn + m, s * nn + k] += wq * kb * v[k] * v[m]
                    continue
                if side == 1:
                    continue            # each interior face once, from its high cell
                cm, ijm = nb            # low cell
                cpl, ijp = c, ij        # high cell
                if cm not in slot and cpl not in slot:
                    continue
                Dm = 1.0 / (3.0 * st[cm]) if cm in slot else 0.0
                Dp = 1.0 / (3.0 * st[cpl]) if cpl in slot else 0.0
                if form == "sip":
                    kap = max(k0[axis], 4.0 * p * (p + 1) * max(Dm, Dp) / prob.h[axis])
                elif form == "nip":
                    kap = k0[axis]
                else:
                    kap = k0[axis] * 0.5 * (f(cm, axis) + f(cpl, axis))
                sym = 1.0 if form == "sip" else 0.0
                side_cells = [(cm, ijm, +1.0, Dm), (cpl, ijp, -1.0, Dp)]
                for x, wq in B.face_points(ij, axis, 0):
                    # per side: jump sign, value and normal (x_axis) derivative of each basis function
                    vals = {}
                    for cc, cij, sg, Dc in side_cells:
                        vals[cc] = [B.val_grad(cij, k, x) for k in range(nn)]
                    for cr, rij, sgr, Dr in side_cells:
                        if cr not in slot:
                            continue
                        for cq, qij, sgq, Dq in side_cells:
                            if cq not in slot:
                                continue
                            for m in range(nn):
                                vm, gm = vals[cr][m]
                                for k in range(nn):
                                    vk, gk = vals[cq][k]
                                    jr, jq = sgr * vm, sgq * vk                  # [[v]], [[u]]
                                    ar, aq = 0.5 * Dr * gm[axis], 0.5 * Dq * gk[axis]  # {D dv/dn}, {D du/dn}
                                    A[slot[cr] * nn + m, slot[cq] * nn + k] += wq * (-aq * jr - sym * ar * jq +
                                                                                      kap * jq * jr)
    return A, thick
