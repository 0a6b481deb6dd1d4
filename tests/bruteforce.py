"""Brute-force dense assembly of the discrete problem for tiny meshes.

An independent path to the same discrete operators the oracle builds: every
matrix here is obtained by evaluating the weak forms with Gauss-Legendre
quadrature on the actual Q1 basis functions at global coordinates, cell by
cell and face by face, and the resulting global matrices are solved densely
with numpy.  Nothing here uses the oracle's 1D/Kronecker formulas.

Weak forms (uniform Cartesian grid, Q1 Lagrange basis on cell corners):
* transport (Section 3.1, eq. Tmat1 at eps = 1), direction Omega, cell K:
    int_K (Omega.grad u) v + sigma_t u v
    + sum_{faces F of K, Omega.n < 0} int_F |Omega.n| (u_K - u_upwind) v
  with u_upwind the neighbour's trace or the boundary inflow;
* block system (eq. system): rows L_d psi_d - Sigma_s phi = q_d and
  phi - sum_d w_d psi_d = 0, Sigma_s the mass matrix of sigma_s/4pi,
  q_d the load of q/4pi;
* SIP diffusion on thick cells (eq. SIP), evaluated pointwise:
    int D grad u.grad v + sigma_a u v
    + sum_faces [ -int {D dn u}[[v]] - int [[u]]{D dn v} + kappa int [[u]][[v]] ]
  with thin neighbours contributing zero values, D = 1/(3 sigma_t).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

_GX, _GW = np.polynomial.legendre.leggauss(3)


def _gauss(a, b):
    x = 0.5 * (b - a) * _GX + 0.5 * (a + b)
    return x, 0.5 * (b - a) * _GW


def _cells(p):
    for k in range(p.nz):
        for j in range(p.ny):
            for i in range(p.nx):
                yield (k * p.ny + j) * p.nx + i, (i, j, k)


def _nodes(p):
    return list(range(p.nn))


def _basis(p, cell_ijk, n, x):
    """Value and gradient of node-n basis of the given cell at global point x (len dim)."""
    h = p.h
    a, b, c = n & 1, (n >> 1) & 1, (n >> 2) & 1
    sides = (a, b, c)
    val = 1.0
    grads = np.zeros(p.dim)
    fac, dfac = [], []
    for ax in range(p.dim):
        lo = cell_ijk[ax] * h[ax]
        t = (x[ax] - lo) / h[ax]
        if sides[ax] == 1:
            fac.append(t)
            dfac.append(1.0 / h[ax])
        else:
            fac.append(1.0 - t)
            dfac.append(-1.0 / h[ax])
    for ax in range(p.dim):
        val *= fac[ax]
        g = dfac[ax]
        for o in range(p.dim):
            if o != ax:
                g *= fac[o]
        grads[ax] = g
    return val, grads


def _cell_points(p, ijk):
    pts = []
    for ax in range(p.dim):
        lo = ijk[ax] * p.h[ax]
        pts.append(_gauss(lo, lo + p.h[ax]))
    for combo in itertools.product(*[range(3)] * p.dim):
        x = np.array([pts[ax][0][combo[ax]] for ax in range(p.dim)])
        wq = np.prod([pts[ax][1][combo[ax]] for ax in range(p.dim)])
        yield x, wq


def _face_points(p, ijk, axis, side):
    """Quadrature on the face of cell ijk normal to `axis` at side 0/1."""
    others = [ax for ax in range(p.dim) if ax != axis]
    pos = (ijk[axis] + side) * p.h[axis]
    pts = []
    for ax in others:
        lo = ijk[ax] * p.h[ax]
        pts.append(_gauss(lo, lo + p.h[ax]))
    for combo in itertools.product(*[range(3)] * len(others)):
        x = np.zeros(p.dim)
        x[axis] = pos
        wq = 1.0
        for o, ax in enumerate(others):
            x[ax] = pts[o][0][combo[o]]
            wq *= pts[o][1][combo[o]]
        yield x, wq


def _neighbour(p, ijk, axis, step):
    nb = list(ijk)
    nb[axis] += step
    lim = (p.nx, p.ny, p.nz)
    if nb[axis] < 0 or nb[axis] >= lim[axis]:
        return None
    return (nb[2] * p.ny + nb[1]) * p.nx + nb[0], tuple(nb)


def _inflow_trace(p, d, inflow, axis, ijk, x):
    """Value at x of the Q1 interpolant of the inflow data on a boundary face."""
    F = 2 if p.dim == 2 else 4
    i, j, k = ijk
    if axis == 0:
        base = (k * p.ny + j) * F
    elif axis == 1:
        base = p.ny * p.nz * F + (k * p.nx + i) * F
    else:
        base = p.ny * p.nz * F + p.nx * p.nz * F + (j * p.nx + i) * F
    others = [ax for ax in range(p.dim) if ax != axis]
    v = 0.0
    for t in range(F):
        bits = [(t >> o) & 1 for o in range(len(others))]
        phi = 1.0
        for o, ax in enumerate(others):
            lo = ijk[ax] * p.h[ax]
            s = (x[ax] - lo) / p.h[ax]
            phi *= s if bits[o] else 1.0 - s
        v += inflow[d, base + t] * phi
    return v


def transport_matrix(p, d, sigma_t=None):
    """Global dense L_d [N x N], N = ncells*nn, rows = test functions."""
    st = p.sigma_t if sigma_t is None else sigma_t
    om = p.omega[d][: p.dim]
    nn = p.nn
    N = p.ncells * nn
    L = np.zeros((N, N))
    for c, ijk in _cells(p):
        for x, wq in _cell_points(p, ijk):
            vals = [_basis(p, ijk, n, x) for n in range(nn)]
            for m in range(nn):
                for n in range(nn):
                    L[c * nn + m, c * nn + n] += wq * (om @ vals[n][1] * vals[m][0] + st[c] * vals[n][0] * vals[m][0])
        for axis in range(p.dim):
            for side in (0, 1):
                on = om[axis] * (1.0 if side == 1 else -1.0)   # Omega . n
                if on >= 0:
                    continue
                nb = _neighbour(p, ijk, axis, 1 if side == 1 else -1)
                for x, wq in _face_points(p, ijk, axis, side):
                    for m in range(nn):
                        vm = _basis(p, ijk, m, x)[0]
                        for n in range(nn):
                            L[c * nn + m, c * nn + n] += wq * abs(on) * _basis(p, ijk, n, x)[0] * vm
                            if nb is not None:
                                L[c * nn + m, nb[0] * nn + n] -= wq * abs(on) * _basis(p, nb[1], n, x)[0] * vm
    return L


def inflow_load(p, d, inflow):
    om = p.omega[d][: p.dim]
    nn = p.nn
    f = np.zeros(p.ncells * nn)
    if inflow is None:
        return f
    for c, ijk in _cells(p):
        for axis in range(p.dim):
            for side in (0, 1):
                on = om[axis] * (1.0 if side == 1 else -1.0)
                if on >= 0 or _neighbour(p, ijk, axis, 1 if side == 1 else -1) is not None:
                    continue
                for x, wq in _face_points(p, ijk, axis, side):
                    g = _inflow_trace(p, d, inflow, axis, ijk, x)
                    for m in range(nn):
                        f[c * nn + m] += wq * abs(on) * g * _basis(p, ijk, m, x)[0]
    return f


def mass_matrix(p, coef):
    """Block-diagonal mass with per-cell coefficient coef[c]."""
    nn = p.nn
    N = p.ncells * nn
    Mg = np.zeros((N, N))
    for c, ijk in _cells(p):
        for x, wq in _cell_points(p, ijk):
            vals = [_basis(p, ijk, n, x)[0] for n in range(nn)]
            for m in range(nn):
                for n in range(nn):
                    Mg[c * nn + m, c * nn + n] += wq * coef[c] * vals[n] * vals[m]
    return Mg


def cell_load(p, dens):
    """Load vector int dens_c v over each cell (dens per cell)."""
    nn = p.nn
    f = np.zeros(p.ncells * nn)
    for c, ijk in _cells(p):
        for x, wq in _cell_points(p, ijk):
            for m in range(nn):
                f[c * nn + m] += wq * dens[c] * _basis(p, ijk, m, x)[0]
    return f


def block_system(p, q=None, inflow=None, sigma_t=None, sigma_s=None):
    """Dense block system of eq. system: unknowns [psi_1..psi_D, phi]."""
    st = p.sigma_t if sigma_t is None else sigma_t
    ss = p.sigma_s if sigma_s is None else sigma_s
    q = p.q if q is None else q
    N = p.ncells * p.nn
    D = p.ndirs
    A = np.zeros(((D + 1) * N, (D + 1) * N))
    rhs = np.zeros((D + 1) * N)
    Ss = mass_matrix(p, ss / (4 * math.pi))
    qd = cell_load(p, q / (4 * math.pi))
    for d in range(D):
        A[d * N:(d + 1) * N, d * N:(d + 1) * N] = transport_matrix(p, d, st)
        A[d * N:(d + 1) * N, D * N:] = -Ss
        A[D * N:, d * N:(d + 1) * N] = -p.w[d] * np.eye(N)
        rhs[d * N:(d + 1) * N] = qd + inflow_load(p, d, inflow)
    A[D * N:, D * N:] = np.eye(N)
    return A, rhs


def sip_matrix(p, eta, sigma_t=None, sigma_s=None, ckappa=8.0, form="sip"):
    """Dense diffusion matrix on the thick cells (sigma_s >= eta), pointwise
    quadrature.  form "sip": eq. SIP with the penalty max(kappa_0, ckappa D/h);
    "nip": the term -int [[u]]{D dv/dn} left out and the penalty kappa_0;
    "mnip": "nip" with the penalty of eq. ModifiedF0 (each direction's
    |Omega.n| weighted by max(0.2 / (sigma_t h), 1) of its upwind cell, so an
    interior face gets the mean of the two cells' factors and a domain face
    the cell's own)."""
    assert form in ("sip", "nip", "mnip")
    mfac = lambda c, axis: max(0.2 / (st[c] * p.h[axis]), 1.0)
    st = p.sigma_t if sigma_t is None else sigma_t
    ss = p.sigma_s if sigma_s is None else sigma_s
    thick = [c for c in range(p.ncells) if ss[c] >= eta]
    slot = {c: s for s, c in enumerate(thick)}
    nn = p.nn
    nf = len(thick) * nn
    Dm = np.zeros((nf, nf))
    k0 = [np.sum(p.w * np.abs(p.omega[:, ax])) / (8 * math.pi) for ax in range(3)]
    cells = dict(_cells(p))

    def dof(c, n):
        return slot[c] * nn + n

    for c in thick:
        ijk = cells[c]
        Dc = 1.0 / (3.0 * st[c])
        sa = st[c] - ss[c]
        for x, wq in _cell_points(p, ijk):
            vals = [_basis(p, ijk, n, x) for n in range(nn)]
            for m in range(nn):
                for n in range(nn):
                    Dm[dof(c, m), dof(c, n)] += wq * (Dc * vals[n][1] @ vals[m][1] + sa * vals[n][0] * vals[m][0])
    # faces: visit each (cell, axis, side=1) plus boundary faces
    for c, ijk in _cells(p):
        for axis in range(p.dim):
            for side in (0, 1):
                nb = _neighbour(p, ijk, axis, 1 if side == 1 else -1)
                if nb is None:
                    if c not in slot:
                        continue
                    kb = k0[axis] * (mfac(c, axis) if form == "mnip" else 1.0)
                    for x, wq in _face_points(p, ijk, axis, side):
                        vals = [_basis(p, ijk, n, x)[0] for n in range(nn)]
                        for m in range(nn):
                            for n in range(nn):
                                Dm[dof(c, m), dof(c, n)] += wq * kb * vals[n] * vals[m]
                    continue
                if side == 0:
                    continue  # interior faces handled once, from the low cell
                cm, cp = c, nb[0]
                ijm, ijp = ijk, nb[1]
                if cm not in slot and cp not in slot:
                    continue
                Dmn = 1.0 / (3.0 * st[cm]) if cm in slot else 0.0
                Dpl = 1.0 / (3.0 * st[cp]) if cp in slot else 0.0
                if form == "sip":
                    kap = max(k0[axis], ckappa * max(Dmn, Dpl) / p.h[axis])
                elif form == "nip":
                    kap = k0[axis]
                else:
                    kap = k0[axis] * 0.5 * (mfac(cm, axis) + mfac(cp, axis))
                sym = 1.0 if form == "sip" else 0.0
                for x, wq in _face_points(p, ijm, axis, 1):
                    # functionals over the DOFs of both cells; thin side contributes nothing
                    ent = []
                    for (cc, ij, sgn, Dc) in ((cm, ijm, 1.0, Dmn), (cp, ijp, -1.0, Dpl)):
                        if cc not in slot:
                            continue
                        for n in range(nn):
                            v, g = _basis(p, ij, n, x)
                            ent.append((dof(cc, n), sgn * v, 0.5 * Dc * g[axis]))
                    for (r, jr, ar) in ent:
                        for (s, js, as_) in ent:
                            Dm[r, s] += wq * (-jr * as_ - sym * ar * js + kap * jr * js)
    return Dm, np.array(thick, dtype=np.int64)
