"""CPU FP64 oracle of the higher-order path: upwind DG of order p = 1..4 (Q_p)
in 2D, source iteration and the heterogeneous DSA at that order.

TEST INFRASTRUCTURE ONLY: the independent checker of the GPU library's
order-p path.  Only the test suite may import it; the product path never
does.  It shares no code with the GPU library.  Plain numpy, slow, small
problems only.

Discretisation (Sec. 3.1 at order p; the paper runs orders 2 and 4 in
Sec. 4):
* Basis: on each cell the tensor product of the 1D Lagrange polynomials on
  the p + 1 Gauss-Lobatto points of [0, 1] (both ends included, so a face
  trace is the values of the nodes on that face).  Node n = i + (p + 1) j,
  i along x.  Integrals are exact (Gauss-Legendre with p + 2 points).
* Transport, direction Omega, cell K (eq. Tmat1 at eps = 1):
    int_K (Omega.grad u) v + sigma_t u v + sum_{inflow faces} int |Omega.n| (u - u_up) v
  with u_up the upwind neighbour's trace, or the boundary inflow.
* Loads: the total isotropic source s = (sigma_s phi + q) / 4pi enters as
  int s v with s nodal (q per cell, constant).
* Diffusion (Sec. 3.1, eqs. SIP, NIP, ModifiedF0) at order p on the thick
  cells (principal submatrix, Sec. 3.2):
    int D grad u.grad v + sigma_a u v + sum_interior faces [ -int {D du/dn}[[v]]
      - sym int [[u]]{D dv/dn} + kappa int [[u]][[v]] ] + sum_domain faces kappa_b int u v,
  D = 1/(3 sigma_t), thin neighbours contributing zero values.
  SIP: sym = 1, kappa = max(kappa_0, 4 p (p + 1) max(D-, D+) / h)  (8 D / h at p = 1);
  NIP: sym = 0, kappa = kappa_0;  mNIP: sym = 0, kappa = kappa_0 (f- + f+) / 2 with
  f = max(c(p) / (sigma_t h), 1), c(p) = 0.1 p (p + 1) (eq. ModifiedF0, C = 0.1);
  kappa_b = kappa_0 (mNIP: times the cell's f); kappa_0 = (1/8pi) sum_d w_d |Omega_d . n|.
  D_ff^{-1} is applied exactly (dense solve).
"""
from __future__ import annotations

import functools
import math

import numpy as np

SIP, NIP, MNIP = 0, 1, 2


def gll_nodes(p):
    """The p + 1 Gauss-Lobatto points on [0, 1]: the ends and the roots of P_p'."""
    if p < 1:
        raise ValueError("order must be >= 1")
    inner = np.polynomial.legendre.Legendre.basis(p).deriv().roots() if p > 1 else np.array([])
    x = np.concatenate(([-1.0], np.sort(inner.real), [1.0]))
    return 0.5 * (x + 1.0)


def lagrange(nodes, k, x):
    """Value of the k-th Lagrange polynomial of `nodes` at x (product form)."""
    v = 1.0
    for m, xm in enumerate(nodes):
        if m != k:
            v *= (x - xm) / (nodes[k] - xm)
    return v


def lagrange_deriv(nodes, k, x):
    """Derivative of the k-th Lagrange polynomial at x (product rule)."""
    s = 0.0
    for j, xj in enumerate(nodes):
        if j == k:
            continue
        t = 1.0 / (nodes[k] - xj)
        for m, xm in enumerate(nodes):
            if m != k and m != j:
                t *= (x - xm) / (nodes[k] - xm)
        s += t
    return s


class Ref1D:
    """1D reference matrices on [0, 1] for order p:
    M[i, j] = int l_i l_j, D[i, j] = int l_i l_j', K[i, j] = int l_i' l_j',
    dl0[i] = l_i'(0), dl1[i] = l_i'(1)."""

    def __init__(self, p):
        self.p = p
        self.np = p + 1
        self.nodes = gll_nodes(p)
        gx, gw = np.polynomial.legendre.leggauss(p + 2)
        gx = 0.5 * (gx + 1.0)
        gw = 0.5 * gw
        n = self.np
        L = np.array([[lagrange(self.nodes, k, x) for x in gx] for k in range(n)])
        dL = np.array([[lagrange_deriv(self.nodes, k, x) for x in gx] for k in range(n)])
        self.M = (L * gw) @ L.T
        self.D = (L * gw) @ dL.T
        self.K = (dL * gw) @ dL.T
        self.dl0 = np.array([lagrange_deriv(self.nodes, k, 0.0) for k in range(n)])
        self.dl1 = np.array([lagrange_deriv(self.nodes, k, 1.0) for k in range(n)])


@functools.lru_cache(maxsize=None)
def ref1d(p):
    """The Ref1D tables of order p, built once."""
    return Ref1D(p)


def _kron2(Y, X):
    """Matrix of the 2D operator X along x, Y along y, for nodes n = i + np j."""
    return np.kron(Y, X)


def cell_mass(p, h):
    r = ref1d(p)
    return _kron2(h[1] * r.M, h[0] * r.M)


def cell_matrix(p, h, om, sigma_t):
    """Transport matrix of one cell for direction om (2D)."""
    r = ref1d(p)
    n = r.np
    B = []
    for a in range(2):
        E = np.zeros((n, n))
        if om[a] > 0:
            E[0, 0] = 1.0          # inflow through the low face
        elif om[a] < 0:
            E[n - 1, n - 1] = 1.0  # inflow through the high face
        B.append(om[a] * r.D + abs(om[a]) * E)
    Mx, My = h[0] * r.M, h[1] * r.M
    return _kron2(h[1] * r.M, B[0]) + _kron2(B[1], h[0] * r.M) + sigma_t * _kron2(My, Mx)


def inflow_size(p, nx, ny):
    """Boundary values per direction: x faces (ny of them) then y faces (nx),
    (p + 1) face nodes each, in the order of the face's tangential node index."""
    return (ny + nx) * (p + 1)


def sweep_src(prob, src, inflow=None, sigma_t=None):
    """psi[c, d, n] = L_d^{-1} (M src_c + inflow load), src nodal [ncells, nn]
    (the total isotropic source density), lexicographic upwind order."""
    p = prob.order
    assert prob.dim == 2
    r = ref1d(p)
    n = r.np
    nx, ny = prob.nx, prob.ny
    h = prob.h
    st = prob.sigma_t if sigma_t is None else sigma_t
    src = np.asarray(src, dtype=np.float64).reshape(prob.ncells, n * n)
    psi = np.zeros((prob.ncells, prob.ndirs, n * n))
    Mc = cell_mass(p, h)
    Fy = h[1] * r.M          # face mass of an x face (tangential y)
    Fx = h[0] * r.M          # face mass of a y face (tangential x)
    for d in range(prob.ndirs):
        om = prob.omega[d][:2]
        A_cache = {}
        ix = range(nx) if om[0] > 0 else range(nx - 1, -1, -1)
        jy = range(ny) if om[1] > 0 else range(ny - 1, -1, -1)
        for j in jy:
            for i in ix:
                c = j * nx + i
                if st[c] not in A_cache:
                    A_cache[st[c]] = cell_matrix(p, h, om, st[c])
                f = Mc @ src[c]
                # x inflow face: nodes i_loc = 0 (om_x > 0) or p, values along y
                ii = 0 if om[0] > 0 else n - 1
                nb = i - 1 if om[0] > 0 else i + 1
                if 0 <= nb < nx:
                    up = psi[j * nx + nb, d].reshape(n, n)[:, n - 1 - ii]   # neighbour's facing nodes, by j_loc
                elif inflow is not None:
                    up = inflow[d, j * n:(j + 1) * n]
                else:
                    up = np.zeros(n)
                load = abs(om[0]) * (Fy @ up)
                for jl in range(n):
                    f[jl * n + ii] += load[jl]
                jj = 0 if om[1] > 0 else n - 1
                nb = j - 1 if om[1] > 0 else j + 1
                if 0 <= nb < ny:
                    up = psi[nb * nx + i, d].reshape(n, n)[n - 1 - jj, :]   # by i_loc
                elif inflow is not None:
                    up = inflow[d, ny * n + i * n: ny * n + (i + 1) * n]
                else:
                    up = np.zeros(n)
                load = abs(om[1]) * (Fx @ up)
                for il in range(n):
                    f[jj * n + il] += load[il]
                psi[c, d] = np.linalg.solve(A_cache[st[c]], f)
    return psi


def source(prob, phi, q, sigma_s=None):
    """Nodal total isotropic source (sigma_s phi + q) / 4pi."""
    ss = prob.sigma_s if sigma_s is None else sigma_s
    phi = np.zeros((prob.ncells, prob.nn)) if phi is None else np.asarray(phi).reshape(prob.ncells, prob.nn)
    q = np.zeros(prob.ncells) if q is None else np.asarray(q)
    return (ss[:, None] * phi + q[:, None]) / (4.0 * math.pi)


def sweep(prob, phi, q, inflow=None, sigma_t=None, sigma_s=None):
    return sweep_src(prob, source(prob, phi, q, sigma_s), inflow, sigma_t)


def moment(prob, psi):
    """phi = sum_d w_d psi_d (eq. phi)."""
    return np.einsum("d,cdn->cn", prob.w, psi)


def kappa0(prob, axis):
    return float(np.sum(prob.w * np.abs(prob.omega[:, axis]))) / (8.0 * math.pi)


def dsa_dense(prob, eta=None, form=SIP, sigma_t=None, sigma_s=None):
    """Dense D_ff of the given form on the thick cells, and the thick cell list."""
    p = prob.order
    r = ref1d(p)
    n = r.np
    nn = n * n
    nx, ny = prob.nx, prob.ny
    h = prob.h
    st = prob.sigma_t if sigma_t is None else sigma_t
    ss = prob.sigma_s if sigma_s is None else sigma_s
    e = prob.eta if eta is None else eta
    cells = np.flatnonzero(ss >= e)
    slot = -np.ones(prob.ncells, dtype=np.int64)
    slot[cells] = np.arange(len(cells))
    N = len(cells) * nn
    A = np.zeros((N, N))
    cp = 0.1 * p * (p + 1)

    def mfac(c, ax):
        if not st[c] > 0.0:
            raise ValueError("mNIP needs sigma_t > 0 at thick cells and their neighbours")
        return max(cp / (st[c] * h[ax]), 1.0)

    M = [h[0] * r.M, h[1] * r.M]
    Kd = [r.K / h[0], r.K / h[1]]
    for s, c in enumerate(cells):
        D = 1.0 / (3.0 * st[c])
        blk = D * (_kron2(M[1], Kd[0]) + _kron2(Kd[1], M[0])) + (st[c] - ss[c]) * _kron2(M[1], M[0])
        A[s * nn:(s + 1) * nn, s * nn:(s + 1) * nn] += blk
    # face helper: the nodal index of (normal index a, tangential index t) along axis ax
    def idx(ax, a, t):
        return (t * n + a) if ax == 0 else (a * n + t)

    k0 = [kappa0(prob, 0), kappa0(prob, 1)]
    for ax in range(2):
        F = M[1 - ax]                          # face mass (tangential axis)
        hn = h[ax]
        ext = (nx + 1, ny) if ax == 0 else (nx, ny + 1)
        for jf in range(ext[1]):
            for i_f in range(ext[0]):
                lo = (i_f - 1, jf) if ax == 0 else (i_f, jf - 1)
                hi = (i_f, jf)
                cl = lo[1] * nx + lo[0] if (lo[ax] >= 0) else -1
                ch = hi[1] * nx + hi[0] if (hi[ax] < (nx, ny)[ax]) else -1
                sl = slot[cl] if cl >= 0 else -1
                sh = slot[ch] if ch >= 0 else -1
                if sl < 0 and sh < 0:
                    continue
                if cl < 0 or ch < 0:
                    c = cl if cl >= 0 else ch
                    s = sl if cl >= 0 else sh
                    a = n - 1 if cl >= 0 else 0
                    kb = k0[ax] * (mfac(c, ax) if form == MNIP else 1.0)
                    for t in range(n):
                        for tp in range(n):
                            A[s * nn + idx(ax, a, t), s * nn + idx(ax, a, tp)] += kb * F[t, tp]
                    continue
                Dm = 1.0 / (3.0 * st[cl]) if sl >= 0 else 0.0
                Dp = 1.0 / (3.0 * st[ch]) if sh >= 0 else 0.0
                if form == SIP:
                    kap = max(k0[ax], 4.0 * p * (p + 1) * max(Dm, Dp) / hn)
                elif form == NIP:
                    kap = k0[ax]
                else:
                    kap = k0[ax] * 0.5 * (mfac(cl, ax) + mfac(ch, ax))
                sym = 1.0 if form == SIP else 0.0
                # local vectors over [K- nodes | K+ nodes]: jump and average normal derivative,
                # per tangential face node t
                jump = np.zeros((n, 2 * nn))
                avg = np.zeros((n, 2 * nn))
                for t in range(n):
                    jump[t, idx(ax, n - 1, t)] += 1.0
                    jump[t, nn + idx(ax, 0, t)] -= 1.0
                    for a in range(n):
                        avg[t, idx(ax, a, t)] += 0.5 * Dm * r.dl1[a] / hn
                        avg[t, nn + idx(ax, a, t)] += 0.5 * Dp * r.dl0[a] / hn
                Bf = (-jump.T @ F @ avg - sym * avg.T @ F @ jump + kap * jump.T @ F @ jump)
                sides = (sl, sh)
                for rs in range(2):
                    if sides[rs] < 0:
                        continue
                    for cs in range(2):
                        if sides[cs] < 0:
                            continue
                        A[sides[rs] * nn:(sides[rs] + 1) * nn, sides[cs] * nn:(sides[cs] + 1) * nn] += \
                            Bf[rs * nn:(rs + 1) * nn, cs * nn:(cs + 1) * nn]
    return A, cells


def dsa_correct(prob, phi_old, phi_si, eta=None, mass_kind=0, form=SIP, A=None):
    """Alg. 2 on the SI residual: phi_si + P_T D_ff^{-1} Sigma_f R_T (phi_si - phi_old)."""
    nn = prob.nn
    if A is None:
        A, cells = dsa_dense(prob, eta, form)
    else:
        A, cells = A
    Mc = cell_mass(prob.order, prob.h)
    coef = prob.sigma_t if mass_kind == 1 else prob.sigma_s
    dphi = np.asarray(phi_si).reshape(prob.ncells, nn) - np.asarray(phi_old).reshape(prob.ncells, nn)
    b = np.concatenate([coef[c] * (Mc @ dphi[c]) for c in cells]) if len(cells) else np.zeros(0)
    out = np.array(phi_si, dtype=np.float64).reshape(prob.ncells, nn).copy()
    if len(cells):
        x = np.linalg.solve(A, b)
        out[cells] += x.reshape(-1, nn)
    return out


def source_iterate(prob, tol=1e-8, max_it=200, use_dsa=True, mass_kind=0, form=SIP, eta=None, phi0=None):
    """Source iteration (eq. DSA_fp) at order p, stop test ||phi_SI - phi|| / ||b|| <= tol
    taken before the DSA step (b: the sweep of q from phi = 0).  Returns dict(phi, iters, res_hist)."""
    nn = prob.nn
    b = moment(prob, sweep(prob, None, prob.q))
    bn = np.linalg.norm(b)
    bn = bn if bn > 0 else 1.0
    phi = np.zeros((prob.ncells, nn)) if phi0 is None else np.array(phi0, dtype=np.float64).reshape(prob.ncells, nn)
    A = dsa_dense(prob, eta, form) if use_dsa else None
    res = []
    it = 0
    while it < max_it:
        phi_si = moment(prob, sweep(prob, phi, prob.q))
        rho = np.linalg.norm(phi_si - phi) / bn
        res.append(rho)
        it += 1
        if use_dsa:
            phi_new = dsa_correct(prob, phi, phi_si, eta, mass_kind, form, A)
        else:
            phi_new = phi_si
        if rho <= tol:
            phi = phi_new
            break
        phi = phi_new
    return {"phi": phi, "iters": it, "res_hist": np.array(res)}


def gmres(prob, tol=1e-8, max_it=200, restart=30, use_dsa=True, mass_kind=0, form=SIP, eta=None):
    """Flexible GMRES(restart) on S phi = b (Sec. 2.2; S = I - sum_d w_d L_d^{-1}
    Sigma_s, b the moment of the sweep of q from phi = 0), right-preconditioned
    by the heterogeneous DSA applied to a vector v as to a residual,
    v + P_T D_ff^{-1} Sigma_f R_T v; modified Gram-Schmidt; zero start.  An
    iteration is one application of S.  Returns dict(phi, iters, res_hist)."""
    nn = prob.nn
    N = prob.ncells * nn
    b = moment(prob, sweep(prob, None, prob.q)).ravel()
    bn = np.linalg.norm(b)
    bn = bn if bn > 0 else 1.0
    A = dsa_dense(prob, eta, form) if use_dsa else None
    zero = np.zeros((prob.ncells, nn))

    def S(x):
        return x - moment(prob, sweep(prob, x.reshape(prob.ncells, nn), None)).ravel()

    def M(v):
        if not use_dsa:
            return v.copy()
        return dsa_correct(prob, zero, v.reshape(prob.ncells, nn), eta, mass_kind, form, A).ravel()

    x = np.zeros(N)
    res = []
    it = 0
    while it < max_it:
        r = b - S(x)
        beta = np.linalg.norm(r)
        if beta / bn <= tol:
            break
        m = restart
        V = np.zeros((m + 1, N))
        Z = np.zeros((m, N))
        H = np.zeros((m + 1, m))
        V[0] = r / beta
        g = np.zeros(m + 1)
        g[0] = beta
        cs = np.zeros(m)
        sn = np.zeros(m)
        j = 0
        done = False
        while j < m and it < max_it:
            Z[j] = M(V[j])
            w = S(Z[j])
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j], H[i + 1, j] = cs[i] * a + sn[i] * c, -sn[i] * a + cs[i] * c
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (H[j, j] / den, H[j + 1, j] / den) if den > 0 else (1.0, 0.0)
            H[j, j] = den
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j += 1
            res.append(abs(g[j]) / bn)
            if res[-1] <= tol:
                done = True
                break
        y = np.linalg.solve(np.triu(H[:j, :j]), g[:j])
        x = x + Z[:j].T @ y
        if done:
            break
    return {"phi": x.reshape(prob.ncells, nn), "iters": it, "res_hist": np.array(res)}
