/*
 * oracle.c -- plain FP64 CPU reference for source iteration with
 * heterogeneous (thick-only) DSA on a uniform Cartesian Q1 upwind-DG grid.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent checker of the GPU
 * library: it shares no code, header or table with it, and only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  Nothing in the product path calls it.
 *
 * It is written to be read against the paper, not to be fast:
 *   - every cell matrix is assembled densely from 1D mass / upwind blocks by
 *     explicit Kronecker products and solved by LU with partial pivoting;
 *   - each direction is swept in lexicographic order from its upwind corner
 *     (forward) or from its downwind corner with transposed blocks (adjoint);
 *   - the thick-region diffusion matrix is assembled from the SIP bilinear
 *     form face by face (jump / average functionals) and solved by plain,
 *     unpreconditioned CG.
 *
 * Readings of the paper that it fixes (one per item):
 *   (1) phi = sum_d w_d psi_d with sum w = 4 pi; scattering load
 *       M sigma_s phi / 4pi (Sigma_s has coefficient sigma_s/4pi, Sec. 2.2);
 *       the isotropic source density q enters as M q / 4pi (eq. Tmat1).
 *   (2) Q1 Lagrange basis on the cell corners, exact integrals, no lumping.
 *   (3) upwind coupling: on an inflow face (Omega.n < 0) the load
 *       int |Omega.n| v psi_upwind is added; outflow faces carry nothing.
 *   (4) thick iff sigma_s >= eta (Sec. 2.3, Sec. 3.2), all DOFs of a thick
 *       cell thick.
 *   (5) diffusion operator: SIP form (eq. SIP) with D = 1/(3 sigma_t),
 *       penalty kappa = max((1/8pi) sum_d w_d |Omega_d.n|, 8 D/h), principal
 *       submatrix on thick DOFs (Sec. 3.2): thick-thin faces keep the thick
 *       side's terms only, domain faces get kappa int u v.
 *   (6) Alg. 2 acts on the source-iteration residual: phi <- phi_SI +
 *       P_T D_ff^{-1} Sigma_f (phi_SI - phi) with Sigma_f the mass matrix of
 *       sigma_s (mass_kind 0) or sigma_t (mass_kind 1, Sec. 2.2 footnote).
 *   (7) stopping test ||phi_SI - phi||_2 / ||b||_2 <= tol, b = first sweep
 *       from phi = 0 (eq. source0), tested before the DSA step.
 *   (8) Alg. 1 (triangular heterogeneous DSA) acts on the same residual:
 *       after the thick update of (6), the thick part of the preconditioned
 *       residual, phi_bar = [0; (phi_new - phi)_f], is swept once with zero
 *       external source and vacuum inflow, and the moment of that sweep is
 *       added to the thin DOFs only (eq. approxS and the identity below it).
 *   (9) Krylov view (Sec. 2.2): S phi = b with S = I - sum_d w_d L_d^{-1}
 *       Sigma_s and b = sum_d w_d L_d^{-1} q_d, solved by flexible GMRES(m)
 *       with the heterogeneous DSA of (6) or (8) as the right preconditioner
 *       (applied to a vector v as to a residual: v + P_T D_ff^{-1} Sigma_f
 *       R_T v).  The residual ||b - S phi|| / ||b|| is the same quantity as
 *       the source-iteration residual of (7).
 *   (10) the nonsymmetric forms of Sec. 3.1 (dsa_op): NIP (eq. NIP) drops
 *       the face term -int [[u]]{D dv/dn} of (5), mNIP also replaces the
 *       penalty by the modified one of eq. ModifiedF0 (C = 0.1, p = 1, h the
 *       cell size across the face).  Both take the paper's penalty alone,
 *       without the 8 D/h floor of (5).  D_ff^{-1} is applied exactly for
 *       them, by a banded LU factorisation with partial pivoting of the
 *       assembled matrix (factored once per assembly): the correction's plain
 *       definition, whatever the conditioning of the high-contrast
 *       full-DSA inputs.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

typedef struct {
    int dim, nx, ny, nz;
    double hx, hy, hz;
} orc_mesh;

/* ------------------------------------------------------------------ */
/* 1D building blocks on a cell of width h (nodes at the two ends).    */
/* ------------------------------------------------------------------ */

/* consistent mass: int l_i l_j dx */
static void mass1(double h, double m[2][2]) {
    m[0][0] = m[1][1] = h / 3.0;
    m[0][1] = m[1][0] = h / 6.0;
}

/* stiffness: int l_i' l_j' dx */
static void stiff1(double h, double s[2][2]) {
    s[0][0] = s[1][1] = 1.0 / h;
    s[0][1] = s[1][0] = -1.0 / h;
}

/* upwind streaming block for a direction component c:
 *   int c l_j' l_i dx - (inflow-end) c l_j l_i, divided by |c|.
 * c > 0: inflow at node 0 -> [[1/2, 1/2], [-1/2, 1/2]];
 * c < 0: inflow at node 1 -> its transpose.                          */
static void upwind1(double c, double g[2][2]) {
    double gp[2][2] = {{0.5, 0.5}, {-0.5, 0.5}};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            g[i][j] = (c > 0) ? gp[i][j] : gp[j][i];
}

static int nnodes(const orc_mesh *m) { return m->dim == 2 ? 4 : 8; }
static long ncells(const orc_mesh *m) { return (long)m->nx * m->ny * m->nz; }

/* node n = a + 2b + 4c -> (a, b, c) */
static void node_abc(int n, int *a, int *b, int *c) {
    *a = n & 1;
    *b = (n >> 1) & 1;
    *c = (n >> 2) & 1;
}

/* 3-factor product Z[c][c'] Y[b][b'] X[a][a'] (2D: Z == 1) */
static double kron3(int dim, double X[2][2], double Y[2][2], double Z[2][2], int n, int np) {
    int a, b, c, ap, bp, cp;
    node_abc(n, &a, &b, &c);
    node_abc(np, &ap, &bp, &cp);
    double v = X[a][ap] * Y[b][bp];
    if (dim == 3) v *= Z[c][cp];
    return v;
}

/* Cell mass matrix M_K (nn x nn). */
void orc_cell_mass(int dim, const double h[3], double *M) {
    double mx[2][2], my[2][2], mz[2][2];
    mass1(h[0], mx);
    mass1(h[1], my);
    mass1(h[2], mz);
    int nn = dim == 2 ? 4 : 8;
    for (int n = 0; n < nn; ++n)
        for (int np = 0; np < nn; ++np)
            M[n * nn + np] = kron3(dim, mx, my, mz, n, np);
}

/* Cell matrix of the upwind-DG transport operator for direction om
 * (eq. Tmat1 at eps = 1 on one Cartesian Q1 cell):
 *   A = |mu| Mz (x) My (x) G_x + |eta| Mz (x) G_y (x) Mx
 *     + sigma_t Mz (x) My (x) Mx + |xi| G_z (x) My (x) Mx,
 * summed in that order.  The first two terms (P), the mass (Mm) and the
 * z term (Z) do not depend on the cell, so a sweep forms them once per
 * direction and each cell adds sigma_t Mm: A = (P + sigma_t Mm) + Z. */
static void cell_matrix_parts(int dim, const double h[3], const double om[3], double *P, double *Mm, double *Z) {
    double mx[2][2], my[2][2], mz[2][2], gx[2][2], gy[2][2], gz[2][2];
    mass1(h[0], mx);
    mass1(h[1], my);
    mass1(h[2], mz);
    upwind1(om[0], gx);
    upwind1(om[1], gy);
    upwind1(om[2], gz);
    int nn = dim == 2 ? 4 : 8;
    for (int n = 0; n < nn; ++n)
        for (int np = 0; np < nn; ++np) {
            P[n * nn + np] = fabs(om[0]) * kron3(dim, gx, my, mz, n, np)
                           + fabs(om[1]) * kron3(dim, mx, gy, mz, n, np);
            Mm[n * nn + np] = kron3(dim, mx, my, mz, n, np);
            Z[n * nn + np] = dim == 3 ? fabs(om[2]) * kron3(dim, mx, my, gz, n, np) : 0.0;
        }
}

static void cell_matrix_from_parts(int dim, const double *P, const double *Mm, const double *Z, double sigma_t,
                                   double *A) {
    int nn = dim == 2 ? 4 : 8;
    for (int e = 0; e < nn * nn; ++e) {
        double v = P[e] + sigma_t * Mm[e];
        if (dim == 3) v += Z[e];
        A[e] = v;
    }
}

void orc_cell_matrix(int dim, const double h[3], const double om[3], double sigma_t, double *A) {
    double P[64], Mm[64], Z[64];
    cell_matrix_parts(dim, h, om, P, Mm, Z);
    cell_matrix_from_parts(dim, P, Mm, Z, sigma_t, A);
}

/* Solve A x = b in place (b -> x) by LU with partial pivoting. A is destroyed.
 * Returns 0, or 1 if a pivot is exactly zero. */
static int lu_solve(int n, double *A, double *b) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > fabs(A[p * n + k])) p = i;
        if (A[p * n + k] == 0.0) return 1;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = A[k * n + j];
                A[k * n + j] = A[p * n + j];
                A[p * n + j] = t;
            }
            double t = b[k];
            b[k] = b[p];
            b[p] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            b[i] -= f * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j];
        b[i] = s / A[i * n + i];
    }
    return 0;
}

/* Transverse face mass on a face normal to `axis`, indexed by the face-local
 * node t (2D: the other axis' node; 3D: (first other) + 2 (second other)). */
static void face_mass(const orc_mesh *m, int axis, double *Mf /* F x F */) {
    double hh[3] = {m->hx, m->hy, m->hz};
    double m1[2][2], m2[2][2];
    int o1 = axis == 0 ? 1 : 0;
    int o2 = axis == 2 ? 1 : 2;
    mass1(hh[o1], m1);
    if (m->dim == 2) {
        for (int t = 0; t < 2; ++t)
            for (int tp = 0; tp < 2; ++tp) Mf[t * 2 + tp] = m1[t][tp];
        return;
    }
    mass1(hh[o2], m2);
    for (int t = 0; t < 4; ++t)
        for (int tp = 0; tp < 4; ++tp)
            Mf[t * 4 + tp] = m1[t & 1][tp & 1] * m2[t >> 1][tp >> 1];
}

/* Cell node with coordinate `side` along `axis` and face-local index t. */
static int face_node(int dim, int axis, int side, int t) {
    int o1 = t & 1, o2 = (t >> 1) & 1;
    int a, b, c;
    if (axis == 0) { a = side; b = o1; c = o2; }
    else if (axis == 1) { a = o1; b = side; c = o2; }
    else { a = o1; b = o2; c = side; }
    (void)dim;
    return a + 2 * b + 4 * c;
}

/* Index of a boundary face node in the per-direction inflow layout. */
static long inflow_index(const orc_mesh *m, int axis, int i, int j, int k, int t) {
    int F = m->dim == 2 ? 2 : 4;
    long offy = (long)m->ny * m->nz * F;
    long offz = offy + (long)m->nx * m->nz * F;
    if (axis == 0) return ((long)k * m->ny + j) * F + t;
    if (axis == 1) return offy + ((long)k * m->nx + i) * F + t;
    return offz + ((long)j * m->nx + i) * F + t;
}

long orc_inflow_size(const orc_mesh *m) {
    if (m->dim == 2) return 2L * m->ny + 2L * m->nx;
    return 4L * ((long)m->ny * m->nz + (long)m->nx * m->nz + (long)m->nx * m->ny);
}

/* ------------------------------------------------------------------ */
/* Transport sweep for one direction (eq. psi: psi_d = L_d^{-1}(...)).  */
/* ------------------------------------------------------------------ */

/* load[c*nn + n]: volume load vector of every cell.
 * Forward (transpose == 0): visit cells from the upwind corner in
 *   lexicographic order; on each inflow face add |Omega_a| Mf psi_upwind
 *   (neighbour's values on the shared face, or the boundary inflow).
 * Transpose (transpose == 1): solve with L_d^T, visiting cells from the
 *   downwind corner; on each outflow face add |Omega_a| Mf x_downwind
 *   (or the boundary data), then solve with A_K^T.
 * psi_out[c*nn + n] receives this direction's solution. */
static int sweep_one(const orc_mesh *m, const double om[3], const double *sigma_t,
                     const double *load, const double *inflow_d, int transpose,
                     double *psi_out) {
    int nn = nnodes(m), dim = m->dim;
    int F = nn / 2;
    double h[3] = {m->hx, m->hy, m->hz};
    int n3[3] = {m->nx, m->ny, m->nz};
    double Mf[3][16];
    for (int ax = 0; ax < dim; ++ax) face_mass(m, ax, Mf[ax]);
    /* per axis: step direction of the visiting order, and the side of the
     * cell whose face couples to the previously visited neighbour */
    int step[3], cside[3];
    for (int ax = 0; ax < 3; ++ax) {
        int pos = om[ax] > 0;
        if (!transpose) {          /* upwind first; couple through inflow face */
            step[ax] = pos ? 1 : -1;
            cside[ax] = pos ? 0 : 1;
        } else {                   /* downwind first; couple through outflow face */
            step[ax] = pos ? -1 : 1;
            cside[ax] = pos ? 1 : 0;
        }
    }
    double A[64], rhs[8];
    double Pd[64], Md[64], Zd[64];
    cell_matrix_parts(dim, h, om, Pd, Md, Zd);
    for (int kk = 0; kk < n3[2]; ++kk) {
        int k = step[2] > 0 ? kk : n3[2] - 1 - kk;
        if (dim == 2) k = 0;
        for (int jj = 0; jj < n3[1]; ++jj) {
            int j = step[1] > 0 ? jj : n3[1] - 1 - jj;
            for (int ii = 0; ii < n3[0]; ++ii) {
                int i = step[0] > 0 ? ii : n3[0] - 1 - ii;
                long c = ((long)k * m->ny + j) * m->nx + i;
                for (int n = 0; n < nn; ++n) rhs[n] = load[c * nn + n];
                int idx[3] = {i, j, k};
                for (int ax = 0; ax < dim; ++ax) {
                    /* neighbour across the coupling face */
                    int nb[3] = {i, j, k};
                    nb[ax] -= step[ax];
                    const double *val = NULL;
                    double bval[4];
                    int nbside = 1 - cside[ax];
                    if (nb[ax] < 0 || nb[ax] >= n3[ax]) {
                        if (!inflow_d) continue;  /* vacuum */
                        for (int t = 0; t < F; ++t)
                            bval[t] = inflow_d[inflow_index(m, ax, idx[0], idx[1], idx[2], t)];
                        val = bval;
                    } else {
                        long cn = ((long)nb[2] * m->ny + nb[1]) * m->nx + nb[0];
                        for (int t = 0; t < F; ++t)
                            bval[t] = psi_out[cn * nn + face_node(dim, ax, nbside, t)];
                        val = bval;
                    }
                    for (int t = 0; t < F; ++t) {
                        double s = 0.0;
                        for (int tp = 0; tp < F; ++tp) s += Mf[ax][t * F + tp] * val[tp];
                        rhs[face_node(dim, ax, cside[ax], t)] += fabs(om[ax]) * s;
                    }
                }
                double Ak[64];
                cell_matrix_from_parts(dim, Pd, Md, Zd, sigma_t[c], Ak);
                if (transpose) {
                    for (int r = 0; r < nn; ++r)
                        for (int s2 = 0; s2 < nn; ++s2) A[r * nn + s2] = Ak[s2 * nn + r];
                } else {
                    memcpy(A, Ak, sizeof(double) * nn * nn);
                }
                if (lu_solve(nn, A, rhs)) return 1;
                for (int n = 0; n < nn; ++n) psi_out[c * nn + n] = rhs[n];
            }
        }
    }
    return 0;
}

/* Volume load of every cell: M_K (sigma_s,K phi_K + q_K) / 4pi. */
static void volume_load(const orc_mesh *m, const double *sigma_s, const double *phi,
                        const double *q, double *load) {
    int nn = nnodes(m);
    double h[3] = {m->hx, m->hy, m->hz};
    double M[64];
    orc_cell_mass(m->dim, h, M);
    long nc = ncells(m);
    for (long c = 0; c < nc; ++c)
        for (int n = 0; n < nn; ++n) {
            double s = 0.0;
            for (int np = 0; np < nn; ++np) {
                double f = (phi ? sigma_s[c] * phi[c * nn + np] : 0.0) + (q ? q[c] : 0.0);
                s += M[n * nn + np] * f;
            }
            load[c * nn + n] = s / (4.0 * ORC_PI);
        }
}

/* All directions: psi[(c*ndirs + d)*nn + n]. inflow: [ndirs][nbf] or NULL. */
int orc_sweep(const orc_mesh *m, int ndirs, const double *omega, const double *sigma_t,
              const double *sigma_s, const double *phi, const double *q, const double *inflow,
              int transpose, double *psi) {
    int nn = nnodes(m);
    long nc = ncells(m), nbf = orc_inflow_size(m);
    double *load = malloc(sizeof(double) * nc * nn);
    if (!load) return 3;
    volume_load(m, sigma_s, phi, q, load);
    int err = 0;
#pragma omp parallel
    {
        double *pd = malloc(sizeof(double) * nc * nn);
#pragma omp for schedule(static)
        for (int d = 0; d < ndirs; ++d) {
            if (!pd) { err = 3; continue; }
            if (sweep_one(m, &omega[3 * d], sigma_t, load, inflow ? inflow + (long)d * nbf : NULL,
                          transpose, pd))
                err = 4;
            for (long c = 0; c < nc; ++c)
                for (int n = 0; n < nn; ++n) psi[(c * ndirs + d) * nn + n] = pd[c * nn + n];
        }
        free(pd);
    }
    free(load);
    return err;
}

/* phi = sum_d w_d psi_d (the scalar-flux moment). */
void orc_moment(const orc_mesh *m, int ndirs, const double *w, const double *psi, double *phi) {
    int nn = nnodes(m);
    long nc = ncells(m);
    for (long c = 0; c < nc; ++c)
        for (int n = 0; n < nn; ++n) {
            double s = 0.0;
            for (int d = 0; d < ndirs; ++d) s += w[d] * psi[(c * ndirs + d) * nn + n];
            phi[c * nn + n] = s;
        }
}

/* One transport update without storing psi: phi_si = sum_d w_d L_d^{-1}(load).
 * Directions are split statically over threads; each thread accumulates its
 * directions in order into a private array, and the partial arrays are added
 * in thread order. */
static int transport_update(const orc_mesh *m, int ndirs, const double *omega, const double *w,
                            const double *sigma_t, const double *load, const double *inflow,
                            int transpose, double *phi_si) {
    int nn = nnodes(m);
    long nc = ncells(m), nbf = orc_inflow_size(m);
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *part = calloc((size_t)nth * nc * nn, sizeof(double));
    if (!part) return 3;
    int err = 0;
#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *pd = malloc(sizeof(double) * nc * nn);
        double *acc = part + (size_t)tid * nc * nn;
#pragma omp for schedule(static)
        for (int d = 0; d < ndirs; ++d) {
            if (!pd) { err = 3; continue; }
            if (sweep_one(m, &omega[3 * d], sigma_t, load, inflow ? inflow + (long)d * nbf : NULL,
                          transpose, pd))
                err = 4;
            for (long i = 0; i < nc * nn; ++i) acc[i] += w[d] * pd[i];
        }
        free(pd);
    }
    for (long i = 0; i < nc * nn; ++i) {
        double s = 0.0;
        for (int t = 0; t < nth; ++t) s += part[(size_t)t * nc * nn + i];
        phi_si[i] = s;
    }
    free(part);
    return err;
}

/* ------------------------------------------------------------------ */
/* Heterogeneous DSA: SIP diffusion on the thick cells (Alg. 2).        */
/* ------------------------------------------------------------------ */

/* Block-sparse matrix over thick cells: for thick slot s the blocks
 * (s, s) and (s, neighbour slot) for each thick face neighbour. */
typedef struct {
    int nn, nthick, nb;          /* nb = 1 + 2*dim blocks per row */
    int op;                      /* 0 SIP, 1 NIP, 2 mNIP (eq. SIP, eq. NIP, eq. ModifiedF0) */
    long *cell;                  /* slot -> cell */
    int *col;                    /* [nthick][nb] neighbour slot or -1 */
    double *blk;                 /* [nthick][nb][nn][nn] */
    /* NIP, mNIP: band LU factors of the whole matrix (n = nthick nn rows),
     * row i holding columns i - kl .. i + kl + ku at lu[i * ldb + j - i + kl] */
    double *lu;
    long *piv;
    long kl, ku, ldb;
} dsa_mat;

static void dsa_free(dsa_mat *A) {
    free(A->cell);
    free(A->col);
    free(A->blk);
    free(A->lu);
    free(A->piv);
    memset(A, 0, sizeof(*A));
}

/* kappa_0 along an axis: (1/8pi) sum_d w_d |Omega_d,axis| */
static double kappa0(int ndirs, const double *omega, const double *w, int axis) {
    double s = 0.0;
    for (int d = 0; d < ndirs; ++d) s += w[d] * fabs(omega[3 * d + axis]);
    return s / (8.0 * ORC_PI);
}

static double *blockp(dsa_mat *A, int s, int b) {
    return A->blk + ((size_t)s * A->nb + b) * A->nn * A->nn;
}

/* Band LU with partial pivoting (Gaussian elimination restricted to the
 * band; the pivot search looks kl rows down, and a row swap widens the upper
 * band to kl + ku).  Returns 8 for a zero pivot (singular matrix). */
static int band_factor(dsa_mat *A) {
    const int nn = A->nn;
    const long n = (long)A->nthick * nn;
    long kl = 0, ku = 0;
    for (int s = 0; s < A->nthick; ++s)
        for (int b = 0; b < A->nb; ++b) {
            int c = A->col[s * A->nb + b];
            if (c < 0) continue;
            long lo = ((long)s - c) * nn + (nn - 1), hi = ((long)c - s) * nn + (nn - 1);
            if (lo > kl) kl = lo;
            if (hi > ku) ku = hi;
        }
    A->kl = kl;
    A->ku = ku;
    A->ldb = 2 * kl + ku + 1;
    A->lu = calloc((size_t)(n ? n : 1) * A->ldb, sizeof(double));
    A->piv = malloc(sizeof(long) * (n ? n : 1));
    if (!A->lu || !A->piv) return 3;
#define LU(i, j) A->lu[(size_t)(i) * A->ldb + ((j) - (i) + kl)]
    for (int s = 0; s < A->nthick; ++s)
        for (int b = 0; b < A->nb; ++b) {
            int c = A->col[s * A->nb + b];
            if (c < 0) continue;
            const double *B = A->blk + ((size_t)s * A->nb + b) * nn * nn;
            for (int r = 0; r < nn; ++r)
                for (int q = 0; q < nn; ++q) LU((long)s * nn + r, (long)c * nn + q) += B[r * nn + q];
        }
    for (long k = 0; k < n; ++k) {
        long last = k + kl < n - 1 ? k + kl : n - 1;
        long jend = k + kl + ku < n - 1 ? k + kl + ku : n - 1;
        long p = k;
        for (long i = k + 1; i <= last; ++i)
            if (fabs(LU(i, k)) > fabs(LU(p, k))) p = i;
        A->piv[k] = p;
        if (LU(p, k) == 0.0) return 8;
        if (p != k)
            for (long j = k; j <= jend; ++j) {
                double t = LU(k, j);
                LU(k, j) = LU(p, j);
                LU(p, j) = t;
            }
        for (long i = k + 1; i <= last; ++i) {
            double l = LU(i, k) / LU(k, k);
            LU(i, k) = l;
            for (long j = k + 1; j <= jend; ++j) LU(i, j) -= l * LU(k, j);
        }
    }
    return 0;
}

/* x = D^{-1} b from the band LU factors */
static void band_solve(const dsa_mat *A, const double *b, double *x) {
    const long n = (long)A->nthick * A->nn, kl = A->kl, ku = A->ku;
    for (long i = 0; i < n; ++i) x[i] = b[i];
    for (long k = 0; k < n; ++k) {
        long p = A->piv[k];
        if (p != k) {
            double t = x[k];
            x[k] = x[p];
            x[p] = t;
        }
        long last = k + kl < n - 1 ? k + kl : n - 1;
        for (long i = k + 1; i <= last; ++i) x[i] -= LU(i, k) * x[k];
    }
    for (long i = n - 1; i >= 0; --i) {
        long jend = i + kl + ku < n - 1 ? i + kl + ku : n - 1;
        double v = x[i];
        for (long j = i + 1; j <= jend; ++j) v -= LU(i, j) * x[j];
        x[i] = v / LU(i, i);
    }
}
#undef LU

/* mNIP penalty factor of one side of a face (eq. ModifiedF0 for linear
 * elements: c(p) = C p (p+1) with C = 0.1, p = 1), h the cell size across
 * the face */
static double mnip_factor(double sigma_t, double h) {
    double f = 0.2 / (sigma_t * h);
    return f > 1.0 ? f : 1.0;
}

/* Assemble the thick-cell diffusion matrix (principal submatrix, Sec. 3.2) of
 * one of the forms of Sec. 3.1 at eps = 1:
 * Cell terms: D int grad u . grad v + sigma_a int u v, D = 1/(3 sigma_t).
 * Interior face between K- (low) and K+ (high) along axis a, normal +e_a:
 *   SIP (eq. SIP): -int {D du/dn}[[v]] - int [[u]]{D dv/dn} + kappa int [[u]][[v]],
 *     kappa = max(kappa_0, 8 max(D-, D+)/h);
 *   NIP (eq. NIP): the term -int [[u]]{D dv/dn} dropped, kappa = kappa_0;
 *   mNIP: NIP with kappa = kappa_0 (f(sigma_t-) + f(sigma_t+))/2 (eq.
 *     ModifiedF0: each direction's term weighted by the factor f of its upwind
 *     side, mnip_factor; half of the weighted sum comes from either side),
 *     the thin side's sigma_t included;
 *   [[u]] = u- - u+, {D du/dn} = (D- du-/dx_a + D+ du+/dx_a)/2;
 *   rows/columns of a thin cell are dropped (its D never enters).
 * Domain-boundary face of a thick cell: kappa_0 int u v (mNIP: times f of
 * the cell).  Returns 1 for mNIP with a void (sigma_t = 0) cell next to a
 * thick one, where eq. ModifiedF0 is undefined. */
static int dsa_assemble(const orc_mesh *m, int ndirs, const double *omega, const double *w,
                        const double *sigma_t, const double *sigma_s, double eta, int op, dsa_mat *A,
                        long **slot_of_cell_out) {
    int nn = nnodes(m), dim = m->dim, F = nn / 2;
    long nc = ncells(m);
    long *slot = malloc(sizeof(long) * nc);
    if (!slot) return 3;
    int nthick = 0;
    for (long c = 0; c < nc; ++c) slot[c] = (sigma_s[c] >= eta) ? nthick++ : -1;
    A->nn = nn;
    A->nthick = nthick;
    A->nb = 1 + 2 * dim;
    A->op = op;
    A->cell = malloc(sizeof(long) * (nthick ? nthick : 1));
    A->col = malloc(sizeof(int) * (size_t)(nthick ? nthick : 1) * A->nb);
    A->blk = calloc((size_t)(nthick ? nthick : 1) * A->nb * nn * nn, sizeof(double));
    if (!A->cell || !A->col || !A->blk) { free(slot); return 3; }
    for (long c = 0; c < nc; ++c)
        if (slot[c] >= 0) A->cell[slot[c]] = c;
    for (int s = 0; s < nthick; ++s)
        for (int b = 0; b < A->nb; ++b) A->col[s * A->nb + b] = (b == 0) ? s : -1;

    double h[3] = {m->hx, m->hy, m->hz};
    int n3[3] = {m->nx, m->ny, m->nz};
    double mx[2][2], my[2][2], mz[2][2], sx[2][2], sy[2][2], sz[2][2];
    mass1(h[0], mx); mass1(h[1], my); mass1(h[2], mz);
    stiff1(h[0], sx); stiff1(h[1], sy); stiff1(h[2], sz);
    double k0[3];
    for (int ax = 0; ax < 3; ++ax) k0[ax] = kappa0(ndirs, omega, w, ax);

    /* cell terms */
    for (int s = 0; s < nthick; ++s) {
        long c = A->cell[s];
        double D = 1.0 / (3.0 * sigma_t[c]);
        double sa = sigma_t[c] - sigma_s[c];
        double *B = blockp(A, s, 0);
        for (int n = 0; n < nn; ++n)
            for (int np = 0; np < nn; ++np) {
                double st = kron3(dim, sx, my, mz, n, np) + kron3(dim, mx, sy, mz, n, np);
                if (dim == 3) st += kron3(dim, mx, my, sz, n, np);
                B[n * nn + np] += D * st + sa * kron3(dim, mx, my, mz, n, np);
            }
    }
    /* faces */
    for (int ax = 0; ax < dim; ++ax) {
        double Mf[16];
        face_mass(m, ax, Mf);
        int lim[3] = {n3[0], n3[1], dim == 3 ? n3[2] : 1};
        /* face position p along ax: between cell p-1 and p (p = 0..n) */
        int ext[3] = {lim[0], lim[1], lim[2]};
        ext[ax] += 1;
        for (int k = 0; k < ext[2]; ++k)
            for (int j = 0; j < ext[1]; ++j)
                for (int i = 0; i < ext[0]; ++i) {
                    int p[3] = {i, j, k};
                    int lo[3] = {i, j, k}, hi[3] = {i, j, k};
                    lo[ax] -= 1;
                    long cl = -1, chh = -1;
                    if (lo[ax] >= 0) cl = ((long)lo[2] * m->ny + lo[1]) * m->nx + lo[0];
                    if (hi[ax] < n3[ax]) chh = ((long)hi[2] * m->ny + hi[1]) * m->nx + hi[0];
                    long sl = cl >= 0 ? slot[cl] : -1, sh = chh >= 0 ? slot[chh] : -1;
                    if (sl < 0 && sh < 0) continue;
                    (void)p;
                    if (cl < 0 || chh < 0) {
                        /* domain boundary face of a thick cell */
                        long s = cl >= 0 ? sl : sh;
                        int side = cl >= 0 ? 1 : 0;
                        double kb = k0[ax];
                        if (op == 2) {
                            double stc = sigma_t[cl >= 0 ? cl : chh];
                            if (!(stc > 0.0)) { free(slot); return 1; }
                            kb *= mnip_factor(stc, h[ax]);
                        }
                        double *B = blockp(A, (int)s, 0);
                        for (int t = 0; t < F; ++t)
                            for (int tp = 0; tp < F; ++tp)
                                B[face_node(dim, ax, side, t) * nn + face_node(dim, ax, side, tp)] +=
                                    kb * Mf[t * F + tp];
                        continue;
                    }
                    /* interior face: local DOF vector = [K- (nn) | K+ (nn)] */
                    double Dm = sl >= 0 ? 1.0 / (3.0 * sigma_t[cl]) : 0.0;
                    double Dp = sh >= 0 ? 1.0 / (3.0 * sigma_t[chh]) : 0.0;
                    double kap = k0[ax];
                    if (op == 0) {
                        double Dmax = Dm > Dp ? Dm : Dp;
                        if (8.0 * Dmax / h[ax] > kap) kap = 8.0 * Dmax / h[ax];
                    } else if (op == 2) {
                        if (!(sigma_t[cl] > 0.0) || !(sigma_t[chh] > 0.0)) { free(slot); return 1; }
                        kap = k0[ax] * 0.5 * (mnip_factor(sigma_t[cl], h[ax]) + mnip_factor(sigma_t[chh], h[ax]));
                    }
                    const double sym = op == 0 ? 1.0 : 0.0;  /* the -int [[u]]{D dv/dn} term */
                    double jump[4][16], avg[4][16];
                    for (int t = 0; t < F; ++t) {
                        for (int q = 0; q < 2 * nn; ++q) jump[t][q] = avg[t][q] = 0.0;
                        jump[t][face_node(dim, ax, 1, t)] += 1.0;           /* u-  */
                        jump[t][nn + face_node(dim, ax, 0, t)] -= 1.0;      /* -u+ */
                        avg[t][face_node(dim, ax, 1, t)] += 0.5 * Dm / h[ax];
                        avg[t][face_node(dim, ax, 0, t)] -= 0.5 * Dm / h[ax];
                        avg[t][nn + face_node(dim, ax, 1, t)] += 0.5 * Dp / h[ax];
                        avg[t][nn + face_node(dim, ax, 0, t)] -= 0.5 * Dp / h[ax];
                    }
                    double Bf[16][16];
                    for (int r = 0; r < 2 * nn; ++r)
                        for (int q = 0; q < 2 * nn; ++q) {
                            double v = 0.0;
                            for (int t = 0; t < F; ++t)
                                for (int tp = 0; tp < F; ++tp)
                                    v += Mf[t * F + tp] * (-jump[t][r] * avg[tp][q] - sym * avg[t][r] * jump[tp][q] +
                                                           kap * jump[t][r] * jump[tp][q]);
                            Bf[r][q] = v;
                        }
                    /* scatter the thick part */
                    long sides[2] = {sl, sh};
                    for (int rs = 0; rs < 2; ++rs) {
                        if (sides[rs] < 0) continue;
                        for (int cs = 0; cs < 2; ++cs) {
                            if (sides[cs] < 0) continue;
                            int bslot;
                            if (rs == cs) bslot = 0;
                            else bslot = 1 + 2 * ax + (cs == 1 ? 1 : 0); /* high or low neighbour */
                            A->col[sides[rs] * A->nb + bslot] = (int)sides[cs];
                            double *B = blockp(A, (int)sides[rs], bslot);
                            for (int r = 0; r < nn; ++r)
                                for (int q = 0; q < nn; ++q) B[r * nn + q] += Bf[rs * nn + r][cs * nn + q];
                        }
                    }
                }
    }
    *slot_of_cell_out = slot;
    if (op != 0) {
        int rc = band_factor(A);
        if (rc) return rc;
    }
    return 0;
}

/* y = D_ff x, row block by row block (rows are independent, so the rows are
 * shared out over threads; each row's sum is formed in the same order). */
static void dsa_apply(const dsa_mat *A, const double *x, double *y) {
    int nn = A->nn;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < A->nthick; ++s) {
        for (int r = 0; r < nn; ++r) {
            double v = 0.0;
            for (int b = 0; b < A->nb; ++b) {
                int cs = A->col[s * A->nb + b];
                if (cs < 0) continue;
                const double *B = A->blk + ((size_t)s * A->nb + b) * nn * nn;
                for (int q = 0; q < nn; ++q) v += B[r * nn + q] * x[(size_t)cs * nn + q];
            }
            y[(size_t)s * nn + r] = v;
        }
    }
}

static double dot(long n, const double *a, const double *b) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Plain conjugate gradients from a zero guess; stops when ||r|| <= rtol ||b||. */
static int cg_solve(const dsa_mat *A, const double *b, double *x, double rtol, int maxit, int *iters,
                    double *relres) {
    long n = (long)A->nthick * A->nn;
    double *r = malloc(sizeof(double) * (n ? n : 1));
    double *p = malloc(sizeof(double) * (n ? n : 1));
    double *q = malloc(sizeof(double) * (n ? n : 1));
    if (!r || !p || !q) { free(r); free(p); free(q); return 3; }
    for (long i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; p[i] = b[i]; }
    double bn = sqrt(dot(n, b, b));
    double rr = bn * bn;
    int it = 0, rc = 0;
    if (bn == 0.0) { *iters = 0; *relres = 0.0; free(r); free(p); free(q); return 0; }
    while (sqrt(rr) > rtol * bn && it < maxit) {
        dsa_apply(A, p, q);
        double pq = dot(n, p, q);
        if (!(pq > 0.0)) { rc = 7; break; }
        double alpha = rr / pq;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        double rr2 = dot(n, r, r);
        double beta = rr2 / rr;
        rr = rr2;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        ++it;
    }
    *iters = it;
    *relres = sqrt(rr) / bn;
    free(r); free(p); free(q);
    return rc;
}

/* The nonsymmetric forms: x = D^{-1} b by the band LU factors; relres is
 * the true residual ||b - D x|| / ||b|| of the result. */
static int direct_solve(const dsa_mat *A, const double *b, double *x, int *iters, double *relres) {
    long n = (long)A->nthick * A->nn;
    double *r = malloc(sizeof(double) * (n ? n : 1));
    if (!r) return 3;
    band_solve(A, b, x);
    dsa_apply(A, x, r);
    for (long i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double bn = sqrt(dot(n, b, b)), rn = sqrt(dot(n, r, r));
    *iters = 0;
    *relres = bn > 0.0 ? rn / bn : 0.0;
    free(r);
    return (rn == rn) ? 0 : 7;
}

/* Alg. 2 applied to the SI residual:
 *   phi_out = phi_si + P_T D_ff^{-1} Sigma_f R_T (phi_si - phi_old). */
static int dsa_correct_with(const orc_mesh *m, const dsa_mat *A, const double *sigma_t,
                            const double *sigma_s, int mass_kind, const double *phi_old,
                            const double *phi_si, double cg_rtol, int cg_maxit, double *phi_out,
                            int *cg_iters, double *cg_relres) {
    int nn = nnodes(m);
    long nc = ncells(m);
    long nf = (long)A->nthick * nn;
    double h[3] = {m->hx, m->hy, m->hz};
    double M[64];
    orc_cell_mass(m->dim, h, M);
    double *b = malloc(sizeof(double) * (nf ? nf : 1));
    double *x = malloc(sizeof(double) * (nf ? nf : 1));
    if (!b || !x) { free(b); free(x); return 3; }
    for (int s = 0; s < A->nthick; ++s) {
        long c = A->cell[s];
        double coef = mass_kind == 1 ? sigma_t[c] : sigma_s[c];
        for (int n = 0; n < nn; ++n) {
            double v = 0.0;
            for (int np = 0; np < nn; ++np) v += M[n * nn + np] * (phi_si[c * nn + np] - phi_old[c * nn + np]);
            b[(size_t)s * nn + n] = coef * v;
        }
    }
    int it = 0;
    double rr = 0.0;
    int rc = A->op == 0 ? cg_solve(A, b, x, cg_rtol, cg_maxit, &it, &rr)
                        : direct_solve(A, b, x, &it, &rr);
    if (phi_out != phi_si) memcpy(phi_out, phi_si, sizeof(double) * nc * nn);
    for (int s = 0; s < A->nthick; ++s) {
        long c = A->cell[s];
        for (int n = 0; n < nn; ++n) phi_out[c * nn + n] += x[(size_t)s * nn + n];
    }
    if (cg_iters) *cg_iters = it;
    if (cg_relres) *cg_relres = rr;
    free(b);
    free(x);
    return rc;
}

int orc_dsa_correct(const orc_mesh *m, int ndirs, const double *omega, const double *w,
                    const double *sigma_t, const double *sigma_s, double eta, int mass_kind, int dsa_op,
                    const double *phi_old, const double *phi_si, double cg_rtol, int cg_maxit,
                    double *phi_out, int *cg_iters, double *cg_relres) {
    dsa_mat A;
    memset(&A, 0, sizeof(A));
    long *slot = NULL;
    int rc = dsa_assemble(m, ndirs, omega, w, sigma_t, sigma_s, eta, dsa_op, &A, &slot);
    if (rc) { dsa_free(&A); free(slot); return rc; }
    rc = dsa_correct_with(m, &A, sigma_t, sigma_s, mass_kind, phi_old, phi_si, cg_rtol, cg_maxit,
                          phi_out, cg_iters, cg_relres);
    dsa_free(&A);
    free(slot);
    return rc;
}

/* Dense copy of D_ff (for small problems): D[(s*nn+r)*nf + cs*nn+q];
 * thick_cells[s] = cell of slot s.  Returns the number of thick cells via *nthick. */
int orc_dsa_dense(const orc_mesh *m, int ndirs, const double *omega, const double *w,
                  const double *sigma_t, const double *sigma_s, double eta, int dsa_op, double *D,
                  long *thick_cells, int *nthick) {
    dsa_mat A;
    memset(&A, 0, sizeof(A));
    long *slot = NULL;
    int rc = dsa_assemble(m, ndirs, omega, w, sigma_t, sigma_s, eta, dsa_op, &A, &slot);
    if (rc) { dsa_free(&A); free(slot); return rc; }
    int nn = A.nn;
    long nf = (long)A.nthick * nn;
    *nthick = A.nthick;
    if (D) {
        memset(D, 0, sizeof(double) * nf * nf);
        for (int s = 0; s < A.nthick; ++s)
            for (int b = 0; b < A.nb; ++b) {
                int cs = A.col[s * A.nb + b];
                if (cs < 0) continue;
                const double *B = A.blk + ((size_t)s * A.nb + b) * nn * nn;
                for (int r = 0; r < nn; ++r)
                    for (int q = 0; q < nn; ++q) D[((long)s * nn + r) * nf + (long)cs * nn + q] += B[r * nn + q];
            }
    }
    if (thick_cells)
        for (int s = 0; s < A.nthick; ++s) thick_cells[s] = A.cell[s];
    dsa_free(&A);
    free(slot);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Source iteration with optional heterogeneous DSA (eq. DSA_fp).       */
/* ------------------------------------------------------------------ */

static double norm2(long n, const double *a) { return sqrt(dot(n, a, a)); }

/* Alg. 1, second step: phi_new restricted to the thin cells gains the moment
 * of one sweep of phi_bar = [0; (phi_new - phi_old)_f] with zero external
 * source and vacuum inflow (the thick part of the preconditioned residual
 * carried into the thin region by a transport update). */
static int triangular_step(const orc_mesh *m, int ndirs, const double *omega, const double *w,
                           const double *sigma_t, const double *sigma_s, const long *slot, int transpose,
                           const double *phi_old, double *phi_new, double *work_bar, double *work_load,
                           double *work_zeta) {
    int nn = nnodes(m);
    long nc = ncells(m);
    for (long c = 0; c < nc; ++c)
        for (int n = 0; n < nn; ++n)
            work_bar[c * nn + n] = slot[c] >= 0 ? phi_new[c * nn + n] - phi_old[c * nn + n] : 0.0;
    volume_load(m, sigma_s, work_bar, NULL, work_load);
    int e = transport_update(m, ndirs, omega, w, sigma_t, work_load, NULL, transpose, work_zeta);
    if (e) return e;
    for (long c = 0; c < nc; ++c)
        if (slot[c] < 0)
            for (int n = 0; n < nn; ++n) phi_new[c * nn + n] += work_zeta[c * nn + n];
    return 0;
}

/* phi_inout: initial guess in, last iterate out.  res_hist / cg_hist: [max_it]
 * (may be NULL).  dsa_form: 0 diagonal (Alg. 2), 1 triangular (Alg. 1).
 * Returns 0 converged, 5 not converged, 6 diverged (non-finite or residual
 * above 1e6 times the first), or an error code. */
int orc_source_iterate(const orc_mesh *m, int ndirs, const double *omega, const double *w,
                       const double *sigma_t, const double *sigma_s, const double *q,
                       const double *inflow, double eta, int use_dsa, int mass_kind, int dsa_op, double tol,
                       int max_it, double cg_rtol, int cg_maxit, int transpose, int dsa_form,
                       double *phi_inout, double *res_hist, int *cg_hist, int *iters_out) {
    int nn = nnodes(m);
    long nc = ncells(m), n = nc * nn;
    double *load = malloc(sizeof(double) * n);
    double *phi_si = malloc(sizeof(double) * n);
    double *phi_old = malloc(sizeof(double) * n);
    double *bar = malloc(sizeof(double) * n);
    double *zeta = malloc(sizeof(double) * n);
    dsa_mat A;
    memset(&A, 0, sizeof(A));
    long *slot = NULL;
    int rc = 0;
    if (!load || !phi_si || !phi_old || !bar || !zeta) { rc = 3; goto done; }
    if (use_dsa) {
        rc = dsa_assemble(m, ndirs, omega, w, sigma_t, sigma_s, eta, dsa_op, &A, &slot);
        if (rc) goto done;
    }
    /* ||b||: the first transport update from phi = 0 */
    double bnorm;
    {
        volume_load(m, sigma_s, NULL, q, load);
        rc = transport_update(m, ndirs, omega, w, sigma_t, load, inflow, transpose, phi_si);
        if (rc) goto done;
        bnorm = norm2(n, phi_si);
        if (bnorm == 0.0) bnorm = 1.0;
    }
    double first = -1.0;
    int it;
    rc = 5;
    for (it = 0; it < max_it; ++it) {
        volume_load(m, sigma_s, phi_inout, q, load);
        int e = transport_update(m, ndirs, omega, w, sigma_t, load, inflow, transpose, phi_si);
        if (e) { rc = e; break; }
        double rr = 0.0;
        for (long i = 0; i < n; ++i) {
            double d = phi_si[i] - phi_inout[i];
            rr += d * d;
        }
        double res = sqrt(rr) / bnorm;
        if (res_hist) res_hist[it] = res;
        if (first < 0) first = res;
        int stop = res <= tol;
        int cgi = 0;
        if (use_dsa) {
            double crr;
            memcpy(phi_old, phi_inout, sizeof(double) * n);
            e = dsa_correct_with(m, &A, sigma_t, sigma_s, mass_kind, phi_inout, phi_si, cg_rtol,
                                 cg_maxit, phi_inout, &cgi, &crr);
            if (e) { rc = e; break; }
            if (dsa_form == 1) {
                e = triangular_step(m, ndirs, omega, w, sigma_t, sigma_s, slot, transpose, phi_old, phi_inout,
                                    bar, load, zeta);
                if (e) { rc = e; break; }
            }
        } else {
            memcpy(phi_inout, phi_si, sizeof(double) * n);
        }
        if (cg_hist) cg_hist[it] = cgi;
        if (!isfinite(res) || res > 1e6 * first) { rc = 6; ++it; break; }
        if (stop) { rc = 0; ++it; break; }
    }
    if (iters_out) *iters_out = it;
done:
    dsa_free(&A);
    free(slot);
    free(load);
    free(phi_si);
    free(phi_old);
    free(bar);
    free(zeta);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Krylov view: flexible GMRES(m) on S phi = b (eq. schur).            */
/* ------------------------------------------------------------------ */

/* y = S x = x - sum_d w_d L_d^{-1} (M sigma_s x / 4pi), homogeneous
 * boundary (the operator of eq. schur). */
static int schur_apply(const orc_mesh *m, int ndirs, const double *omega, const double *w,
                       const double *sigma_t, const double *sigma_s, int transpose, const double *x,
                       double *load, double *y) {
    long n = ncells(m) * nnodes(m);
    volume_load(m, sigma_s, x, NULL, load);
    int e = transport_update(m, ndirs, omega, w, sigma_t, load, NULL, transpose, y);
    if (e) return e;
    for (long i = 0; i < n; ++i) y[i] = x[i] - y[i];
    return 0;
}

/* z = M^{-1} v: heterogeneous DSA applied to v as to a residual,
 * z = v + P_T D_ff^{-1} Sigma_f R_T v (Alg. 2), plus for Alg. 1 the thin
 * update of triangular_step from the thick part of z. */
static int dsa_precond(const orc_mesh *m, int ndirs, const double *omega, const double *w,
                       const double *sigma_t, const double *sigma_s, const dsa_mat *A, const long *slot,
                       int mass_kind, int dsa_form, int transpose, double cg_rtol, int cg_maxit,
                       const double *v, double *z, double *zero, double *bar, double *load, double *zeta,
                       int *cg_iters) {
    long n = ncells(m) * nnodes(m);
    double crr;
    for (long i = 0; i < n; ++i) zero[i] = 0.0;
    int e = dsa_correct_with(m, A, sigma_t, sigma_s, mass_kind, zero, v, cg_rtol, cg_maxit, z, cg_iters, &crr);
    if (e) return e;
    if (dsa_form == 1)
        return triangular_step(m, ndirs, omega, w, sigma_t, sigma_s, slot, transpose, zero, z, bar, load, zeta);
    return 0;
}

/* Flexible GMRES(restart) from the initial guess phi_inout, right
 * preconditioned by the heterogeneous DSA (use_dsa) or not at all.  Modified
 * Gram-Schmidt Arnoldi, Givens rotations; an iteration is one application
 * of S (one sweep of every direction).  res_hist[k] = the least-squares
 * residual estimate |g_{j+1}| / ||b|| after iteration k (at a restart the
 * true residual is recomputed).  Stops when that estimate is <= tol. */
int orc_gmres(const orc_mesh *m, int ndirs, const double *omega, const double *w, const double *sigma_t,
              const double *sigma_s, const double *q, const double *inflow, double eta, int use_dsa,
              int mass_kind, int dsa_op, int dsa_form, double tol, int max_it, int restart, double cg_rtol,
              int cg_maxit, int transpose, double *phi_inout, double *res_hist, int *cg_hist, int *iters_out) {
    int nn = nnodes(m);
    long n = ncells(m) * nn;
    int mr = restart;
    if (mr < 1) return 1;
    double *b = malloc(sizeof(double) * n), *r = malloc(sizeof(double) * n);
    double *load = malloc(sizeof(double) * n), *wv = malloc(sizeof(double) * n);
    double *zero = malloc(sizeof(double) * n), *bar = malloc(sizeof(double) * n);
    double *zeta = malloc(sizeof(double) * n);
    double *V = malloc(sizeof(double) * n * (mr + 1)), *Z = malloc(sizeof(double) * n * mr);
    double *H = calloc((size_t)(mr + 1) * mr, sizeof(double));
    double *cs = malloc(sizeof(double) * mr), *sn = malloc(sizeof(double) * mr);
    double *g = malloc(sizeof(double) * (mr + 1)), *y = malloc(sizeof(double) * mr);
    dsa_mat A;
    memset(&A, 0, sizeof(A));
    long *slot = NULL;
    int rc = 0, it = 0;
    if (!b || !r || !load || !wv || !zero || !bar || !zeta || !V || !Z || !H || !cs || !sn || !g || !y) {
        rc = 3;
        goto done;
    }
    if (use_dsa && (rc = dsa_assemble(m, ndirs, omega, w, sigma_t, sigma_s, eta, dsa_op, &A, &slot))) goto done;
    /* b = sum_d w_d L_d^{-1}(q_d + inflow load) */
    volume_load(m, sigma_s, NULL, q, load);
    if ((rc = transport_update(m, ndirs, omega, w, sigma_t, load, inflow, transpose, b))) goto done;
    double bnorm = norm2(n, b);
    if (bnorm == 0.0) bnorm = 1.0;
    rc = 5;
    while (it < max_it) {
        /* r = b - S x */
        int e = schur_apply(m, ndirs, omega, w, sigma_t, sigma_s, transpose, phi_inout, load, r);
        if (e) { rc = e; break; }
        for (long i = 0; i < n; ++i) r[i] = b[i] - r[i];
        double beta = norm2(n, r);
        if (!isfinite(beta)) { rc = 6; break; }
        if (beta / bnorm <= tol) { rc = 0; break; }
        for (long i = 0; i < n; ++i) V[i] = r[i] / beta;
        for (int k = 0; k <= mr; ++k) g[k] = 0.0;
        g[0] = beta;
        int j, done_cycle = 0;
        for (j = 0; j < mr && it < max_it; ++j) {
            double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
            int cgi = 0;
            if (use_dsa) {
                e = dsa_precond(m, ndirs, omega, w, sigma_t, sigma_s, &A, slot, mass_kind, dsa_form, transpose,
                                cg_rtol, cg_maxit, vj, zj, zero, bar, load, zeta, &cgi);
                if (e) { rc = e; break; }
            } else {
                memcpy(zj, vj, sizeof(double) * n);
            }
            e = schur_apply(m, ndirs, omega, w, sigma_t, sigma_s, transpose, zj, load, wv);
            if (e) { rc = e; break; }
            for (int i = 0; i <= j; ++i) {
                const double *vi = V + (size_t)i * n;
                double h = dot(n, wv, vi);
                H[(size_t)i * mr + j] = h;
                for (long k = 0; k < n; ++k) wv[k] -= h * vi[k];
            }
            double hn = norm2(n, wv);
            H[(size_t)(j + 1) * mr + j] = hn;
            if (hn > 0.0)
                for (long k = 0; k < n; ++k) V[(size_t)(j + 1) * n + k] = wv[k] / hn;
            /* previous rotations on the new column, then a new rotation */
            for (int i = 0; i < j; ++i) {
                double a = H[(size_t)i * mr + j], c2 = H[(size_t)(i + 1) * mr + j];
                H[(size_t)i * mr + j] = cs[i] * a + sn[i] * c2;
                H[(size_t)(i + 1) * mr + j] = -sn[i] * a + cs[i] * c2;
            }
            {
                double a = H[(size_t)j * mr + j], c2 = H[(size_t)(j + 1) * mr + j];
                double den = sqrt(a * a + c2 * c2);
                cs[j] = den > 0.0 ? a / den : 1.0;
                sn[j] = den > 0.0 ? c2 / den : 0.0;
                H[(size_t)j * mr + j] = den;
                H[(size_t)(j + 1) * mr + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
            }
            double res = fabs(g[j + 1]) / bnorm;
            if (res_hist) res_hist[it] = res;
            if (cg_hist) cg_hist[it] = cgi;
            ++it;
            if (!isfinite(res)) { rc = 6; done_cycle = 1; ++j; break; }
            if (res <= tol || hn == 0.0) { done_cycle = 1; ++j; break; }
        }
        if (rc != 5 && rc != 6) break;
        /* x += Z y, with H(0:j, 0:j) y = g(0:j) by back substitution */
        for (int i = j - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < j; ++k) s -= H[(size_t)i * mr + k] * y[k];
            y[i] = s / H[(size_t)i * mr + i];
        }
        for (int k = 0; k < j; ++k)
            for (long i = 0; i < n; ++i) phi_inout[i] += y[k] * Z[(size_t)k * n + i];
        if (rc == 6) break;
        if (done_cycle) {
            rc = 0;
            break;
        }
    }
    if (iters_out) *iters_out = it;
done:
    dsa_free(&A);
    free(slot);
    free(b); free(r); free(load); free(wv); free(zero); free(bar); free(zeta);
    free(V); free(Z); free(H); free(cs); free(sn); free(g); free(y);
    return rc;
}

/* Gradient of a linear response J with respect to per-cell log cross sections
 * (adjoint of the discrete block system, eq. system):
 *   dJ/dlog sigma_t,K = -sigma_t,K sum_d w_d psiadj_d,K^T M_K psi_d,K
 *   dJ/dlog sigma_s,K =  sigma_s,K chi_K^T M_K phi_K / 4pi
 * psi, psi_adj: [(c*ndirs + d)*nn + n]; phi, chi: [c*nn + n]. */
void orc_gradient(const orc_mesh *m, int ndirs, const double *w, const double *sigma_t,
                  const double *sigma_s, const double *psi, const double *psi_adj, const double *phi,
                  const double *chi, double *g_lst, double *g_lss) {
    int nn = nnodes(m);
    long nc = ncells(m);
    double h[3] = {m->hx, m->hy, m->hz};
    double M[64];
    orc_cell_mass(m->dim, h, M);
    for (long c = 0; c < nc; ++c) {
        double st = 0.0;
        for (int d = 0; d < ndirs; ++d) {
            const double *a = psi_adj + (c * ndirs + d) * nn;
            const double *b = psi + (c * ndirs + d) * nn;
            double v = 0.0;
            for (int r = 0; r < nn; ++r)
                for (int q2 = 0; q2 < nn; ++q2) v += a[r] * M[r * nn + q2] * b[q2];
            st += w[d] * v;
        }
        g_lst[c] = -sigma_t[c] * st;
        double ss = 0.0;
        for (int r = 0; r < nn; ++r)
            for (int q2 = 0; q2 < nn; ++q2) ss += chi[c * nn + r] * M[r * nn + q2] * phi[c * nn + q2];
        g_lss[c] = sigma_s[c] * ss / (4.0 * ORC_PI);
    }
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
