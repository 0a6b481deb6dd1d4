// Order-p (p = 2, 3, 4) 2D path: the constant tables of the discretisation and
// the launchers of hp.hip.  hp_tables builds the tables on the host from the
// Gauss-Lobatto nodes (see hp.hip for how the sweep and the diffusion rows
// use them).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>

#include "sn_kernels.hpp"

namespace sn {

constexpr int kHpMaxN = 5;  // nodes per axis at the highest order built (p = 4)
struct HpTab {
    int p;
    double lr[kHpMaxN], li[kHpMaxN];                    // eigenvalues of G = M^{-1} (D + e0 e0^T)
    double Vr[kHpMaxN][kHpMaxN], Vi[kHpMaxN][kHpMaxN];  // V[node][k]: eigenvectors in the columns
    double Wr[kHpMaxN][kHpMaxN], Wi[kHpMaxN][kHpMaxN];  // V^{-1}[k][node]
    double c0[kHpMaxN];                                 // M^{-1} e_0
    double M[kHpMaxN][kHpMaxN], K[kHpMaxN][kHpMaxN];    // int l_i l_j, int l_i' l_j' on [0, 1]
    double dl0[kHpMaxN], dl1[kHpMaxN];                  // l_i'(0), l_i'(1)
};

hipError_t launch_sweep_hp(const HpTab& tb, int nx, int ny, int ndirs, long nbf, const DirInfo* dirs,
                           const double* sigt, const double* sigs, const double* phi, const double* q,
                           const double* inflow, double* psi, hipStream_t st);
hipError_t launch_moment_hp(long nc, int ndirs, int nn, const double* w, const double* psi, double* phi,
                            hipStream_t st);
// blk [nthick][5][nn][nn], col [nthick][5] (block 0 the cell, 1 + 2 axis + side the face neighbour)
hipError_t launch_hp_assemble(const HpTab& tb, const DsaGeom& g, int op, const int* thick_cell, const int* nbr,
                              const double* sigma_t, const double* sigma_s, double* blk, int* col, int* bad,
                              hipStream_t st);
hipError_t launch_hp_spmv(int nn, int nthick, const double* blk, const int* col, const double* x, const double* b,
                          double* y, hipStream_t st);
hipError_t launch_hp_block_inverse(int nn, int nthick, const double* blk, double* binv, int* bad, hipStream_t st);
hipError_t launch_hp_block_apply(int nn, int nthick, const double* binv, const double* v, double* z, hipStream_t st);
hipError_t launch_hp_rhs(const HpTab& tb, int nthick, double hx, double hy, const int* thick_cell,
                         const double* sigma_t, const double* sigma_s, int mass_kind, const double* phi_old,
                         const double* phi_si, double* b, hipStream_t st);
hipError_t launch_hp_band(int nn, int nthick, const double* blk, const int* col, int kl, int ldb, double* band,
                          hipStream_t st);

namespace hp_detail {

using cplx = std::complex<double>;

// Solve A x = b (n <= kHpMaxN, complex) by Gaussian elimination with partial pivoting.
inline bool csolve(int n, cplx A[kHpMaxN][kHpMaxN], cplx b[kHpMaxN], cplx x[kHpMaxN]) {
    int perm[kHpMaxN] = {0, 1, 2, 3, 4};
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (std::abs(A[i][k]) > std::abs(A[p][k])) p = i;
        if (std::abs(A[p][k]) == 0.0) return false;
        if (p != k) {
            for (int j = 0; j < n; ++j) std::swap(A[k][j], A[p][j]);
            std::swap(b[k], b[p]);
            std::swap(perm[k], perm[p]);
        }
        for (int i = k + 1; i < n; ++i) {
            const cplx f = A[i][k] / A[k][k];
            for (int j = k; j < n; ++j) A[i][j] -= f * A[k][j];
            b[i] -= f * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        cplx s = b[i];
        for (int j = i + 1; j < n; ++j) s -= A[i][j] * x[j];
        x[i] = s / A[i][i];
    }
    return true;
}

// Lagrange polynomial k of `nodes` at x, and its derivative (product forms)
inline double lag(int n, const double* nodes, int k, double x) {
    double v = 1.0;
    for (int m = 0; m < n; ++m)
        if (m != k) v *= (x - nodes[m]) / (nodes[k] - nodes[m]);
    return v;
}
inline double dlag(int n, const double* nodes, int k, double x) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
        if (j == k) continue;
        double t = 1.0 / (nodes[k] - nodes[j]);
        for (int m = 0; m < n; ++m)
            if (m != k && m != j) t *= (x - nodes[m]) / (nodes[k] - nodes[m]);
        s += t;
    }
    return s;
}

}  // namespace hp_detail

// The tables of order p (2, 3 or 4).  Returns false if the eigenbasis check
// fails (||G V - V diag(lambda)|| or ||V V^{-1} - I|| above 1e-11).
inline bool hp_tables(int p, HpTab* tb) {
    using namespace hp_detail;
    const int n = p + 1;
    *tb = HpTab{};
    tb->p = p;
    double nodes[kHpMaxN];
    if (p == 2) {
        const double v[3] = {0.0, 0.5, 1.0};
        for (int i = 0; i < 3; ++i) nodes[i] = v[i];
    } else if (p == 3) {
        const double r = 0.5 / std::sqrt(5.0);   // roots of P_3' on [-1, 1] are +-1/sqrt5
        const double v[4] = {0.0, 0.5 - r, 0.5 + r, 1.0};
        for (int i = 0; i < 4; ++i) nodes[i] = v[i];
    } else if (p == 4) {
        const double r = 0.5 * std::sqrt(3.0 / 7.0);  // roots of P_4' on [-1, 1] are 0 and +-sqrt(3/7)
        const double v[5] = {0.0, 0.5 - r, 0.5, 0.5 + r, 1.0};
        for (int i = 0; i < 5; ++i) nodes[i] = v[i];
    } else {
        return false;
    }
    // Gauss-Legendre, 5 points on [0, 1] (exact to degree 9 >= 2p for p <= 4)
    const double gx[5] = {-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831, 0.9061798459386640};
    const double gw[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889, 0.4786286704993665,
                          0.2369268850561891};
    double D[kHpMaxN][kHpMaxN] = {};
    for (int g = 0; g < 5; ++g) {
        const double x = 0.5 * (gx[g] + 1.0), w = 0.5 * gw[g];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double li = lag(n, nodes, i, x), lj = lag(n, nodes, j, x);
                const double di = dlag(n, nodes, i, x), dj = dlag(n, nodes, j, x);
                tb->M[i][j] += w * li * lj;
                D[i][j] += w * li * dj;
                tb->K[i][j] += w * di * dj;
            }
    }
    for (int i = 0; i < n; ++i) {
        tb->dl0[i] = dlag(n, nodes, i, 0.0);
        tb->dl1[i] = dlag(n, nodes, i, 1.0);
    }
    // G = M^{-1} (D + e0 e0^T), c0 = M^{-1} e0
    double G[kHpMaxN][kHpMaxN];
    {
        cplx A[kHpMaxN][kHpMaxN], b[kHpMaxN], x[kHpMaxN];
        for (int col = 0; col <= n; ++col) {
            for (int i = 0; i < n; ++i) {
                for (int j = 0; j < n; ++j) A[i][j] = tb->M[i][j];
                b[i] = col < n ? D[i][col] + (i == 0 && col == 0 ? 1.0 : 0.0) : (i == 0 ? 1.0 : 0.0);
            }
            if (!csolve(n, A, b, x)) return false;
            for (int i = 0; i < n; ++i) {
                if (col < n) G[i][col] = x[i].real();
                else tb->c0[i] = x[i].real();
            }
        }
    }
    // characteristic polynomial det(z I - G) = sum_k a[k] z^k (Faddeev-LeVerrier)
    double a[kHpMaxN + 1] = {};
    {
        double Mk[kHpMaxN][kHpMaxN] = {}, T[kHpMaxN][kHpMaxN];
        a[n] = 1.0;
        for (int k = 1; k <= n; ++k) {
            // Mk = G M_{k-1} + a[n-k+1] I
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    double s = 0.0;
                    for (int m = 0; m < n; ++m) s += G[i][m] * Mk[m][j];
                    T[i][j] = s + (i == j ? a[n - k + 1] : 0.0);
                }
            double tr = 0.0;
            for (int i = 0; i < n; ++i)
                for (int m = 0; m < n; ++m) tr += G[i][m] * T[m][i];
            a[n - k] = -tr / k;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) Mk[i][j] = T[i][j];
        }
    }
    auto poly = [&](cplx z) {
        cplx v = a[n];
        for (int k = n - 1; k >= 0; --k) v = v * z + a[k];
        return v;
    };
    auto dpoly = [&](cplx z) {
        cplx v = double(n) * a[n];
        for (int k = n - 1; k >= 1; --k) v = v * z + double(k) * a[k];
        return v;
    };
    // roots: Durand-Kerner from distinct complex starts, then Newton polish
    cplx z[kHpMaxN];
    for (int i = 0; i < n; ++i) z[i] = std::pow(cplx(0.4, 0.9), i) * 3.0;
    for (int it = 0; it < 500; ++it) {
        for (int i = 0; i < n; ++i) {
            cplx den = 1.0;
            for (int j = 0; j < n; ++j)
                if (j != i) den *= (z[i] - z[j]);
            z[i] -= poly(z[i]) / den;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int it = 0; it < 3; ++it) {
            const cplx dp = dpoly(z[i]);
            if (std::abs(dp) > 0.0) z[i] -= poly(z[i]) / dp;
        }
    // eigenvectors by inverse iteration at a slightly shifted eigenvalue
    cplx V[kHpMaxN][kHpMaxN];
    for (int k = 0; k < n; ++k) {
        cplx v[kHpMaxN];
        for (int i = 0; i < n; ++i) v[i] = cplx(1.0 + 0.1 * i, 0.05 * i);
        const cplx mu = z[k] * (1.0 + 1e-9) + 1e-12;
        for (int it = 0; it < 3; ++it) {
            cplx A[kHpMaxN][kHpMaxN], x[kHpMaxN];
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) A[i][j] = (i == j ? G[i][j] - mu : cplx(G[i][j]));
            if (!csolve(n, A, v, x)) return false;
            double nrm = 0.0;
            for (int i = 0; i < n; ++i) nrm += std::norm(x[i]);
            nrm = std::sqrt(nrm);
            for (int i = 0; i < n; ++i) v[i] = x[i] / nrm;
        }
        for (int i = 0; i < n; ++i) V[i][k] = v[i];
    }
    // V^{-1} column by column
    cplx W[kHpMaxN][kHpMaxN];
    for (int col = 0; col < n; ++col) {
        cplx A[kHpMaxN][kHpMaxN], b[kHpMaxN], x[kHpMaxN];
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) A[i][j] = V[i][j];
            b[i] = i == col ? 1.0 : 0.0;
        }
        if (!csolve(n, A, b, x)) return false;
        for (int i = 0; i < n; ++i) W[i][col] = x[i];
    }
    // checks: G V = V Lambda and V W = I
    double gmax = 0.0, e1 = 0.0, e2 = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) gmax = std::max(gmax, std::fabs(G[i][j]));
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            cplx s = 0.0, t = 0.0;
            for (int m = 0; m < n; ++m) {
                s += G[i][m] * V[m][k];
                t += V[i][m] * W[m][k];
            }
            e1 = std::max(e1, std::abs(s - V[i][k] * z[k]));
            e2 = std::max(e2, std::abs(t - (i == k ? 1.0 : 0.0)));
        }
    if (!(e1 <= 1e-11 * gmax) || !(e2 <= 1e-11)) return false;
    for (int k = 0; k < n; ++k) {
        tb->lr[k] = z[k].real();
        tb->li[k] = z[k].imag();
        for (int i = 0; i < n; ++i) {
            tb->Vr[i][k] = V[i][k].real();
            tb->Vi[i][k] = V[i][k].imag();
            tb->Wr[k][i] = W[k][i].real();
            tb->Wi[k][i] = W[k][i].imag();
        }
    }
    return true;
}

}  // namespace sn
