// Upwind DG of order p = 2, 3 in 2D (Q_p on the Gauss-Lobatto nodes of each
// cell; Sec. 3.1 at the orders the paper runs in Sec. 4): the sweep with a
// fast-diagonalisation cell solve, the moment, and the thick diffusion
// matrices (SIP, NIP, mNIP) assembled as block-sparse rows.
//
// Cell solve.  Every direction is reflected into the frame where both of its
// components are positive (node index a -> p - a along a reflected axis; the
// 1D matrices satisfy P D P = -D for the reversal P, so the frame changes
// nothing else).  There the cell system times the inverse cell mass is
//   a_x G (x) I + a_y I (x) G + sigma_t I,   a = |Omega_axis| / h_axis,
// with G = M^{-1} (D + e_0 e_0^T) the 1D upwind operator on [0, 1]
// (M mass, D[i][j] = int l_i l_j').  G = V diag(lambda) V^{-1} with complex
// lambda of positive real part (the tables are computed once on the host),
// so the solve is two complex transforms and an elementwise division by
// a_x lambda_k + a_y lambda_l + sigma_t.  The right-hand side is the nodal
// source (sigma_s phi + q) / 4pi plus, for an inflow face, a_axis c0 (x) u_up
// with c0 = M^{-1} e_0 and u_up the upwind trace (the neighbour's face nodes).
//
// The sweep runs one workgroup per direction over the cell diagonals of its
// frame, a barrier between diagonals; neighbours' psi are read from memory
// written by the same workgroup before the barrier.
#include "../../include/sn.h"
#include "sn_kernels.hpp"
#include "hp.hpp"

namespace sn {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;  // 1 / (4 pi)

__device__ __forceinline__ int refl(int a, int r, int P) { return r ? P - a : a; }

template <int P>
__global__ void __launch_bounds__(256) sweep_hp_kernel(HpTab tb, int nx, int ny, int ndirs, long nbf,
                                                      const DirInfo* __restrict__ dirs,
                                                      const double* __restrict__ sigt,
                                                      const double* __restrict__ sigs,
                                                      const double* __restrict__ phi, const double* __restrict__ q,
                                                      const double* __restrict__ inflow, double* __restrict__ psi) {
    constexpr int N = P + 1, NN = N * N;
    const int d = blockIdx.x;
    const DirInfo di = dirs[d];
    const double ax = di.ax, ay = di.ay;
    const int rx = di.rx, ry = di.ry;
    for (int k = 0; k <= nx + ny - 2; ++k) {
        const int ilo = max(0, k - (ny - 1)), ihi = min(k, nx - 1);
        for (int ir = ilo + (int)threadIdx.x; ir <= ihi; ir += blockDim.x) {
            const int jr = k - ir;
            const int i = rx ? nx - 1 - ir : ir, j = ry ? ny - 1 - jr : jr;
            const long c = (long)j * nx + i;
            const double st = sigt[c], ss = sigs[c], qq = q ? q[c] : 0.0;
            double f[N][N];  // [a][b]: a along x, b along y, in the direction's frame
#pragma unroll
            for (int b = 0; b < N; ++b)
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    const int n = refl(a, rx, P) + N * refl(b, ry, P);
                    f[a][b] = (ss * (phi ? phi[c * NN + n] : 0.0) + qq) * kInv4Pi;
                }
            // x inflow face (a = 0 in the frame): the upwind values by b
#pragma unroll
            for (int b = 0; b < N; ++b) {
                const int bp = refl(b, ry, P);
                double up = 0.0;
                if (ir > 0) {
                    const long cn = c + (rx ? 1 : -1);
                    up = psi[(cn * ndirs + d) * NN + refl(P, rx, P) + N * bp];
                } else if (inflow) {
                    up = inflow[(long)d * nbf + (long)j * N + bp];
                }
#pragma unroll
                for (int a = 0; a < N; ++a) f[a][b] = fma(ax * tb.c0[a], up, f[a][b]);
            }
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const int apx = refl(a, rx, P);
                double up = 0.0;
                if (jr > 0) {
                    const long cn = c + (ry ? nx : -nx);
                    up = psi[(cn * ndirs + d) * NN + apx + N * refl(P, ry, P)];
                } else if (inflow) {
                    up = inflow[(long)d * nbf + (long)ny * N + (long)i * N + apx];
                }
#pragma unroll
                for (int b = 0; b < N; ++b) f[a][b] = fma(ay * tb.c0[b], up, f[a][b]);
            }
            // T[k][b] = sum_a W[k][a] f[a][b];  F[k][l] = sum_b W[l][b] T[k][b]
            double Tr[N][N], Ti[N][N];
#pragma unroll
            for (int kk = 0; kk < N; ++kk)
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    double sr = 0.0, si = 0.0;
#pragma unroll
                    for (int a = 0; a < N; ++a) {
                        sr = fma(tb.Wr[kk][a], f[a][b], sr);
                        si = fma(tb.Wi[kk][a], f[a][b], si);
                    }
                    Tr[kk][b] = sr;
                    Ti[kk][b] = si;
                }
            double Ur[N][N], Ui[N][N];
#pragma unroll
            for (int kk = 0; kk < N; ++kk)
#pragma unroll
                for (int l = 0; l < N; ++l) {
                    double sr = 0.0, si = 0.0;
#pragma unroll
                    for (int b = 0; b < N; ++b) {
                        sr = fma(tb.Wr[l][b], Tr[kk][b], sr);
                        sr = fma(-tb.Wi[l][b], Ti[kk][b], sr);
                        si = fma(tb.Wr[l][b], Ti[kk][b], si);
                        si = fma(tb.Wi[l][b], Tr[kk][b], si);
                    }
                    // divide by z = a_x lambda_k + a_y lambda_l + sigma_t
                    const double zr = ax * tb.lr[kk] + ay * tb.lr[l] + st;
                    const double zi = ax * tb.li[kk] + ay * tb.li[l];
                    const double inv = 1.0 / (zr * zr + zi * zi);
                    Ur[kk][l] = (sr * zr + si * zi) * inv;
                    Ui[kk][l] = (si * zr - sr * zi) * inv;
                }
            // T2[a][l] = sum_k V[a][k] U[k][l];  u[a][b] = Re sum_l V[b][l] T2[a][l]
#pragma unroll
            for (int a = 0; a < N; ++a) {
                double t2r[N], t2i[N];
#pragma unroll
                for (int l = 0; l < N; ++l) {
                    double sr = 0.0, si = 0.0;
#pragma unroll
                    for (int kk = 0; kk < N; ++kk) {
                        sr = fma(tb.Vr[a][kk], Ur[kk][l], sr);
                        sr = fma(-tb.Vi[a][kk], Ui[kk][l], sr);
                        si = fma(tb.Vr[a][kk], Ui[kk][l], si);
                        si = fma(tb.Vi[a][kk], Ur[kk][l], si);
                    }
                    t2r[l] = sr;
                    t2i[l] = si;
                }
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    double s = 0.0;
#pragma unroll
                    for (int l = 0; l < N; ++l) {
                        s = fma(tb.Vr[b][l], t2r[l], s);
                        s = fma(-tb.Vi[b][l], t2i[l], s);
                    }
                    psi[(c * ndirs + d) * NN + refl(a, rx, P) + N * refl(b, ry, P)] = s;
                }
            }
        }
        __syncthreads();
    }
}

// phi[c][n] = sum_d w_d psi[c][d][n], directions in index order
__global__ void __launch_bounds__(256) moment_hp_kernel(long nc, int ndirs, int nn, const double* __restrict__ w,
                                                       const double* __restrict__ psi, double* __restrict__ phi) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nc * nn; e += (long)gridDim.x * blockDim.x) {
        const long c = e / nn;
        const int n = (int)(e - c * nn);
        double s = 0.0;
        for (int d = 0; d < ndirs; ++d) s = fma(w[d], psi[(c * ndirs + d) * nn + n], s);
        phi[e] = s;
    }
}

// ---------------------------------------------------------------------------
// thick diffusion rows at order p (2D)
// ---------------------------------------------------------------------------
// Node of normal index a and tangential index t for a face normal to `ax`.
template <int N>
__device__ __forceinline__ int fnode(int ax, int a, int t) {
    return ax == 0 ? a + N * t : t + N * a;
}

__device__ __forceinline__ double mfac_hp(double cp, double sigma_t, double h) {
    const double f = cp / (sigma_t * h);
    return f > 1.0 ? f : 1.0;
}

// Rows of thick slot s: block 0 the cell's own, block 1 + 2 ax + sd the
// neighbour across face (ax, sd) (zero, column -1, when that neighbour is thin
// or absent).  blk: [nthick][5][NN][NN]; col: [nthick][5].  *bad is set for
// mNIP with sigma_t <= 0 at the cell or a face neighbour.
template <int P, int OP>
__global__ void __launch_bounds__(128) hp_assemble_kernel(HpTab tb, DsaGeom g, const int* __restrict__ thick_cell,
                                                         const int* __restrict__ nbr,
                                                         const double* __restrict__ sigma_t,
                                                         const double* __restrict__ sigma_s,
                                                         double* __restrict__ blk, int* __restrict__ col,
                                                         int* __restrict__ bad) {
    constexpr int N = P + 1, NN = N * N;
    const double cp = 0.1 * P * (P + 1);
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.nthick; s += gridDim.x * blockDim.x) {
        const long cell = thick_cell[s];
        const double stK = sigma_t[cell];
        const double DK = 1.0 / (3.0 * stK), sa = stK - sigma_s[cell];
        const double hx = g.h[0], hy = g.h[1];
        double* B0 = blk + (size_t)s * 5 * NN * NN;
        col[s * 5] = s;
        for (int r = 0; r < NN; ++r)
            for (int q = 0; q < NN; ++q) {
                const int ir = r % N, jr = r / N, iq = q % N, jq = q / N;
                B0[r * NN + q] = DK * (tb.K[ir][iq] / hx * hy * tb.M[jr][jq] + hx * tb.M[ir][iq] * tb.K[jr][jq] / hy) +
                                 sa * hx * hy * tb.M[ir][iq] * tb.M[jr][jq];
            }
        for (int ax = 0; ax < 2; ++ax)
            for (int sd = 0; sd < 2; ++sd) {
                const int b = 1 + 2 * ax + sd;
                double* Bn = blk + ((size_t)s * 5 + b) * NN * NN;
                for (int e = 0; e < NN * NN; ++e) Bn[e] = 0.0;
                const int ns = nbr[s * 4 + 2 * ax + sd];
                col[s * 5 + b] = ns >= 0 ? ns : -1;
                const double h = g.h[ax], ht = g.h[1 - ax];
                const int far = sd ? P : 0;          // this cell's face nodes (normal index)
                if (ns == -2) {                      // domain face
                    double kb = g.kappa0[ax];
                    if constexpr (OP == SN_DIFFUSION_MNIP) {
                        if (!(stK > 0.0)) *bad = 1;
                        kb *= mfac_hp(cp, stK, h);
                    }
                    for (int tr = 0; tr < N; ++tr)
                        for (int tq = 0; tq < N; ++tq)
                            B0[fnode<N>(ax, far, tr) * NN + fnode<N>(ax, far, tq)] += kb * ht * tb.M[tr][tq];
                    continue;
                }
                const long stride = ax == 0 ? 1 : g.nx;
                const long nbc = cell + (sd ? stride : -stride);
                const double stN = sigma_t[nbc];
                const double DN = ns >= 0 ? 1.0 / (3.0 * stN) : 0.0;
                const double sgr = sd ? 1.0 : -1.0;    // this cell's sign in [[u]] = u- - u+
                const double sgn = -sgr;
                const int fan = sd ? 0 : P;            // neighbour's face nodes
                const double* dlr = sd ? tb.dl1 : tb.dl0;
                const double* dln = sd ? tb.dl0 : tb.dl1;
                double kap = g.kappa0[ax];
                if constexpr (OP == SN_DIFFUSION_SIP) {
                    const double Dm = DK > DN ? DK : DN;
                    const double fl = 4.0 * P * (P + 1) * Dm / h;
                    if (fl > kap) kap = fl;
                } else if constexpr (OP == SN_DIFFUSION_MNIP) {
                    if (!(stK > 0.0) || !(stN > 0.0)) *bad = 1;
                    kap *= 0.5 * (mfac_hp(cp, stK, h) + mfac_hp(cp, stN, h));
                }
                const double sym = OP == SN_DIFFUSION_SIP ? 1.0 : 0.0;
                for (int tr = 0; tr < N; ++tr)
                    for (int tq = 0; tq < N; ++tq) {
                        const double F = ht * tb.M[tr][tq];
                        for (int ar = 0; ar < N; ++ar)
                            for (int aq = 0; aq < N; ++aq) {
                                const int r = fnode<N>(ax, ar, tr), q = fnode<N>(ax, aq, tq);
                                const double jr = ar == far ? sgr : 0.0;
                                // own columns
                                double v = -F * jr * 0.5 * DK * dlr[aq] / h;
                                v -= sym * F * 0.5 * DK * dlr[ar] / h * (aq == far ? sgr : 0.0);
                                v += kap * F * jr * (aq == far ? sgr : 0.0);
                                B0[r * NN + q] += v;
                                if (ns >= 0) {
                                    double u = -F * jr * 0.5 * DN * dln[aq] / h;
                                    u -= sym * F * 0.5 * DK * dlr[ar] / h * (aq == fan ? sgn : 0.0);
                                    u += kap * F * jr * (aq == fan ? sgn : 0.0);
                                    Bn[r * NN + q] = u;
                                }
                            }
                    }
            }
    }
}

// y = A x over the block rows (or y = b - A x with b given); thread per row
template <int NN>
__global__ void __launch_bounds__(256) hp_spmv_kernel(int nthick, const double* __restrict__ blk,
                                                     const int* __restrict__ col, const double* __restrict__ x,
                                                     const double* __restrict__ b, double* __restrict__ y) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)nthick * NN;
         e += (long)gridDim.x * blockDim.x) {
        const int s = (int)(e / NN), r = (int)(e - (long)s * NN);
        double v = 0.0;
        for (int k = 0; k < 5; ++k) {
            const int cs = col[s * 5 + k];
            if (cs < 0) continue;
            const double* B = blk + (((size_t)s * 5 + k) * NN + r) * NN;
            const double* xs = x + (size_t)cs * NN;
#pragma unroll
            for (int q = 0; q < NN; ++q) v = fma(B[q], xs[q], v);
        }
        y[e] = b ? b[e] - v : v;
    }
}

// full inverse of each diagonal block (Gauss-Jordan, partial pivoting), row
// major per slot; *bad = 1 on a zero pivot
template <int NN>
__global__ void __launch_bounds__(64) hp_block_inverse_kernel(int nthick, const double* __restrict__ blk,
                                                             double* __restrict__ binv, int* __restrict__ bad) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nthick; s += gridDim.x * blockDim.x) {
        double B[NN][NN], I[NN][NN];
        const double* D = blk + (size_t)s * 5 * NN * NN;
        for (int r = 0; r < NN; ++r)
            for (int c = 0; c < NN; ++c) {
                B[r][c] = D[r * NN + c];
                I[r][c] = r == c ? 1.0 : 0.0;
            }
        bool ok = true;
        for (int p = 0; p < NN && ok; ++p) {
            int pv = p;
            for (int r = p + 1; r < NN; ++r)
                if (fabs(B[r][p]) > fabs(B[pv][p])) pv = r;
            if (!(fabs(B[pv][p]) > 0.0)) {
                ok = false;
                break;
            }
            if (pv != p)
                for (int c = 0; c < NN; ++c) {
                    double t = B[p][c];
                    B[p][c] = B[pv][c];
                    B[pv][c] = t;
                    t = I[p][c];
                    I[p][c] = I[pv][c];
                    I[pv][c] = t;
                }
            const double ip = 1.0 / B[p][p];
            for (int c = 0; c < NN; ++c) {
                B[p][c] *= ip;
                I[p][c] *= ip;
            }
            for (int r = 0; r < NN; ++r) {
                if (r == p) continue;
                const double f = B[r][p];
                for (int c = 0; c < NN; ++c) {
                    B[r][c] -= f * B[p][c];
                    I[r][c] -= f * I[p][c];
                }
            }
        }
        if (!ok) *bad = 1;
        for (int r = 0; r < NN; ++r)
            for (int c = 0; c < NN; ++c) binv[((size_t)s * NN + r) * NN + c] = ok ? I[r][c] : 0.0;
    }
}

// z = Binv v, block by block
template <int NN>
__global__ void __launch_bounds__(256) hp_block_apply_kernel(int nthick, const double* __restrict__ binv,
                                                            const double* __restrict__ v, double* __restrict__ z) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)nthick * NN;
         e += (long)gridDim.x * blockDim.x) {
        const int s = (int)(e / NN), r = (int)(e - (long)s * NN);
        const double* B = binv + ((size_t)s * NN + r) * NN;
        const double* vs = v + (size_t)s * NN;
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < NN; ++q) a = fma(B[q], vs[q], a);
        z[e] = a;
    }
}

// b = coef M (phi_si - phi_old) on the thick cells (M the order-p cell mass)
template <int P>
__global__ void __launch_bounds__(256) hp_rhs_kernel(HpTab tb, int nthick, double hx, double hy,
                                                    const int* __restrict__ thick_cell,
                                                    const double* __restrict__ sigma_t,
                                                    const double* __restrict__ sigma_s, int mass_kind,
                                                    const double* __restrict__ phi_old,
                                                    const double* __restrict__ phi_si, double* __restrict__ b) {
    constexpr int N = P + 1, NN = N * N;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)nthick * NN;
         e += (long)gridDim.x * blockDim.x) {
        const int s = (int)(e / NN), r = (int)(e - (long)s * NN);
        const long c = thick_cell[s];
        const double coef = mass_kind == 1 ? sigma_t[c] : sigma_s[c];
        const int ir = r % N, jr = r / N;
        double v = 0.0;
        for (int q = 0; q < NN; ++q) {
            const int iq = q % N, jq = q / N;
            v = fma(hx * tb.M[ir][iq] * hy * tb.M[jr][jq], phi_si[c * NN + q] - phi_old[c * NN + q], v);
        }
        b[e] = coef * v;
    }
}

// band storage of the block rows (row i at band[i ldb + j - i + kl], zeroed before)
template <int NN>
__global__ void __launch_bounds__(256) hp_band_kernel(int nthick, const double* __restrict__ blk,
                                                     const int* __restrict__ col, int kl, int ldb,
                                                     double* __restrict__ band) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)nthick * NN;
         e += (long)gridDim.x * blockDim.x) {
        const int s = (int)(e / NN), r = (int)(e - (long)s * NN);
        for (int k = 0; k < 5; ++k) {
            const int cs = col[s * 5 + k];
            if (cs < 0) continue;
            const double* B = blk + (((size_t)s * 5 + k) * NN + r) * NN;
            for (int q = 0; q < NN; ++q) {
                const long j = (long)cs * NN + q;
                band[e * ldb + (j - e + kl)] = B[q];
            }
        }
    }
}

int blocks_of(long n, int bs) { return (int)std::max<long>(1, std::min<long>((n + bs - 1) / bs, 65536)); }

}  // namespace

hipError_t launch_sweep_hp(const HpTab& tb, int nx, int ny, int ndirs, long nbf, const DirInfo* dirs,
                           const double* sigt, const double* sigs, const double* phi, const double* q,
                           const double* inflow, double* psi, hipStream_t st) {
    const int threads = std::min(256, std::max(64, ((std::min(nx, ny) + 63) / 64) * 64));
    if (tb.p == 2)
        hipLaunchKernelGGL(sweep_hp_kernel<2>, dim3(ndirs), dim3(threads), 0, st, tb, nx, ny, ndirs, nbf, dirs, sigt,
                           sigs, phi, q, inflow, psi);
    else
        hipLaunchKernelGGL(sweep_hp_kernel<3>, dim3(ndirs), dim3(threads), 0, st, tb, nx, ny, ndirs, nbf, dirs, sigt,
                           sigs, phi, q, inflow, psi);
    return hipGetLastError();
}

hipError_t launch_moment_hp(long nc, int ndirs, int nn, const double* w, const double* psi, double* phi,
                            hipStream_t st) {
    hipLaunchKernelGGL(moment_hp_kernel, dim3(blocks_of(nc * nn, 256)), dim3(256), 0, st, nc, ndirs, nn, w, psi, phi);
    return hipGetLastError();
}

hipError_t launch_hp_assemble(const HpTab& tb, const DsaGeom& g, int op, const int* thick_cell, const int* nbr,
                              const double* sigma_t, const double* sigma_s, double* blk, int* col, int* bad,
                              hipStream_t st) {
    if (g.nthick == 0) return hipSuccess;
    const int nb = blocks_of(g.nthick, 128);
#define SN_HA(P, OP)                                                                                              \
    hipLaunchKernelGGL((hp_assemble_kernel<P, OP>), dim3(nb), dim3(128), 0, st, tb, g, thick_cell, nbr, sigma_t, \
                       sigma_s, blk, col, bad)
    if (tb.p == 2) {
        if (op == SN_DIFFUSION_SIP) SN_HA(2, SN_DIFFUSION_SIP);
        else if (op == SN_DIFFUSION_NIP) SN_HA(2, SN_DIFFUSION_NIP);
        else SN_HA(2, SN_DIFFUSION_MNIP);
    } else {
        if (op == SN_DIFFUSION_SIP) SN_HA(3, SN_DIFFUSION_SIP);
        else if (op == SN_DIFFUSION_NIP) SN_HA(3, SN_DIFFUSION_NIP);
        else SN_HA(3, SN_DIFFUSION_MNIP);
    }
#undef SN_HA
    return hipGetLastError();
}

hipError_t launch_hp_spmv(int nn, int nthick, const double* blk, const int* col, const double* x, const double* b,
                          double* y, hipStream_t st) {
    if (nthick == 0) return hipSuccess;
    const int nb = blocks_of((long)nthick * nn, 256);
    if (nn == 9)
        hipLaunchKernelGGL(hp_spmv_kernel<9>, dim3(nb), dim3(256), 0, st, nthick, blk, col, x, b, y);
    else
        hipLaunchKernelGGL(hp_spmv_kernel<16>, dim3(nb), dim3(256), 0, st, nthick, blk, col, x, b, y);
    return hipGetLastError();
}

hipError_t launch_hp_block_inverse(int nn, int nthick, const double* blk, double* binv, int* bad, hipStream_t st) {
    if (nthick == 0) return hipSuccess;
    const int nb = blocks_of(nthick, 64);
    if (nn == 9)
        hipLaunchKernelGGL(hp_block_inverse_kernel<9>, dim3(nb), dim3(64), 0, st, nthick, blk, binv, bad);
    else
        hipLaunchKernelGGL(hp_block_inverse_kernel<16>, dim3(nb), dim3(64), 0, st, nthick, blk, binv, bad);
    return hipGetLastError();
}

hipError_t launch_hp_block_apply(int nn, int nthick, const double* binv, const double* v, double* z, hipStream_t st) {
    if (nthick == 0) return hipSuccess;
    const int nb = blocks_of((long)nthick * nn, 256);
    if (nn == 9)
        hipLaunchKernelGGL(hp_block_apply_kernel<9>, dim3(nb), dim3(256), 0, st, nthick, binv, v, z);
    else
        hipLaunchKernelGGL(hp_block_apply_kernel<16>, dim3(nb), dim3(256), 0, st, nthick, binv, v, z);
    return hipGetLastError();
}

hipError_t launch_hp_rhs(const HpTab& tb, int nthick, double hx, double hy, const int* thick_cell,
                         const double* sigma_t, const double* sigma_s, int mass_kind, const double* phi_old,
                         const double* phi_si, double* b, hipStream_t st) {
    if (nthick == 0) return hipSuccess;
    const int nn = (tb.p + 1) * (tb.p + 1);
    const int nb = blocks_of((long)nthick * nn, 256);
    if (tb.p == 2)
        hipLaunchKernelGGL(hp_rhs_kernel<2>, dim3(nb), dim3(256), 0, st, tb, nthick, hx, hy, thick_cell, sigma_t,
                           sigma_s, mass_kind, phi_old, phi_si, b);
    else
        hipLaunchKernelGGL(hp_rhs_kernel<3>, dim3(nb), dim3(256), 0, st, tb, nthick, hx, hy, thick_cell, sigma_t,
                           sigma_s, mass_kind, phi_old, phi_si, b);
    return hipGetLastError();
}

hipError_t launch_hp_band(int nn, int nthick, const double* blk, const int* col, int kl, int ldb, double* band,
                          hipStream_t st) {
    if (nthick == 0) return hipSuccess;
    const int nb = blocks_of((long)nthick * nn, 256);
    if (nn == 9)
        hipLaunchKernelGGL(hp_band_kernel<9>, dim3(nb), dim3(256), 0, st, nthick, blk, col, kl, ldb, band);
    else
        hipLaunchKernelGGL(hp_band_kernel<16>, dim3(nb), dim3(256), 0, st, nthick, blk, col, kl, ldb, band);
    return hipGetLastError();
}

}  // namespace sn
