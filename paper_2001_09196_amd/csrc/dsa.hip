// Heterogeneous (thick-only) DSA, Alg. 2 of the paper, applied to the source-
// iteration residual:  phi <- phi_SI + P_T D_ff^{-1} Sigma_f R_T (phi_SI - phi).
//
// * Thick set (Sec. 2.3, Sec. 3.2): cell K is thick iff sigma_s,K >= eta; the
//   thick cells are compacted in increasing cell order by a deterministic scan.
// * D_ff: the SIP diffusion form (eq. SIP at eps = 1) restricted to the thick
//   DOFs (principal submatrix, Sec. 3.2), applied matrix-free:
//     cell:  D_K int grad u . grad v + sigma_a,K int u v,  D_K = 1/(3 sigma_t,K)
//     face (outward normal n of K, neighbour values zero if it is thin):
//       -int {D d_n u} v_K - 1/2 int (u_K - u_nb) D_K d_n v_K + kappa int (u_K - u_nb) v_K
//     domain face: kappa_0 int u v,  kappa_0 = (1/8pi) sum_d w_d |Omega_d . n|,
//     kappa = max(kappa_0, 8 max(D) / h) on interior faces.
// * Solver: conjugate gradients preconditioned by the inverse diagonal cell
//   blocks (block Jacobi), FP64 throughout, zero initial guess, stopping on
//   ||r|| <= rtol ||b||.  Scalars stay on the device: every dot product is a
//   fixed-order block reduction whose partials every consumer block re-reduces
//   in the same order, so results do not depend on scheduling.
#include "../../include/sn.h"
#include "sn_kernels.hpp"

namespace sn {

// ---------------------------------------------------------------------------
// thick classification and compaction
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) thick_flags_kernel(long nc, const double* __restrict__ sigma_s, double eta,
                                                          int* __restrict__ flags, int* __restrict__ block_sums) {
    __shared__ int sh[256];
    long c = (long)blockIdx.x * 256 + threadIdx.x;
    int f = (c < nc && sigma_s[c] >= eta) ? 1 : 0;
    if (c < nc) flags[c] = f;
    sh[threadIdx.x] = f;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = sh[0];
}

// exclusive scan of block_sums in place (one block); total -> *total
__global__ void __launch_bounds__(1024) thick_scan_kernel(int nblk, int* __restrict__ block_sums,
                                                          int* __restrict__ total) {
    __shared__ int sh[1024];
    const int per = (nblk + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    int loc = 0;
    for (int b = b0; b < min(nblk, b0 + per); ++b) loc += block_sums[b];
    sh[threadIdx.x] = loc;
    __syncthreads();
    // Hillis-Steele inclusive scan over 1024 partials
    for (int off = 1; off < 1024; off <<= 1) {
        int v = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    int run = threadIdx.x ? sh[threadIdx.x - 1] : 0;
    for (int b = b0; b < min(nblk, b0 + per); ++b) {
        int v = block_sums[b];
        block_sums[b] = run;
        run += v;
    }
    if (threadIdx.x == 1023) *total = sh[1023];
}

__global__ void __launch_bounds__(256) thick_scatter_kernel(long nc, const int* __restrict__ flags,
                                                            const int* __restrict__ block_sums,
                                                            int* __restrict__ slot_of_cell,
                                                            int* __restrict__ thick_cell) {
    __shared__ int sh[256];
    long c = (long)blockIdx.x * 256 + threadIdx.x;
    int f = c < nc ? flags[c] : 0;
    sh[threadIdx.x] = f;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int v = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    if (c < nc) {
        int slot = block_sums[blockIdx.x] + sh[threadIdx.x] - f;
        slot_of_cell[c] = f ? slot : -1;
        if (f) thick_cell[slot] = (int)c;
    }
}

hipError_t launch_thick_flags(long nc, const double* sigma_s, double eta, int* flags, int* block_sums, int nblk,
                              hipStream_t st) {
    hipLaunchKernelGGL(thick_flags_kernel, dim3(nblk), dim3(256), 0, st, nc, sigma_s, eta, flags, block_sums);
    return hipGetLastError();
}
hipError_t launch_thick_scan(int nblk, int* block_sums, int* total, hipStream_t st) {
    hipLaunchKernelGGL(thick_scan_kernel, dim3(1), dim3(1024), 0, st, nblk, block_sums, total);
    return hipGetLastError();
}
hipError_t launch_thick_scatter(long nc, const int* flags, const int* block_sums, int* slot_of_cell,
                                int* thick_cell, hipStream_t st) {
    int nblk = (int)((nc + 255) / 256);
    hipLaunchKernelGGL(thick_scatter_kernel, dim3(nblk), dim3(256), 0, st, nc, flags, block_sums, slot_of_cell,
                       thick_cell);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// matrix-free SIP on one thick cell
// ---------------------------------------------------------------------------
// 1D mass along `axis` of a tensor-product nodal vector (node bit `axis`)
template <int NN>
__device__ __forceinline__ void mass_along(double h, int axis, double t[NN]) {
    const int st = 1 << axis;
    const double a = h / 3.0, b = h / 6.0;
    double o[NN];
#pragma unroll
    for (int n = 0; n < NN; ++n) o[n] = a * t[n] + b * t[n ^ st];
#pragma unroll
    for (int n = 0; n < NN; ++n) t[n] = o[n];
}
template <int NN>
__device__ __forceinline__ void stiff_along(double h, int axis, double t[NN]) {
    const int st = 1 << axis;
    const double a = 1.0 / h;
    double o[NN];
#pragma unroll
    for (int n = 0; n < NN; ++n) o[n] = a * (t[n] - t[n ^ st]);
#pragma unroll
    for (int n = 0; n < NN; ++n) t[n] = o[n];
}

// out = rows of D_ff u belonging to thick cell `cell`, given its own values uK
// and the global thick vector u (indexed by slot); thin or missing neighbours
// contribute zero values.  With self_only the neighbour values are taken as
// zero, which yields the cell's diagonal block.
template <int NN>
__device__ void sip_cell_apply(const DsaGeom& g, long cell, const int* __restrict__ slot_of_cell,
                               const double* __restrict__ sigma_t, const double* __restrict__ sigma_s,
                               const double uK[NN], const double* __restrict__ u, bool self_only, double out[NN]) {
    constexpr int DIM = NN == 4 ? 2 : 3;
    const int i = (int)(cell % g.nx);
    const int j = (int)((cell / g.nx) % g.ny);
    const int k = (int)(cell / ((long)g.nx * g.ny));
    const double DK = 1.0 / (3.0 * sigma_t[cell]);
    const double sa = sigma_t[cell] - sigma_s[cell];
    // volume: D sum_axes (stiff_a (x) mass_others) u + sigma_a M u
#pragma unroll
    for (int n = 0; n < NN; ++n) out[n] = 0.0;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        double t[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) t[n] = uK[n];
#pragma unroll
        for (int o = 0; o < DIM; ++o) {
            if (o == ax) stiff_along<NN>(g.h[o], o, t);
            else mass_along<NN>(g.h[o], o, t);
        }
#pragma unroll
        for (int n = 0; n < NN; ++n) out[n] = fma(DK, t[n], out[n]);
    }
    {
        double t[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) t[n] = uK[n];
#pragma unroll
        for (int o = 0; o < DIM; ++o) mass_along<NN>(g.h[o], o, t);
#pragma unroll
        for (int n = 0; n < NN; ++n) out[n] = fma(sa, t[n], out[n]);
    }
    const int ext[3] = {g.nx, g.ny, g.nz};
    const int pos[3] = {i, j, k};
    const long stride[3] = {1, g.nx, (long)g.nx * g.ny};
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        const int st = 1 << ax;
        const double h = g.h[ax];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int npos = pos[ax] + (s ? 1 : -1);
            double t[NN];
            if (npos < 0 || npos >= ext[ax]) {
                // domain boundary: kappa_0 (face mass) u on the face nodes
#pragma unroll
                for (int n = 0; n < NN; ++n) t[n] = (((n >> ax) & 1) == s) ? uK[n] : 0.0;
#pragma unroll
                for (int o = 0; o < DIM; ++o)
                    if (o != ax) mass_along<NN>(g.h[o], o, t);
#pragma unroll
                for (int n = 0; n < NN; ++n)
                    if (((n >> ax) & 1) == s) out[n] = fma(g.kappa0[ax], t[n], out[n]);
                continue;
            }
            const long nb = cell + (s ? stride[ax] : -stride[ax]);
            const int nslot = slot_of_cell[nb];
            double un[NN];
            double Dn = 0.0;
#pragma unroll
            for (int n = 0; n < NN; ++n) un[n] = 0.0;
            if (nslot >= 0) {
                Dn = 1.0 / (3.0 * sigma_t[nb]);
                if (!self_only) {
#pragma unroll
                    for (int n = 0; n < NN; ++n) un[n] = u[(long)nslot * NN + n];
                }
            }
            double kap = g.kappa0[ax];
            const double Dmax = DK > Dn ? DK : Dn;
            if (8.0 * Dmax / h > kap) kap = 8.0 * Dmax / h;
            double J[NN], G[NN];
#pragma unroll
            for (int n = 0; n < NN; ++n) {
                if (((n >> ax) & 1) == s) {
                    J[n] = uK[n] - un[n ^ st];
                    G[n] = 0.5 * (DK * (uK[n] - uK[n ^ st]) + Dn * (un[n] - un[n ^ st])) / h;
                } else {
                    J[n] = 0.0;
                    G[n] = 0.0;
                }
            }
#pragma unroll
            for (int o = 0; o < DIM; ++o)
                if (o != ax) {
                    mass_along<NN>(g.h[o], o, J);
                    mass_along<NN>(g.h[o], o, G);
                }
            const double hd = 0.5 * DK / h;
#pragma unroll
            for (int n = 0; n < NN; ++n) {
                if (((n >> ax) & 1) == s) {
                    out[n] += -G[n] + kap * J[n] - hd * J[n];
                    out[n ^ st] += hd * J[n];
                }
            }
        }
    }
}

// neighbour table of each thick cell: for face f = 2*axis + side, the slot of
// the neighbour across that face, -1 for a thin neighbour, -2 at the domain
// boundary
template <int NN>
__global__ void neighbour_table_kernel(DsaGeom g, const int* __restrict__ thick_cell,
                                       const int* __restrict__ slot_of_cell, int* __restrict__ nbr) {
    constexpr int DIM = NN == 4 ? 2 : 3;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.nthick; s += gridDim.x * blockDim.x) {
        const long cell = thick_cell[s];
        const int pos[3] = {(int)(cell % g.nx), (int)((cell / g.nx) % g.ny), (int)(cell / ((long)g.nx * g.ny))};
        const int ext[3] = {g.nx, g.ny, g.nz};
        const long stride[3] = {1, g.nx, (long)g.nx * g.ny};
        for (int ax = 0; ax < DIM; ++ax)
            for (int sd = 0; sd < 2; ++sd) {
                const int np = pos[ax] + (sd ? 1 : -1);
                int v = -2;
                if (np >= 0 && np < ext[ax]) v = slot_of_cell[cell + (sd ? stride[ax] : -stride[ax])];
                nbr[s * 2 * DIM + 2 * ax + sd] = v < 0 ? (np >= 0 && np < ext[ax] ? -1 : -2) : v;
            }
    }
}

hipError_t launch_neighbour_table(const DsaGeom& g, const int* thick_cell, const int* slot_of_cell, int* nbr,
                                  hipStream_t st) {
    if (g.nthick == 0) return hipSuccess;
    int blocks = std::min((g.nthick + 255) / 256, 65536);
    if (g.nn == 4)
        hipLaunchKernelGGL(neighbour_table_kernel<4>, dim3(blocks), dim3(256), 0, st, g, thick_cell, slot_of_cell, nbr);
    else
        hipLaunchKernelGGL(neighbour_table_kernel<8>, dim3(blocks), dim3(256), 0, st, g, thick_cell, slot_of_cell, nbr);
    return hipGetLastError();
}

// mNIP penalty factor of one side of a face (eq. ModifiedF0 with linear
// elements: c(p) = 0.1 p (p + 1) = 0.2), h the cell size across the face
__device__ __forceinline__ double mnip_factor(double sigma_t, double h) {
    const double f = 0.2 / (sigma_t * h);
    return f > 1.0 ? f : 1.0;
}

// Rows of D_ff u for thick cell `cell` (slot s) with the neighbour values
// supplied by get(nslot, un) -- the same bilinear form as sip_cell_apply,
// reading neighbours through the neighbour table.  OP selects the form of
// Sec. 3.1: SN_DIFFUSION_SIP (eq. SIP), SN_DIFFUSION_NIP (eq. NIP: the term
// -int [[u]]{D dv/dn} dropped, penalty kappa_0 without the 8 D/h floor) or
// SN_DIFFUSION_MNIP (NIP with the penalty of eq. ModifiedF0: kappa_0 times the
// mean of the two sides' factors, the thin side's sigma_t included; on a
// domain face the cell's own factor).
template <int NN, int OP = SN_DIFFUSION_SIP, typename Get>
__device__ __forceinline__ void sip_rows(const DsaGeom& g, int s, long cell, const int* __restrict__ nbr,
                                         const int* __restrict__ thick_cell, const double* __restrict__ sigma_t,
                                         const double* __restrict__ sigma_s, const double uK[NN], Get get,
                                         double out[NN]) {
    constexpr int DIM = NN == 4 ? 2 : 3;
    const double DK = 1.0 / (3.0 * sigma_t[cell]);
    const double sa = sigma_t[cell] - sigma_s[cell];
#pragma unroll
    for (int n = 0; n < NN; ++n) out[n] = 0.0;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        double t[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) t[n] = uK[n];
#pragma unroll
        for (int o = 0; o < DIM; ++o) {
            if (o == ax) stiff_along<NN>(g.h[o], o, t);
            else mass_along<NN>(g.h[o], o, t);
        }
#pragma unroll
        for (int n = 0; n < NN; ++n) out[n] = fma(DK, t[n], out[n]);
    }
    {
        double t[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) t[n] = uK[n];
#pragma unroll
        for (int o = 0; o < DIM; ++o) mass_along<NN>(g.h[o], o, t);
#pragma unroll
        for (int n = 0; n < NN; ++n) out[n] = fma(sa, t[n], out[n]);
    }
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        const int st = 1 << ax;
        const double h = g.h[ax];
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            const int ns = nbr[s * 2 * DIM + 2 * ax + sd];
            double t[NN];
            if (ns == -2) {
#pragma unroll
                for (int n = 0; n < NN; ++n) t[n] = (((n >> ax) & 1) == sd) ? uK[n] : 0.0;
#pragma unroll
                for (int o = 0; o < DIM; ++o)
                    if (o != ax) mass_along<NN>(g.h[o], o, t);
                double kb = g.kappa0[ax];
                if constexpr (OP == SN_DIFFUSION_MNIP) kb *= mnip_factor(sigma_t[cell], h);
#pragma unroll
                for (int n = 0; n < NN; ++n)
                    if (((n >> ax) & 1) == sd) out[n] = fma(kb, t[n], out[n]);
                continue;
            }
            double un[NN];
            double Dn = 0.0;
#pragma unroll
            for (int n = 0; n < NN; ++n) un[n] = 0.0;
            if (ns >= 0) {
                Dn = 1.0 / (3.0 * sigma_t[thick_cell[ns]]);
                get(ns, un);
            }
            double kap = g.kappa0[ax];
            if constexpr (OP == SN_DIFFUSION_SIP) {
                const double Dmax = DK > Dn ? DK : Dn;
                if (8.0 * Dmax / h > kap) kap = 8.0 * Dmax / h;
            } else if constexpr (OP == SN_DIFFUSION_MNIP) {
                const long stride = ax == 0 ? 1L : ax == 1 ? (long)g.nx : (long)g.nx * g.ny;
                const long nb = cell + (sd ? stride : -stride);
                kap *= 0.5 * (mnip_factor(sigma_t[cell], h) + mnip_factor(sigma_t[nb], h));
            }
            double J[NN], G[NN];
#pragma unroll
            for (int n = 0; n < NN; ++n) {
                if (((n >> ax) & 1) == sd) {
                    J[n] = uK[n] - un[n ^ st];
                    G[n] = 0.5 * (DK * (uK[n] - uK[n ^ st]) + Dn * (un[n] - un[n ^ st])) / h;
                } else {
                    J[n] = 0.0;
                    G[n] = 0.0;
                }
            }
#pragma unroll
            for (int o = 0; o < DIM; ++o)
                if (o != ax) {
                    mass_along<NN>(g.h[o], o, J);
                    mass_along<NN>(g.h[o], o, G);
                }
            if constexpr (OP == SN_DIFFUSION_SIP) {
                const double hd = 0.5 * DK / h;
#pragma unroll
                for (int n = 0; n < NN; ++n) {
                    if (((n >> ax) & 1) == sd) {
                        out[n] += -G[n] + kap * J[n] - hd * J[n];
                        out[n ^ st] += hd * J[n];
                    }
                }
            } else {
#pragma unroll
                for (int n = 0; n < NN; ++n)
                    if (((n >> ax) & 1) == sd) out[n] += -G[n] + kap * J[n];
            }
        }
    }
}

// diagonal block of D_ff for each thick cell, inverted (Gauss-Jordan; the
// block is symmetric positive definite, so no pivoting is needed)
template <int NN>
__global__ void block_jacobi_kernel(DsaGeom g, const int* __restrict__ thick_cell,
                                    const int* __restrict__ slot_of_cell, const double* __restrict__ sigma_t,
                                    const double* __restrict__ sigma_s, double* __restrict__ binv) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.nthick; s += gridDim.x * blockDim.x) {
        const long cell = thick_cell[s];
        double B[NN][NN], Inv[NN][NN];
        for (int c = 0; c < NN; ++c) {
            double e[NN], col[NN];
            for (int n = 0; n < NN; ++n) e[n] = (n == c) ? 1.0 : 0.0;
            sip_cell_apply<NN>(g, cell, slot_of_cell, sigma_t, sigma_s, e, nullptr, true, col);
            for (int n = 0; n < NN; ++n) B[n][c] = col[n];
        }
        for (int r = 0; r < NN; ++r)
            for (int c = 0; c < NN; ++c) Inv[r][c] = (r == c) ? 1.0 : 0.0;
        for (int p = 0; p < NN; ++p) {
            const double ip = 1.0 / B[p][p];
            for (int c = 0; c < NN; ++c) {
                B[p][c] *= ip;
                Inv[p][c] *= ip;
            }
            for (int r = 0; r < NN; ++r) {
                if (r == p) continue;
                const double f = B[r][p];
                for (int c = 0; c < NN; ++c) {
                    B[r][c] -= f * B[p][c];
                    Inv[r][c] -= f * Inv[p][c];
                }
            }
        }
        // the inverse of a symmetric block is symmetric: its upper triangle,
        // row by row, with the two rounded copies of each off-diagonal entry
        // averaged
        int k = 0;
        for (int r = 0; r < NN; ++r)
            for (int c = r; c < NN; ++c, ++k)
                binv[(long)k * g.nthick + s] = c == r ? Inv[r][r] : 0.5 * (Inv[r][c] + Inv[c][r]);
    }
}

hipError_t launch_block_jacobi(const DsaGeom& g, const int* thick_cell, const int* slot_of_cell,
                               const double* sigma_t, const double* sigma_s, double* binv, hipStream_t st) {
    if (g.nthick == 0) return hipSuccess;
    int blocks = std::min((g.nthick + 127) / 128, 65536);
    if (g.nn == 4)
        hipLaunchKernelGGL(block_jacobi_kernel<4>, dim3(blocks), dim3(128), 0, st, g, thick_cell, slot_of_cell,
                           sigma_t, sigma_s, binv);
    else
        hipLaunchKernelGGL(block_jacobi_kernel<8>, dim3(blocks), dim3(128), 0, st, g, thick_cell, slot_of_cell,
                           sigma_t, sigma_s, binv);
    return hipGetLastError();
}

template <int NN>
__global__ void __launch_bounds__(256) sip_apply_kernel(DsaGeom g, const int* __restrict__ thick_cell, const int* __restrict__ slot_of_cell,
                                 const double* __restrict__ sigma_t, const double* __restrict__ sigma_s,
                                 const double* __restrict__ u, double* __restrict__ y) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.nthick; s += gridDim.x * blockDim.x) {
        double uK[NN], o[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) uK[n] = u[(long)s * NN + n];
        sip_cell_apply<NN>(g, thick_cell[s], slot_of_cell, sigma_t, sigma_s, uK, u, false, o);
#pragma unroll
        for (int n = 0; n < NN; ++n) y[(long)s * NN + n] = o[n];
    }
}

hipError_t launch_sip_apply(const DsaGeom& g, const int* thick_cell, const int* slot_of_cell,
                            const double* sigma_t, const double* sigma_s, const double* u, double* y,
                            hipStream_t st) {
    if (g.nthick == 0) return hipSuccess;
    int blocks = std::min((g.nthick + 255) / 256, 65536);
    if (g.nn == 4)
        hipLaunchKernelGGL(sip_apply_kernel<4>, dim3(blocks), dim3(256), 0, st, g, thick_cell, slot_of_cell, sigma_t,
                           sigma_s, u, y);
    else
        hipLaunchKernelGGL(sip_apply_kernel<8>, dim3(blocks), dim3(256), 0, st, g, thick_cell, slot_of_cell, sigma_t,
                           sigma_s, u, y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// preconditioned CG
// ---------------------------------------------------------------------------
// deterministic block sum (sh: at least 16 doubles): the wave sums, then the
// waves in wave order
__device__ __forceinline__ double block_reduce(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
    for (int k = 1; k < nw; ++k) r += sh[k];
    __syncthreads();
    return r;
}

// every block re-reduces the same partial array in the same order
__device__ __forceinline__ double reduce_parts(const double* __restrict__ part, int nparts, double* sh) {
    double v = 0.0;
    for (int e = threadIdx.x; e < nparts; e += 256) v += part[e];
    return block_reduce(v, sh);
}

// z = B r for a symmetric block B given by its upper triangle, row by row
// (bj_entries<NN>() values); get(k) returns entry k
template <int NN, typename Get>
__device__ __forceinline__ void sym_apply(Get get, const double r[NN], double z[NN]) {
#pragma unroll
    for (int a = 0; a < NN; ++a) z[a] = 0.0;
    int k = 0;
#pragma unroll
    for (int a = 0; a < NN; ++a) {
#pragma unroll
        for (int b = a; b < NN; ++b, ++k) {
            const double v = get(k);
            z[a] = fma(v, r[b], z[a]);
            if (b != a) z[b] = fma(v, r[a], z[b]);
        }
    }
}

template <int NN>
__device__ __forceinline__ void bj_apply(const double* __restrict__ binv, long bj_stride, int s, const double r[NN],
                                         double z[NN]) {
    // element-major storage: entry k of the blocks of all thick cells is
    // contiguous, so consecutive lanes (cells) read consecutive words; only
    // the upper triangle is stored (the inverse of the symmetric block is
    // symmetric), 36 of 64 words per cell in 3D
    const long n = bj_stride;
    sym_apply<NN>([&](int k) { return binv[(long)k * n + s]; }, r, z);
}

// right-hand side of thick slot s: b = coef M (phi_si - phi_old)
template <int NN>
__device__ __forceinline__ void dsa_rhs_at(const DsaGeom& g, const int* __restrict__ thick_cell,
                                           const double* __restrict__ sigma_t, const double* __restrict__ sigma_s,
                                           int mass_kind, const double* __restrict__ phi_old,
                                           const double* __restrict__ phi_si, int s, double t[NN]) {
    constexpr int DIM = NN == 4 ? 2 : 3;
    const long c = thick_cell[s];
    const double coef = mass_kind == 1 ? sigma_t[c] : sigma_s[c];
#pragma unroll
    for (int n = 0; n < NN; ++n) t[n] = phi_si[c * NN + n] - phi_old[c * NN + n];
#pragma unroll
    for (int o = 0; o < DIM; ++o) mass_along<NN>(g.h[o], o, t);
#pragma unroll
    for (int n = 0; n < NN; ++n) t[n] *= coef;
}

// ---------------------------------------------------------------------------
// the nonsymmetric forms (NIP, mNIP): operator pieces of the GMRES inner solve
// ---------------------------------------------------------------------------
// Full inverse of each thick cell's diagonal block (Gauss-Jordan with partial
// pivoting: the NIP block is not symmetric and need not be definite), stored
// element-major, entry r NN + c of all cells contiguous.  Sets *bad to 1 for
// a singular block, and for mNIP when a thick cell or a face neighbour has
// sigma_t <= 0 (eq. ModifiedF0 divides by it).
template <int NN, int OP>
__global__ void __launch_bounds__(128) block_inverse_full_kernel(DsaGeom g, const int* __restrict__ thick_cell,
                                                                 const int* __restrict__ nbr,
                                                                 const double* __restrict__ sigma_t,
                                                                 const double* __restrict__ sigma_s,
                                                                 double* __restrict__ binv, int* __restrict__ bad) {
    constexpr int DIM = NN == 4 ? 2 : 3;
    auto zero = [](int, double o[NN]) {
        for (int n = 0; n < NN; ++n) o[n] = 0.0;
    };
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.nthick; s += gridDim.x * blockDim.x) {
        const long cell = thick_cell[s];
        bool ok = true;
        if constexpr (OP == SN_DIFFUSION_MNIP) {
            ok = sigma_t[cell] > 0.0;
            const long stride[3] = {1, g.nx, (long)g.nx * g.ny};
            for (int f = 0; f < 2 * DIM; ++f)
                if (nbr[s * 2 * DIM + f] != -2) ok = ok && sigma_t[cell + ((f & 1) ? stride[f >> 1] : -stride[f >> 1])] > 0.0;
        }
        double B[NN][NN], Inv[NN][NN];
        for (int c = 0; c < NN; ++c) {
            double e[NN], col[NN];
            for (int n = 0; n < NN; ++n) e[n] = (n == c) ? 1.0 : 0.0;
            sip_rows<NN, OP>(g, s, cell, nbr, thick_cell, sigma_t, sigma_s, e, zero, col);
            for (int n = 0; n < NN; ++n) B[n][c] = col[n];
        }
        for (int r = 0; r < NN; ++r)
            for (int c = 0; c < NN; ++c) Inv[r][c] = (r == c) ? 1.0 : 0.0;
        for (int p = 0; p < NN && ok; ++p) {
            int piv = p;
            for (int r = p + 1; r < NN; ++r)
                if (fabs(B[r][p]) > fabs(B[piv][p])) piv = r;
            if (!(fabs(B[piv][p]) > 0.0)) {
                ok = false;
                break;
            }
            if (piv != p)
                for (int c = 0; c < NN; ++c) {
                    const double a = B[p][c], b = Inv[p][c];
                    B[p][c] = B[piv][c];
                    Inv[p][c] = Inv[piv][c];
                    B[piv][c] = a;
                    Inv[piv][c] = b;
                }
            const double ip = 1.0 / B[p][p];
            for (int c = 0; c < NN; ++c) {
                B[p][c] *= ip;
                Inv[p][c] *= ip;
            }
            for (int r = 0; r < NN; ++r) {
                if (r == p) continue;
                const double f = B[r][p];
                for (int c = 0; c < NN; ++c) {
                    B[r][c] -= f * B[p][c];
                    Inv[r][c] -= f * Inv[p][c];
                }
            }
        }
        if (!ok) *bad = 1;
        for (int r = 0; r < NN; ++r)
            for (int c = 0; c < NN; ++c) binv[(long)(r * NN + c) * g.nthick + s] = ok ? Inv[r][c] : 0.0;
    }
}

template <int NN>
__device__ __forceinline__ void full_block_apply(const double* __restrict__ binv, int nthick, int s,
                                                 const double* __restrict__ v, double z[NN]) {
    double vv[NN];
#pragma unroll
    for (int n = 0; n < NN; ++n) vv[n] = v[(long)s * NN + n];
#pragma unroll
    for (int r = 0; r < NN; ++r) {
        double a = 0.0;
#pragma unroll
        for (int c = 0; c < NN; ++c) a = fma(binv[(long)(r * NN + c) * nthick + s], vv[c], a);
        z[r] = a;
    }
}

// w = D_ff B^{-1} v (right-preconditioned operator; the neighbours' B^{-1} v
// are formed on the fly), or with b given the residual w = b - D_ff B^{-1} v;
// binv = nullptr: B = I
template <int NN, int OP>
__global__ void __launch_bounds__(256) nip_apply_kernel(DsaGeom g, const int* __restrict__ thick_cell,
                                                        const int* __restrict__ nbr,
                                                        const double* __restrict__ sigma_t,
                                                        const double* __restrict__ sigma_s,
                                                        const double* __restrict__ binv,
                                                        const double* __restrict__ v, const double* __restrict__ b,
                                                        double* __restrict__ w) {
    auto get = [&](int slot, double out[NN]) {
        if (binv) {
            full_block_apply<NN>(binv, g.nthick, slot, v, out);
        } else {
#pragma unroll
            for (int n = 0; n < NN; ++n) out[n] = v[(long)slot * NN + n];
        }
    };
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < g.nthick; t += gridDim.x * blockDim.x) {
        double uK[NN], o[NN];
        get(t, uK);
        sip_rows<NN, OP>(g, t, thick_cell[t], nbr, thick_cell, sigma_t, sigma_s, uK, get, o);
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            const long e = (long)t * NN + n;
            w[e] = b ? b[e] - o[n] : o[n];
        }
    }
}

// x = B^{-1} u
template <int NN>
__global__ void __launch_bounds__(256) full_block_apply_kernel(int nthick, const double* __restrict__ binv,
                                                               const double* __restrict__ u,
                                                               double* __restrict__ x) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nthick; t += gridDim.x * blockDim.x) {
        double z[NN];
        full_block_apply<NN>(binv, nthick, t, u, z);
#pragma unroll
        for (int n = 0; n < NN; ++n) x[(long)t * NN + n] = z[n];
    }
}

// b = coef M (phi_si - phi_old) on the thick cells, as a thick vector
template <int NN>
__global__ void __launch_bounds__(256) dsa_rhs_vec_kernel(DsaGeom g, const int* __restrict__ thick_cell,
                                                          const double* __restrict__ sigma_t,
                                                          const double* __restrict__ sigma_s, int mass_kind,
                                                          const double* __restrict__ phi_old,
                                                          const double* __restrict__ phi_si, double* __restrict__ b) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.nthick; s += gridDim.x * blockDim.x) {
        double t[NN];
        dsa_rhs_at<NN>(g, thick_cell, sigma_t, sigma_s, mass_kind, phi_old, phi_si, s, t);
#pragma unroll
        for (int n = 0; n < NN; ++n) b[(long)s * NN + n] = t[n];
    }
}

static int grid_of(int n, int bs) { return std::max(1, std::min((n + bs - 1) / bs, 65536)); }

hipError_t launch_block_inverse_full(const DsaGeom& g, int op, const int* thick_cell, const int* nbr,
                                     const double* sigma_t, const double* sigma_s, double* binv, int* bad,
                                     hipStream_t st) {
    if (g.nthick == 0) return hipSuccess;
    const int blocks = grid_of(g.nthick, 128);
#define SN_BIF(NN, OP)                                                                                      \
    hipLaunchKernelGGL((block_inverse_full_kernel<NN, OP>), dim3(blocks), dim3(128), 0, st, g, thick_cell, nbr, \
                       sigma_t, sigma_s, binv, bad)
    if (g.nn == 4) {
        if (op == SN_DIFFUSION_MNIP) SN_BIF(4, SN_DIFFUSION_MNIP);
        else SN_BIF(4, SN_DIFFUSION_NIP);
    } else {
        if (op == SN_DIFFUSION_MNIP) SN_BIF(8, SN_DIFFUSION_MNIP);
        else SN_BIF(8, SN_DIFFUSION_NIP);
    }
#undef SN_BIF
    return hipGetLastError();
}

hipError_t launch_nip_apply(const DsaGeom& g, int op, const int* thick_cell, const int* nbr, const double* sigma_t,
                            const double* sigma_s, const double* binv, const double* v, const double* b, double* w,
                            hipStream_t st) {
    if (g.nthick == 0) return hipSuccess;
    const int blocks = grid_of(g.nthick, 256);
#define SN_NA(NN, OP)                                                                                          \
    hipLaunchKernelGGL((nip_apply_kernel<NN, OP>), dim3(blocks), dim3(256), 0, st, g, thick_cell, nbr, sigma_t, \
                       sigma_s, binv, v, b, w)
    if (g.nn == 4) {
        if (op == SN_DIFFUSION_MNIP) SN_NA(4, SN_DIFFUSION_MNIP);
        else SN_NA(4, SN_DIFFUSION_NIP);
    } else {
        if (op == SN_DIFFUSION_MNIP) SN_NA(8, SN_DIFFUSION_MNIP);
        else SN_NA(8, SN_DIFFUSION_NIP);
    }
#undef SN_NA
    return hipGetLastError();
}

hipError_t launch_full_block_apply(const DsaGeom& g, const double* binv, const double* u, double* x, hipStream_t st) {
    if (g.nthick == 0) return hipSuccess;
    const int blocks = grid_of(g.nthick, 256);
    if (g.nn == 4)
        hipLaunchKernelGGL(full_block_apply_kernel<4>, dim3(blocks), dim3(256), 0, st, g.nthick, binv, u, x);
    else
        hipLaunchKernelGGL(full_block_apply_kernel<8>, dim3(blocks), dim3(256), 0, st, g.nthick, binv, u, x);
    return hipGetLastError();
}

hipError_t launch_dsa_rhs_vec(const DsaGeom& g, const int* thick_cell, const double* sigma_t, const double* sigma_s,
                              int mass_kind, const double* phi_old, const double* phi_si, double* b, hipStream_t st) {
    if (g.nthick == 0) return hipSuccess;
    const int blocks = grid_of(g.nthick, 256);
    if (g.nn == 4)
        hipLaunchKernelGGL(dsa_rhs_vec_kernel<4>, dim3(blocks), dim3(256), 0, st, g, thick_cell, sigma_t, sigma_s,
                           mass_kind, phi_old, phi_si, b);
    else
        hipLaunchKernelGGL(dsa_rhs_vec_kernel<8>, dim3(blocks), dim3(256), 0, st, g, thick_cell, sigma_t, sigma_s,
                           mass_kind, phi_old, phi_si, b);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exact thick solve for small systems: band LU with partial pivoting
// ---------------------------------------------------------------------------
// The thick matrix in band storage, row i holding columns i - kl .. i + kl + ku
// at lu[i ldb + j - i + kl] (the extra kl columns take the fill of the row
// swaps).  Each thick cell writes its rows: the diagonal block and the blocks
// of its thick face neighbours, one column at a time, by applying the form
// to unit vectors.
template <int NN, int OP>
__global__ void __launch_bounds__(128) band_assemble_kernel(DsaGeom g, const int* __restrict__ thick_cell,
                                                            const int* __restrict__ nbr,
                                                            const double* __restrict__ sigma_t,
                                                            const double* __restrict__ sigma_s, int kl, int ldb,
                                                            double* __restrict__ lu) {
    constexpr int DIM = NN == 4 ? 2 : 3;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.nthick; s += gridDim.x * blockDim.x) {
        const long cell = thick_cell[s];
        for (int f = -1; f < 2 * DIM; ++f) {
            const int t = f < 0 ? s : nbr[s * 2 * DIM + f];
            if (t < 0) continue;
            for (int c = 0; c < NN; ++c) {
                double uK[NN], col[NN];
                for (int n = 0; n < NN; ++n) uK[n] = (f < 0 && n == c) ? 1.0 : 0.0;
                auto unit = [&](int slot, double o[NN]) {
                    for (int n = 0; n < NN; ++n) o[n] = (f >= 0 && slot == t && n == c) ? 1.0 : 0.0;
                };
                sip_rows<NN, OP>(g, s, cell, nbr, thick_cell, sigma_t, sigma_s, uK, unit, col);
                for (int r = 0; r < NN; ++r) {
                    const long i = (long)s * NN + r, j = (long)t * NN + c;
                    lu[i * ldb + (j - i + kl)] = col[r];
                }
            }
        }
    }
}

// largest slot distance to a thick face neighbour (the band's half width in cells)
template <int NN>
__global__ void __launch_bounds__(256) band_width_kernel(DsaGeom g, const int* __restrict__ nbr, int* __restrict__ w) {
    constexpr int DIM = NN == 4 ? 2 : 3;
    int m = 0;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.nthick; s += gridDim.x * blockDim.x)
        for (int f = 0; f < 2 * DIM; ++f) {
            const int t = nbr[s * 2 * DIM + f];
            if (t >= 0) m = max(m, abs(t - s));
        }
    atomicMax(w, m);
}

// In-place band LU with partial pivoting by one workgroup: column k's pivot
// is the entry of largest magnitude among rows k .. k + kl (the first such
// row on ties); rows k and p are swapped over columns k .. k + kl + ku, the
// multipliers stored below the diagonal, and the trailing band block updated.
// The phases of a column are separated by workgroup barriers, which also
// order the global-memory accesses of the workgroup's waves.  *bad = 1 on a
// zero pivot (the factorisation then stops).
constexpr int kBandThreads = 1024;
__global__ void __launch_bounds__(kBandThreads) band_factor_kernel(long n, int kl, int ku, int ldb,
                                                                   double* __restrict__ lu, int* __restrict__ piv,
                                                                   int* __restrict__ bad) {
    __shared__ double sv[kBandThreads / 64];
    __shared__ long si[kBandThreads / 64];
    __shared__ long sp;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    auto at = [&](long i, long j) -> double& { return lu[i * ldb + (j - i + kl)]; };
    for (long k = 0; k < n; ++k) {
        const long last = min(n - 1, k + (long)kl), jend = min(n - 1, k + (long)kl + ku);
        double best = -1.0;
        long bi = k;
        for (long i = k + t; i <= last; i += kBandThreads) {
            const double v = fabs(at(i, k));
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(best, off);
            const long oi = __shfl_xor(bi, off);
            if (ov > best || (ov == best && oi < bi)) {
                best = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            sv[wv] = best;
            si[wv] = bi;
        }
        __syncthreads();
        if (t == 0) {
            double b = sv[0];
            long p = si[0];
            for (int q = 1; q < kBandThreads / 64; ++q)
                if (sv[q] > b || (sv[q] == b && si[q] < p)) {
                    b = sv[q];
                    p = si[q];
                }
            sp = b > 0.0 ? p : -1;
            piv[k] = (int)(b > 0.0 ? p : k);
            if (!(b > 0.0)) *bad = 1;
        }
        __syncthreads();
        const long p = sp;
        if (p < 0) return;
        if (p != k)
            for (long j = k + t; j <= jend; j += kBandThreads) {
                const double a = at(k, j);
                at(k, j) = at(p, j);
                at(p, j) = a;
            }
        __syncthreads();
        const double inv = 1.0 / at(k, k);
        for (long i = k + 1 + t; i <= last; i += kBandThreads) at(i, k) *= inv;
        __syncthreads();
        const long R = last - k, C = jend - k;
        for (long e = t; e < R * C; e += kBandThreads) {
            const long i = k + 1 + e / C, j = k + 1 + e % C;
            at(i, j) = fma(-at(i, k), at(k, j), at(i, j));
        }
        __syncthreads();
    }
}

// x = D^{-1} b from the band factors by one workgroup, the vector in LDS
// (n <= kBandMaxN): forward elimination with the row swaps in factorisation
// order, then back substitution by columns.  Each thread loads its factor
// entry of the next column ahead of the barrier.
constexpr int kBandMaxN = 8192;
__global__ void __launch_bounds__(kBandThreads) band_solve_kernel(long n, int kl, int ku, int ldb,
                                                                  const double* __restrict__ lu,
                                                                  const int* __restrict__ piv,
                                                                  const double* __restrict__ b,
                                                                  double* __restrict__ x) {
    __shared__ double xs[kBandMaxN];
    const int t = threadIdx.x;
    auto at = [&](long i, long j) { return lu[i * ldb + (j - i + kl)]; };
    for (long i = t; i < n; i += kBandThreads) xs[i] = b[i];
    __syncthreads();
    // forward: rows k + 1 .. k + kl of column k; thread t takes row k + 1 + t
    // (kl < kBandThreads: one row per thread)
    double lnext = (1 + t < n && t < kl) ? at(1 + t, 0) : 0.0;
    for (long k = 0; k < n; ++k) {
        if (t == 0) {
            const long p = piv[k];
            if (p != k) {
                const double a = xs[k];
                xs[k] = xs[p];
                xs[p] = a;
            }
        }
        const double l = lnext;
        const long i = k + 1 + t;
        lnext = (i + 1 < n && t < kl) ? at(i + 1, k + 1) : 0.0;
        __syncthreads();
        if (t < kl && i < n) xs[i] = fma(-l, xs[k], xs[i]);
        __syncthreads();
    }
    // backward: x_i = xs_i / U_ii, then rows i - kl - ku .. i - 1 of column i
    const int w = kl + ku;
    double unext = (n - 2 - t >= 0 && t < w) ? at(n - 2 - t, n - 1) : 0.0;
    double dnext = at(n - 1, n - 1);
    for (long i = n - 1; i >= 0; --i) {
        const double u = unext, d = dnext;
        const long j = i - 1 - t;
        unext = (j - 1 >= 0 && t < w && i >= 1) ? at(j - 1, i - 1) : 0.0;
        dnext = i >= 1 ? at(i - 1, i - 1) : 0.0;
        const double xi = xs[i] / d;
        __syncthreads();
        if (t == 0) xs[i] = xi;
        if (t < w && j >= 0) xs[j] = fma(-u, xi, xs[j]);
        __syncthreads();
    }
    for (long i = t; i < n; i += kBandThreads) x[i] = xs[i];
}

hipError_t launch_band_width(const DsaGeom& g, const int* nbr, int* w, hipStream_t st) {
    if (g.nthick == 0) return hipSuccess;
    const int blocks = grid_of(g.nthick, 256);
    if (g.nn == 4) hipLaunchKernelGGL(band_width_kernel<4>, dim3(blocks), dim3(256), 0, st, g, nbr, w);
    else hipLaunchKernelGGL(band_width_kernel<8>, dim3(blocks), dim3(256), 0, st, g, nbr, w);
    return hipGetLastError();
}

hipError_t launch_band_assemble(const DsaGeom& g, int op, const int* thick_cell, const int* nbr,
                                const double* sigma_t, const double* sigma_s, int kl, int ldb, double* lu,
                                hipStream_t st) {
    if (g.nthick == 0) return hipSuccess;
    const int blocks = grid_of(g.nthick, 128);
#define SN_BA(NN, OP)                                                                                         \
    hipLaunchKernelGGL((band_assemble_kernel<NN, OP>), dim3(blocks), dim3(128), 0, st, g, thick_cell, nbr, sigma_t, \
                       sigma_s, kl, ldb, lu)
    if (g.nn == 4) {
        if (op == SN_DIFFUSION_SIP) SN_BA(4, SN_DIFFUSION_SIP);
        else if (op == SN_DIFFUSION_NIP) SN_BA(4, SN_DIFFUSION_NIP);
        else SN_BA(4, SN_DIFFUSION_MNIP);
    } else {
        if (op == SN_DIFFUSION_SIP) SN_BA(8, SN_DIFFUSION_SIP);
        else if (op == SN_DIFFUSION_NIP) SN_BA(8, SN_DIFFUSION_NIP);
        else SN_BA(8, SN_DIFFUSION_MNIP);
    }
#undef SN_BA
    return hipGetLastError();
}

hipError_t launch_band_factor(long n, int kl, int ku, int ldb, double* lu, int* piv, int* bad, hipStream_t st) {
    hipLaunchKernelGGL(band_factor_kernel, dim3(1), dim3(kBandThreads), 0, st, n, kl, ku, ldb, lu, piv, bad);
    return hipGetLastError();
}

hipError_t launch_band_solve(long n, int kl, int ku, int ldb, const double* lu, const int* piv, const double* b,
                             double* x, hipStream_t st) {
    hipLaunchKernelGGL(band_solve_kernel, dim3(1), dim3(kBandThreads), 0, st, n, kl, ku, ldb, lu, piv, b, x);
    return hipGetLastError();
}

// Warm start of the CG from the previous solution x_p (one-dimensional
// Galerkin projection: x0 = alpha x_p with alpha = x_p.b / x_p.D x_p, which
// never increases the D-norm error of the zero start): w = D x_p and the
// partials x_p.b [0..nparts), x_p.w [nparts..2 nparts).
template <int NN>
__global__ void __launch_bounds__(256) dsa_warm_kernel(DsaGeom g, const int* __restrict__ thick_cell,
                                                       const int* __restrict__ nbr,
                                                       const double* __restrict__ sigma_t,
                                                       const double* __restrict__ sigma_s, int mass_kind,
                                                       const double* __restrict__ phi_old,
                                                       const double* __restrict__ phi_si,
                                                       const double* __restrict__ xp, double* __restrict__ w,
                                                       double* __restrict__ part) {
    __shared__ double sh[16];
    auto get = [&](int slot, double out[NN]) {
#pragma unroll
        for (int n = 0; n < NN; ++n) out[n] = xp[(long)slot * NN + n];
    };
    double xb = 0.0, xw = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < g.nthick; t += gridDim.x * blockDim.x) {
        double b[NN], xK[NN], o[NN];
        dsa_rhs_at<NN>(g, thick_cell, sigma_t, sigma_s, mass_kind, phi_old, phi_si, t, b);
        get(t, xK);
        sip_rows<NN>(g, t, thick_cell[t], nbr, thick_cell, sigma_t, sigma_s, xK, get, o);
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            w[(long)t * NN + n] = o[n];
            xb = fma(xK[n], b[n], xb);
            xw = fma(xK[n], o[n], xw);
        }
    }
    xb = block_reduce(xb, sh);
    xw = block_reduce(xw, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = xb;
        part[gridDim.x + blockIdx.x] = xw;
    }
}

// b = coef M (phi_si - phi_old) on thick cells; x = 0 and r = b, or with a
// warm start (wpart != nullptr, partials of dsa_warm_kernel) x = alpha x and
// r = b - alpha w; p = 0.  With the block-Jacobi preconditioner (bj = 1) also
// z = B^{-1} r and the r.z partials [0..nparts); r.r partials go to
// [nparts..2 nparts), b.b partials to [2 nparts..3 nparts).  With the
// multigrid preconditioner the V-cycle produces z and the r.z partials.
// Block 0 also resets the CG scalars and, given res_part, reduces the
// source-iteration residual partials into res_out (device) and res_host
// (pinned host memory).
template <int NN, bool BJ>
__global__ void __launch_bounds__(256) dsa_rhs_kernel(DsaGeom g, const int* __restrict__ thick_cell,
                                                      const double* __restrict__ sigma_t,
                                                      const double* __restrict__ sigma_s, int mass_kind,
                                                      const double* __restrict__ phi_old,
                                                      const double* __restrict__ phi_si,
                                                      const double* __restrict__ binv, double* __restrict__ x,
                                                      double* __restrict__ r, double* __restrict__ z,
                                                      double* __restrict__ p, double* __restrict__ part,
                                                      CgScalars* sc, const double* __restrict__ res_part,
                                                      int res_nparts,
                                                      double* __restrict__ res_out, double* __restrict__ res_host,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ wpart) {
    __shared__ double sh[48];
    double alpha = 0.0;
    if (wpart) {
        const double xb = reduce_parts(wpart, gridDim.x, sh);
        const double xw = reduce_parts(wpart + gridDim.x, gridDim.x, sh);
        alpha = xw > 0.0 ? xb / xw : 0.0;
    }
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            sc->rz[0] = sc->rz[1] = 0.0;
            sc->bb = sc->rr = 0.0;
            sc->iters = 0;
            sc->breakdown = 0;
            sc->done = 0;
        }
        if (res_part) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int e = threadIdx.x; e < res_nparts; e += 256) {
                s0 += res_part[e];
                s1 += res_part[res_nparts + e];
                s2 += res_part[2 * res_nparts + e];
            }
            block_sum3(s0, s1, s2, sh);
            if (threadIdx.x == 0) {
                res_out[0] = s0;
                res_out[1] = s1;
                res_out[2] = s2;
                res_host[0] = s0;
                res_host[1] = s1;
                res_host[2] = s2;
            }
            __syncthreads();
        }
    }
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.nthick; s += gridDim.x * blockDim.x) {
        double b[NN], t[NN], zz[NN];
        dsa_rhs_at<NN>(g, thick_cell, sigma_t, sigma_s, mass_kind, phi_old, phi_si, s, b);
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            const long e = (long)s * NN + n;
            if (wpart) {
                t[n] = fma(-alpha, w[e], b[n]);
                x[e] = alpha * x[e];
            } else {
                t[n] = b[n];
                x[e] = 0.0;
            }
        }
        if constexpr (BJ) bj_apply<NN>(binv, g.nthick, s, t, zz);
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            const long e = (long)s * NN + n;
            r[e] = t[n];
            p[e] = 0.0;
            if constexpr (BJ) {
                z[e] = zz[n];
                rz = fma(t[n], zz[n], rz);
            }
            rr = fma(t[n], t[n], rr);
            bb = fma(b[n], b[n], bb);
        }
    }
    rz = block_reduce(rz, sh);
    rr = block_reduce(rr, sh);
    bb = block_reduce(bb, sh);
    if (threadIdx.x == 0) {
        if constexpr (BJ) part[blockIdx.x] = rz;
        part[gridDim.x + blockIdx.x] = rr;
        part[2 * gridDim.x + blockIdx.x] = bb;
    }
}

hipError_t launch_dsa_warm(const DsaGeom& g, const int* thick_cell, const int* nbr, const double* sigma_t,
                           const double* sigma_s, int mass_kind, const double* phi_old, const double* phi_si,
                           const double* xp, double* w, double* part, int nparts, hipStream_t st) {
    if (g.nn == 4)
        hipLaunchKernelGGL(dsa_warm_kernel<4>, dim3(nparts), dim3(256), 0, st, g, thick_cell, nbr, sigma_t, sigma_s,
                           mass_kind, phi_old, phi_si, xp, w, part);
    else
        hipLaunchKernelGGL(dsa_warm_kernel<8>, dim3(nparts), dim3(256), 0, st, g, thick_cell, nbr, sigma_t, sigma_s,
                           mass_kind, phi_old, phi_si, xp, w, part);
    return hipGetLastError();
}

hipError_t launch_dsa_rhs(const DsaGeom& g, const int* thick_cell, const double* sigma_t, const double* sigma_s,
                          int mass_kind, const double* phi_old, const double* phi_si, const double* binv,
                          double* x, double* r, double* z, double* p, double* part, int nparts, int bj,
                          CgScalars* s, const double* res_part, int res_nparts, double* res_out, double* res_host,
                          const double* w, const double* wpart, hipStream_t st) {
#define SN_RHS(NN, BJ)                                                                                        \
    hipLaunchKernelGGL((dsa_rhs_kernel<NN, BJ>), dim3(nparts), dim3(256), 0, st, g, thick_cell, sigma_t, sigma_s, \
                       mass_kind, phi_old, phi_si, binv, x, r, z, p, part, s, res_part, res_nparts,              \
                       res_out, res_host, w, wpart)
    if (g.nn == 4) {
        if (bj) SN_RHS(4, true);
        else SN_RHS(4, false);
    } else {
        if (bj) SN_RHS(8, true);
        else SN_RHS(8, false);
    }
#undef SN_RHS
    return hipGetLastError();
}

// Two kernels per CG iteration `it`:
//   apply:  every block reduces the r.z / r.r partials of the previous update
//           (of the right-hand-side kernel at it = 0) and stops the solve when
//           ||r|| <= rtol ||b|| or it = maxit; otherwise
//           beta = rz_it / rz_{it-1} (0 at it = 0), p = z + beta p_old for its
//           own and its neighbours' DOFs (on the fly: z and p_old are complete
//           from the previous iteration), q = A p, partials p.q.
//   update: alpha = rz_it / p.q; x += alpha p; r -= alpha q; z = B^{-1} r;
//           partials r.z, r.r.
// p alternates between two buffers (read p_old, write p) so that neighbours
// never see a half-updated direction.  Block 0 of the apply kernel stores
// rz_it in slot it&1 while the other blocks read slot (it-1)&1.
template <int NN>
__global__ void __launch_bounds__(256) cg_apply_kernel(DsaGeom g, const int* __restrict__ thick_cell,
                                                       const int* __restrict__ nbr,
                                                       const double* __restrict__ sigma_t,
                                                       const double* __restrict__ sigma_s,
                                                       const double* __restrict__ z, const double* __restrict__ p_old,
                                                       double* __restrict__ p_new, double* __restrict__ q,
                                                       const double* __restrict__ part_rz, double* __restrict__ part,
                                                       int nparts, CgScalars* s, CgScalars* s_host, double rtol,
                                                       int maxit, int it) {
    if (s->done) return;
    __shared__ double sh[16];
    const double rz = reduce_parts(part_rz, nparts, sh);
    const double rr = reduce_parts(part_rz + nparts, nparts, sh);
    const double bb = it == 0 ? reduce_parts(part_rz + 2 * nparts, nparts, sh) : s->bb;
    if (sqrt(rr) <= rtol * sqrt(bb) || it >= maxit || bb == 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            s->bb = bb;
            s->rr = rr;
            s->iters = it;
            s->done = 1;
            if (s_host) {
                s_host->bb = bb;
                s_host->rr = rr;
                s_host->iters = it;
                __threadfence_system();  // the fields reach the host before the flag
                s_host->done = 1;
            }
        }
        return;
    }
    const double beta = it == 0 ? 0.0 : rz / s->rz[(it + 1) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s->rz[it & 1] = rz;
        s->rr = rr;
        if (it == 0) s->bb = bb;
    }
    auto pdir = [&](int slot, double out[NN]) {
#pragma unroll
        for (int n = 0; n < NN; ++n) out[n] = fma(beta, p_old[(long)slot * NN + n], z[(long)slot * NN + n]);
    };
    double pq = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < g.nthick; t += gridDim.x * blockDim.x) {
        double uK[NN], o[NN];
        pdir(t, uK);
        sip_rows<NN>(g, t, thick_cell[t], nbr, thick_cell, sigma_t, sigma_s, uK, pdir, o);
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            p_new[(long)t * NN + n] = uK[n];
            q[(long)t * NN + n] = o[n];
            pq = fma(uK[n], o[n], pq);
        }
    }
    pq = block_reduce(pq, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = pq;
}

template <int NN, bool BJ>
__global__ void __launch_bounds__(256) cg_update_kernel(DsaGeom g, const double* __restrict__ binv,
                                                        double* __restrict__ x, double* __restrict__ r,
                                                        double* __restrict__ z, const double* __restrict__ p,
                                                        const double* __restrict__ q,
                                                        const double* __restrict__ part_pq,
                                                        double* __restrict__ part_out, int nparts, CgScalars* s,
                                                        CgScalars* s_host, int it) {
    if (s->done) return;
    __shared__ double sh[16];
    // The first cell's operands are loaded before the reduction of the
    // partials, whose barriers also order memory accesses, so that the loads
    // overlap it (the C2 thick set has one cell per thread); in 2D the
    // block inverse too.
    constexpr int NB = NN == 4 ? bj_entries<NN>() : 1;
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    double x0[NN], p0[NN], q0[NN], r0[NN], b0[NB];
    if (t0 < g.nthick) {
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            const long e = (long)t0 * NN + n;
            x0[n] = x[e];
            p0[n] = p[e];
            q0[n] = q[e];
            r0[n] = r[e];
        }
        if constexpr (BJ && NN == 4) {
#pragma unroll
            for (int k = 0; k < NB; ++k) b0[k] = binv[(long)k * g.nthick + t0];
        }
    }
    const double pq = reduce_parts(part_pq, nparts, sh);
    if (!(pq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            s->breakdown = 1;
            s->iters = it;
            s->done = 1;
            if (s_host) {
                s_host->bb = s->bb;
                s_host->rr = s->rr;
                s_host->breakdown = 1;
                s_host->iters = it;
                __threadfence_system();
                s_host->done = 1;
            }
        }
        return;
    }
    const double alpha = s->rz[it & 1] / pq;
    double rz = 0.0, rr = 0.0;
    auto cell = [&](int t, const double xv[NN], const double pv[NN], const double qv[NN], const double rin[NN],
                    bool pre) {
        double rv[NN], zv[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            const long e = (long)t * NN + n;
            x[e] = fma(alpha, pv[n], xv[n]);
            rv[n] = fma(-alpha, qv[n], rin[n]);
            r[e] = rv[n];
        }
        if constexpr (BJ) {
            if constexpr (NN == 4) {
                if (pre) {
                    sym_apply<NN>([&](int k) { return b0[k]; }, rv, zv);
                } else {
                    bj_apply<NN>(binv, g.nthick, t, rv, zv);
                }
            } else {
                bj_apply<NN>(binv, g.nthick, t, rv, zv);
            }
#pragma unroll
            for (int n = 0; n < NN; ++n) {
                z[(long)t * NN + n] = zv[n];
                rz = fma(rv[n], zv[n], rz);
                rr = fma(rv[n], rv[n], rr);
            }
        } else {
#pragma unroll
            for (int n = 0; n < NN; ++n) rr = fma(rv[n], rv[n], rr);
        }
    };
    if (t0 < g.nthick) cell(t0, x0, p0, q0, r0, true);
    for (int t = t0 + stride; t < g.nthick; t += stride) {
        double xv[NN], pv[NN], qv[NN], rin[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            const long e = (long)t * NN + n;
            xv[n] = x[e];
            pv[n] = p[e];
            qv[n] = q[e];
            rin[n] = r[e];
        }
        cell(t, xv, pv, qv, rin, false);
    }
    rz = block_reduce(rz, sh);
    rr = block_reduce(rr, sh);
    if (threadIdx.x == 0) {
        if constexpr (BJ) part_out[blockIdx.x] = rz;
        part_out[gridDim.x + blockIdx.x] = rr;
    }
}

// apply kernel of iteration it (its stop test first; with it = maxit only the
// test); p alternates between p0 and p1 by iteration parity
hipError_t launch_cg_apply(const DsaGeom& g, const int* thick_cell, const int* nbr, const double* sigma_t,
                           const double* sigma_s, const double* z, double* p0, double* p1, double* q,
                           double* part_a, double* part_b, int nparts, CgScalars* s, CgScalars* s_host, double rtol,
                           int maxit, int it, hipStream_t st) {
    double* p_old = (it & 1) ? p1 : p0;
    double* p_new = (it & 1) ? p0 : p1;
    if (g.nn == 4)
        hipLaunchKernelGGL(cg_apply_kernel<4>, dim3(nparts), dim3(256), 0, st, g, thick_cell, nbr, sigma_t, sigma_s,
                           z, p_old, p_new, q, part_b, part_a, nparts, s, s_host, rtol, maxit, it);
    else
        hipLaunchKernelGGL(cg_apply_kernel<8>, dim3(nparts), dim3(256), 0, st, g, thick_cell, nbr, sigma_t, sigma_s,
                           z, p_old, p_new, q, part_b, part_a, nparts, s, s_host, rtol, maxit, it);
    return hipGetLastError();
}

// The stop test of iteration it, ahead of the multigrid V-cycle that would
// give its z: the same test, on the same partials reduced in the same order,
// as the apply kernel of iteration it makes first (so the decision is the
// same), but before the V-cycle, whose kernels and that apply then return at
// once when it passes.  it >= 1, so ||b||^2 is already in s.
__global__ void __launch_bounds__(256) cg_test_kernel(const double* __restrict__ part_rr, int nparts, CgScalars* s,
                                                      CgScalars* s_host, double rtol, int maxit, int it) {
    if (s->done) return;
    __shared__ double sh[16];
    const double rr = reduce_parts(part_rr, nparts, sh);
    const double bb = s->bb;
    if (sqrt(rr) <= rtol * sqrt(bb) || it >= maxit || bb == 0.0) {
        if (threadIdx.x == 0) {
            s->rr = rr;
            s->iters = it;
            s->done = 1;
            if (s_host) {
                s_host->bb = bb;
                s_host->rr = rr;
                s_host->iters = it;
                __threadfence_system();  // the fields reach the host before the flag
                s_host->done = 1;
            }
        }
    }
}

hipError_t launch_cg_test(const double* part_b, int nparts, CgScalars* s, CgScalars* s_host, double rtol,
                          int maxit, int it, hipStream_t st) {
    hipLaunchKernelGGL(cg_test_kernel, dim3(1), dim3(256), 0, st, part_b + nparts, nparts, s, s_host, rtol, maxit,
                       it);
    return hipGetLastError();
}

// update kernel of iteration it (< maxit)
hipError_t launch_cg_update(const DsaGeom& g, const double* binv, double* x, double* r, double* z, double* p0,
                            double* p1, const double* q, double* part_a, double* part_b, int nparts, CgScalars* s,
                            CgScalars* s_host, int it, int bj, hipStream_t st) {
    double* p_new = (it & 1) ? p0 : p1;
#define SN_UPD(NN, BJ)                                                                                       \
    hipLaunchKernelGGL((cg_update_kernel<NN, BJ>), dim3(nparts), dim3(256), 0, st, g, binv, x, r, z, p_new, q, \
                       part_a, part_b, nparts, s, s_host, it)
    if (g.nn == 4) {
        if (bj) SN_UPD(4, true);
        else SN_UPD(4, false);
    } else {
        if (bj) SN_UPD(8, true);
        else SN_UPD(8, false);
    }
#undef SN_UPD
    return hipGetLastError();
}

__global__ void dsa_scatter_kernel(long n, int nn, const int* __restrict__ slot_of_cell,
                                   const double* __restrict__ phi_si, const double* __restrict__ x,
                                   double* __restrict__ phi_out) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const long c = e / nn;
        const int s = slot_of_cell ? slot_of_cell[c] : -1;
        double v = phi_si[e];
        if (s >= 0) v += x[(long)s * nn + (e - c * nn)];
        phi_out[e] = v;
    }
}

hipError_t launch_dsa_scatter(long nc, int nn, const int* slot_of_cell, const double* phi_si, const double* x,
                              double* phi_out, hipStream_t st) {
    long n = nc * nn;
    int blocks = (int)std::min<long>((n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(dsa_scatter_kernel, dim3(blocks), dim3(256), 0, st, n, nn, slot_of_cell, phi_si, x, phi_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// geometric multigrid preconditioner for D_ff
// ---------------------------------------------------------------------------
// Level 0 is the Q1-DG SIP system on the thick cells.  In thick cells the
// face penalty (kappa_0 ~ 1/4) is far larger than D/h, so the low-energy
// functions of D_ff are continuous: level 1 is the continuous Q1 space on the
// vertices of the thick cells (prolongation = the vertex value copied to the
// DG nodes at that vertex), and its operator is the Galerkin product
// P^T D_ff P, a 3^dim-point vertex stencil, evaluated by applying D_ff to
// colourings of the vertices (mod 3 per axis).  Levels 2.. coarsen the vertex
// grid by two with (bi/tri)linear interpolation and Galerkin operators (built
// on the host); the last level is solved with a dense inverse.  One
// symmetric V-cycle: damped block Jacobi on level 0 and damped Jacobi on the
// vertex levels, once before and once after the coarse-grid correction.

// colour of a vertex: (i mod 3) + 3 (j mod 3) + 9 (k mod 3)
__device__ __forceinline__ int vtx_colour(int i, int j, int k) { return i % 3 + 3 * (j % 3) + 9 * (k % 3); }

// x0 = P (indicator of the vertices of colour col) on the DG nodes
template <int NN>
__global__ void vmg_probe_fill_kernel(DsaGeom g, const int* __restrict__ thick_cell, int col,
                                      double* __restrict__ x0) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.nthick; s += gridDim.x * blockDim.x) {
        const long cell = thick_cell[s];
        const int i = (int)(cell % g.nx), j = (int)((cell / g.nx) % g.ny), k = (int)(cell / ((long)g.nx * g.ny));
        for (int n = 0; n < NN; ++n)
            x0[(long)s * NN + n] = vtx_colour(i + (n & 1), j + ((n >> 1) & 1), k + ((n >> 2) & 1)) == col ? 1.0 : 0.0;
    }
}

// coef1[w][o] = (P^T D_ff P)(w, w + o) for the neighbour w + o of colour col:
// the sum of y0 = D_ff x0 over the DG nodes at vertex w
__global__ void vmg_probe_gather_kernel(MgDev m, int nvx, int nvy, const long* __restrict__ vpos, int col,
                                        const double* __restrict__ y0, double* __restrict__ coef) {
    const int nch = 1 << m.dim;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < m.n[1]; w += gridDim.x * blockDim.x) {
        const long p = vpos[w];
        const int c[3] = {(int)(p % nvx), (int)((p / nvx) % nvy), (int)(p / ((long)nvx * nvy))};
        const int cc[3] = {col % 3, (col / 3) % 3, col / 9};
        int idx = 0, mul = 1;
        for (int d = 0; d < m.dim; ++d) {
            const int delta = (cc[d] - c[d] % 3 + 3) % 3;   // 0 -> 0, 1 -> +1, 2 -> -1
            const int o = delta == 2 ? -1 : delta;
            idx += (o + 1) * mul;
            mul *= 3;
        }
        double v = 0.0;
        for (int q = 0; q < nch; ++q) {
            const int e = m.vnodes[(long)q * m.n[1] + w];
            if (e >= 0) v += y0[e];
        }
        coef[(long)w * m.ns + idx] = v;
    }
}

hipError_t launch_vmg_probe(const DsaGeom& g, const int* thick_cell, const int* slot_of_cell,
                            const double* sigma_t, const double* sigma_s, const MgDev& m, int nvx, int nvy,
                            const long* vpos, double* x0, double* y0, double* coef, hipStream_t st) {
    if (g.nthick == 0) return hipSuccess;
    const int ncol = g.dim == 2 ? 9 : 27;
    const int bt = std::min((g.nthick + 255) / 256, 65536), bv = std::min((m.n[1] + 255) / 256, 65536);
    for (int col = 0; col < ncol; ++col) {
        if (g.nn == 4)
            hipLaunchKernelGGL(vmg_probe_fill_kernel<4>, dim3(bt), dim3(256), 0, st, g, thick_cell, col, x0);
        else
            hipLaunchKernelGGL(vmg_probe_fill_kernel<8>, dim3(bt), dim3(256), 0, st, g, thick_cell, col, x0);
        hipError_t e = launch_sip_apply(g, thick_cell, slot_of_cell, sigma_t, sigma_s, x0, y0, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(vmg_probe_gather_kernel, dim3(bv), dim3(256), 0, st, m, nvx, nvy, vpos, col, y0, coef);
    }
    return hipGetLastError();
}

// (A_l v)[f] for vertex level l
__device__ __forceinline__ double vmg_apply_at(const MgDev& m, int l, int f, const double* __restrict__ v) {
    // per-level arrays are offset-major ([o][unknown]): for a fixed offset,
    // consecutive lanes read consecutive words
    const long n = m.n[l];
    const double* c = m.coef + m.so[l] + f;
    const int* nb = m.nbr + m.so[l] + f;
    double a = 0.0;
    for (int o = 0; o < m.ns; ++o) {
        const int g = nb[o * n];
        if (g >= 0) a = fma(c[o * n], v[g], a);
    }
    return a;
}
__device__ __forceinline__ double vmg_diag(const MgDev& m, int l, int f) {
    return m.coef[m.so[l] + (long)(m.ns / 2) * m.n[l] + f];
}
// the post-smoothed vector of level l (the coarsest level has no smoother)
__device__ __forceinline__ const double* vmg_post_vec(const MgDev& m, int l) {
    return l == m.L ? m.x + m.vo[l] : m.y + m.vo[l];
}
__device__ __forceinline__ void vmg_pre_at(const MgDev& m, int l, int f) {
    m.x[m.vo[l] + f] = m.omega * m.b[m.vo[l] + f] / vmg_diag(m, l, f);
}
__device__ __forceinline__ void vmg_res_at(const MgDev& m, int l, int f) {
    m.r[m.vo[l] + f] = m.b[m.vo[l] + f] - vmg_apply_at(m, l, f, m.x + m.vo[l]);
}
// full-weighting restriction (transpose of the interpolation): children of C
// at 2C + o with weight prod_d (o_d == 0 ? 1 : 1/2)
__device__ __forceinline__ void vmg_restrict_at(const MgDev& m, int l, int C) {
    const long nc = m.n[l + 1];
    const int* ch = m.chl + m.so[l + 1] + C;
    const double* rl = m.r + m.vo[l];
    double v = 0.0;
    for (int o = 0; o < m.ns; ++o) {
        const int f = ch[o * nc];
        if (f < 0) continue;
        double w = 1.0;
        int t = o;
        for (int d = 0; d < m.dim; ++d) {
            if (t % 3 != 1) w *= 0.5;
            t /= 3;
        }
        v = fma(w, rl[f], v);
    }
    m.b[m.vo[l + 1] + C] = v;
}
// x_l += P x_{l+1}
__device__ __forceinline__ void vmg_prolong_at(const MgDev& m, int l, int f) {
    const int nch = 1 << m.dim;
    const double* xc = vmg_post_vec(m, l + 1);
    const long n = m.n[l];
    const int* pa = m.par + m.po[l] + f;
    const double* pw = m.pw + m.po[l] + f;
    double v = m.x[m.vo[l] + f];
    for (int q = 0; q < nch; ++q)
        if (pa[q * n] >= 0) v = fma(pw[q * n], xc[pa[q * n]], v);
    m.x[m.vo[l] + f] = v;
}
__device__ __forceinline__ void vmg_post_at(const MgDev& m, int l, int f) {
    const double* xl = m.x + m.vo[l];
    m.y[m.vo[l] + f] = xl[f] + m.omega * (m.b[m.vo[l] + f] - vmg_apply_at(m, l, f, xl)) / vmg_diag(m, l, f);
}

#define VMG_GRID_KERNEL(NAME, N, BODY)                                                                 \
    __global__ void __launch_bounds__(256) NAME(MgDev m, int l, const CgScalars* s) {                  \
        if (s->done) return;                                                                           \
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < (N); i += gridDim.x * blockDim.x) BODY; \
    }
VMG_GRID_KERNEL(vmg_pre_kernel, m.n[l], vmg_pre_at(m, l, i))
VMG_GRID_KERNEL(vmg_res_kernel, m.n[l], vmg_res_at(m, l, i))
VMG_GRID_KERNEL(vmg_restrict_kernel, m.n[l + 1], vmg_restrict_at(m, l, i))
VMG_GRID_KERNEL(vmg_prolong_kernel, m.n[l], vmg_prolong_at(m, l, i))
VMG_GRID_KERNEL(vmg_post_kernel, m.n[l], vmg_post_at(m, l, i))
#undef VMG_GRID_KERNEL

// levels lc .. L in one workgroup (their sizes are small)
__global__ void __launch_bounds__(1024) vmg_coarse_kernel(MgDev m, int lc, const CgScalars* s) {
    if (s->done) return;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int l = lc; l < m.L; ++l) {
        for (int i = tid; i < m.n[l]; i += nt) vmg_pre_at(m, l, i);
        __syncthreads();
        for (int i = tid; i < m.n[l]; i += nt) vmg_res_at(m, l, i);
        __syncthreads();
        for (int i = tid; i < m.n[l + 1]; i += nt) vmg_restrict_at(m, l, i);
        __syncthreads();
    }
    // dense solve: one wave per row at a time, lanes over the columns
    // (coalesced row reads), then a fixed-order butterfly sum across the wave
    const int nL = m.n[m.L];
    const double* bL = m.b + m.vo[m.L];
    const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
    for (int i = wv; i < nL; i += nw) {
        const double* row = m.ainv + (long)i * nL;
        double v = 0.0;
        for (int j = lane; j < nL; j += 64) v = fma(row[j], bL[j], v);
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) m.x[m.vo[m.L] + i] = v;
    }
    __syncthreads();
    for (int l = m.L - 1; l >= lc; --l) {
        for (int i = tid; i < m.n[l]; i += nt) vmg_prolong_at(m, l, i);
        __syncthreads();
        for (int i = tid; i < m.n[l]; i += nt) vmg_post_at(m, l, i);
        __syncthreads();
    }
}

// level 0 pre-smoothing from zero: z0 = omega0 B^{-1} r
template <int NN>
__global__ void __launch_bounds__(256) mg_l0_pre_kernel(DsaGeom g, const double* __restrict__ binv,
                                                        const double* __restrict__ r, double* __restrict__ z0,
                                                        double omega0, const CgScalars* s) {
    if (s->done) return;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < g.nthick; t += gridDim.x * blockDim.x) {
        double rv[NN], zv[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) rv[n] = r[(long)t * NN + n];
        bj_apply<NN>(binv, g.nthick, t, rv, zv);
#pragma unroll
        for (int n = 0; n < NN; ++n) z0[(long)t * NN + n] = omega0 * zv[n];
    }
}

// level 0 residual res0 = r - D_ff z0
template <int NN>
__global__ void __launch_bounds__(256) mg_l0_res_kernel(DsaGeom g, const int* __restrict__ thick_cell,
                                                        const int* __restrict__ nbr,
                                                        const double* __restrict__ sigma_t,
                                                        const double* __restrict__ sigma_s,
                                                        const double* __restrict__ r,
                                                        const double* __restrict__ z0, double* __restrict__ res0,
                                                        const CgScalars* s) {
    if (s->done) return;
    auto get = [&](int slot, double out[NN]) {
#pragma unroll
        for (int n = 0; n < NN; ++n) out[n] = z0[(long)slot * NN + n];
    };
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < g.nthick; t += gridDim.x * blockDim.x) {
        double uK[NN], o[NN];
        get(t, uK);
        sip_rows<NN>(g, t, thick_cell[t], nbr, thick_cell, sigma_t, sigma_s, uK, get, o);
#pragma unroll
        for (int n = 0; n < NN; ++n) res0[(long)t * NN + n] = r[(long)t * NN + n] - o[n];
    }
}

// b1[w] = sum of res0 over the DG nodes at vertex w (fixed order)
__global__ void __launch_bounds__(256) mg_restrict1_kernel(MgDev m, const double* __restrict__ res0,
                                                           const CgScalars* s) {
    if (s->done) return;
    const int nch = 1 << m.dim;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < m.n[1]; w += gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int q = 0; q < nch; ++q) {
            const int e = m.vnodes[(long)q * m.n[1] + w];
            if (e >= 0) v += res0[e];
        }
        m.b[m.vo[1] + w] = v;
    }
}

// level 0 post-smoothing: zp = z0 + P x1, z = zp + omega0 B^{-1} (r - D_ff zp)
// (zp on the fly for the cell and its neighbours); partials r.z -> part[block]
template <int NN>
__global__ void __launch_bounds__(256) mg_l0_post_kernel(DsaGeom g, const int* __restrict__ thick_cell,
                                                         const int* __restrict__ nbr,
                                                         const double* __restrict__ sigma_t,
                                                         const double* __restrict__ sigma_s,
                                                         const double* __restrict__ binv,
                                                         const double* __restrict__ r, const double* __restrict__ z0,
                                                         MgDev m, double omega0, double* __restrict__ z,
                                                         double* __restrict__ part, const CgScalars* s) {
    if (s->done) return;
    __shared__ double sh[16];
    const double* x1 = vmg_post_vec(m, 1);
    auto get = [&](int slot, double out[NN]) {
#pragma unroll
        for (int n = 0; n < NN; ++n) out[n] = z0[(long)slot * NN + n] + x1[m.nodev[(long)slot * NN + n]];
    };
    double rz = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < g.nthick; t += gridDim.x * blockDim.x) {
        double uK[NN], o[NN], rv[NN], zv[NN];
        get(t, uK);
        sip_rows<NN>(g, t, thick_cell[t], nbr, thick_cell, sigma_t, sigma_s, uK, get, o);
#pragma unroll
        for (int n = 0; n < NN; ++n) rv[n] = r[(long)t * NN + n] - o[n];
        bj_apply<NN>(binv, g.nthick, t, rv, zv);
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            const double zz = fma(omega0, zv[n], uK[n]);
            z[(long)t * NN + n] = zz;
            rz = fma(r[(long)t * NN + n], zz, rz);
        }
    }
    rz = block_reduce(rz, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = rz;
}

// One V-cycle z = M^{-1} r; vertex levels 1 .. lc-1 run as grid-wide kernels,
// levels lc .. L in the single-workgroup kernel.  res0: DG scratch.
// part: r.z partials ([0..nparts)).
hipError_t launch_mg_vcycle(const DsaGeom& g, const int* thick_cell, const int* nbr, const double* sigma_t,
                            const double* sigma_s, const double* binv, const double* r, double* z0, double* res0,
                            double* z, const MgDev& m, int lc, double omega0, double* part, int nparts,
                            const CgScalars* s, hipStream_t st) {
    const int gb = nparts;
    auto blocks = [](int n) { return std::max(1, std::min((n + 255) / 256, 4096)); };
    if (g.nn == 4) {
        hipLaunchKernelGGL(mg_l0_pre_kernel<4>, dim3(gb), dim3(256), 0, st, g, binv, r, z0, omega0, s);
        hipLaunchKernelGGL(mg_l0_res_kernel<4>, dim3(gb), dim3(256), 0, st, g, thick_cell, nbr, sigma_t, sigma_s,
                           r, z0, res0, s);
    } else {
        hipLaunchKernelGGL(mg_l0_pre_kernel<8>, dim3(gb), dim3(256), 0, st, g, binv, r, z0, omega0, s);
        hipLaunchKernelGGL(mg_l0_res_kernel<8>, dim3(gb), dim3(256), 0, st, g, thick_cell, nbr, sigma_t, sigma_s,
                           r, z0, res0, s);
    }
    hipLaunchKernelGGL(mg_restrict1_kernel, dim3(blocks(m.n[1])), dim3(256), 0, st, m, res0, s);
    for (int l = 1; l < lc; ++l) {
        hipLaunchKernelGGL(vmg_pre_kernel, dim3(blocks(m.n[l])), dim3(256), 0, st, m, l, s);
        hipLaunchKernelGGL(vmg_res_kernel, dim3(blocks(m.n[l])), dim3(256), 0, st, m, l, s);
        hipLaunchKernelGGL(vmg_restrict_kernel, dim3(blocks(m.n[l + 1])), dim3(256), 0, st, m, l, s);
    }
    hipLaunchKernelGGL(vmg_coarse_kernel, dim3(1), dim3(1024), 0, st, m, lc, s);
    for (int l = lc - 1; l >= 1; --l) {
        hipLaunchKernelGGL(vmg_prolong_kernel, dim3(blocks(m.n[l])), dim3(256), 0, st, m, l, s);
        hipLaunchKernelGGL(vmg_post_kernel, dim3(blocks(m.n[l])), dim3(256), 0, st, m, l, s);
    }
    if (g.nn == 4)
        hipLaunchKernelGGL(mg_l0_post_kernel<4>, dim3(gb), dim3(256), 0, st, g, thick_cell, nbr, sigma_t, sigma_s,
                           binv, r, z0, m, omega0, z, part, s);
    else
        hipLaunchKernelGGL(mg_l0_post_kernel<8>, dim3(gb), dim3(256), 0, st, g, thick_cell, nbr, sigma_t, sigma_s,
                           binv, r, z0, m, omega0, z, part, s);
    return hipGetLastError();
}

}  // namespace sn
