// Scalar-flux side of one source iteration (Section 2.2, eq. psi / eq. phi):
//   source   s = (sigma_s phi + q) / 4pi per node (the M^{-1}-scaled volume load),
//   moment   phi = sum_d w_d psi_d, always accumulated in FP64,
//   residual ||phi_SI - phi||^2, ||phi_SI||^2, ||phi||^2 (eq. source0),
//   gradient contraction of the adjoint (derived from eq. system).
#include "sn_kernels.hpp"

namespace sn {

constexpr double kInv4Pi = 0.079577471545947667884;  // 1 / (4 pi)

// s = (sigma_s (phi - phi_prev) + q) / 4pi, formed in FP64 and rounded once
// to the sweep precision; phi_prev, phi and q may be NULL (zero).
template <typename T>
__global__ void source_kernel(long n, int nn, const double* __restrict__ sigma_s, const double* __restrict__ phi,
                              const double* __restrict__ phi_prev, const double* __restrict__ q,
                              T* __restrict__ src) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        long c = e / nn;
        double f = phi ? phi[e] : 0.0;
        if (phi_prev) f -= phi_prev[e];
        double v = sigma_s[c] * f + (q ? q[c] : 0.0);
        src[e] = T(v * kInv4Pi);
    }
}

template <typename T>
hipError_t launch_source(long nc, int nn, const double* sigma_s, const double* phi, const double* phi_prev,
                         const double* q, T* src, hipStream_t st) {
    long n = nc * nn;
    int blocks = (int)std::min<long>((n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(source_kernel<T>, dim3(blocks), dim3(256), 0, st, n, nn, sigma_s, phi, phi_prev, q, src);
    return hipGetLastError();
}

// Four lanes per cell: lane j of the cell sums directions j, j + 4, j + 8, ...
// (the four lanes read four consecutive direction blocks of the cell's
// contiguous [ndirs][NN] block of psi), then the lanes' sums are combined by
// an xor butterfly, (s0 + s1) + (s2 + s3), and lane j writes nodes j (and
// j + 4 when NN = 8).
// RES: also the block partial sums of (phi - ref)^2, phi^2, ref^2 over the
// written phi (part[3][gridDim.x]), the residual of source iteration.
template <typename T, int NN, bool RES>
__global__ void __launch_bounds__(256) moment_kernel(long nc, int ndirs, const double* __restrict__ w,
                                                     const T* __restrict__ psi, double* __restrict__ phi,
                                                     int accumulate, const double* __restrict__ ref,
                                                     double* __restrict__ part) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const int j = threadIdx.x & 3;
    const long stride = ((long)gridDim.x * blockDim.x) >> 2;
    for (long c = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 2; c < nc; c += stride) {
        double acc[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) acc[n] = 0.0;
        const T* p = psi + c * ndirs * NN;
        for (int d = j; d < ndirs; d += 4) {
            const double wd = w[d];
#pragma unroll
            for (int n = 0; n < NN; ++n) acc[n] = fma(wd, double(p[d * NN + n]), acc[n]);
        }
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            acc[n] += __shfl_xor(acc[n], 1, 4);
            acc[n] += __shfl_xor(acc[n], 2, 4);
        }
#pragma unroll
        for (int h = 0; h < NN / 4; ++h) {
            const int n = j + 4 * h;
            const long e = c * NN + n;
            const double v = accumulate ? phi[e] + acc[n] : acc[n];
            phi[e] = v;
            if constexpr (RES) {
                const double y = ref[e], d = v - y;
                s0 = fma(d, d, s0);
                s1 = fma(v, v, s1);
                s2 = fma(y, y, s2);
            }
        }
    }
    if constexpr (RES) {
        __shared__ double sh[48];
        block_sum3(s0, s1, s2, sh);
        if (threadIdx.x == 0) {
            part[blockIdx.x] = s0;
            part[gridDim.x + blockIdx.x] = s1;
            part[2 * gridDim.x + blockIdx.x] = s2;
        }
    }
}

template <typename T>
hipError_t launch_moment(long nc, int nn, int ndirs, const double* w, const T* psi, double* phi, int accumulate,
                         const double* ref, double* part, hipStream_t st) {
    const int blocks = moment_blocks(nc);
#define SN_MOM(NN, RES)                                                                                          \
    hipLaunchKernelGGL((moment_kernel<T, NN, RES>), dim3(blocks), dim3(256), 0, st, nc, ndirs, w, psi, phi,     \
                       accumulate, ref, part)
    if (nn == 4) {
        if (ref) SN_MOM(4, true);
        else SN_MOM(4, false);
    } else {
        if (ref) SN_MOM(8, true);
        else SN_MOM(8, false);
    }
#undef SN_MOM
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) residual_part_kernel(long n, const double* __restrict__ a,
                                                            const double* __restrict__ b,
                                                            double* __restrict__ part) {
    __shared__ double sh[48];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        double x = a[e], y = b[e], d = x - y;
        s0 = fma(d, d, s0);
        s1 = fma(x, x, s1);
        s2 = fma(y, y, s2);
    }
    block_sum3(s0, s1, s2, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0;
        part[gridDim.x + blockIdx.x] = s1;
        part[2 * gridDim.x + blockIdx.x] = s2;
    }
}

__global__ void __launch_bounds__(256) residual_final_kernel(int nparts, const double* __restrict__ part,
                                                             double* __restrict__ out, double* __restrict__ out_host) {
    __shared__ double sh[48];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int e = threadIdx.x; e < nparts; e += 256) {
        s0 += part[e];
        s1 += part[nparts + e];
        s2 += part[2 * nparts + e];
    }
    block_sum3(s0, s1, s2, sh);
    if (threadIdx.x == 0) {
        out[0] = s0;
        out[1] = s1;
        out[2] = s2;
        if (out_host) {
            out_host[0] = s0;
            out_host[1] = s1;
            out_host[2] = s2;
        }
    }
}

hipError_t launch_residual(long n, const double* a, const double* b, double* partials, int nparts, double* out,
                           hipStream_t st) {
    hipLaunchKernelGGL(residual_part_kernel, dim3(nparts), dim3(256), 0, st, n, a, b, partials);
    hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(256), 0, st, nparts, partials, out, nullptr);
    return hipGetLastError();
}

hipError_t launch_residual_final(int nparts, const double* partials, double* out, double* out_host,
                                 hipStream_t st) {
    hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(256), 0, st, nparts, partials, out, out_host);
    return hipGetLastError();
}

// dJ/dlog sigma_t,K = -sigma_t,K sum_d w_d psia_d,K^T M_K psi_d,K
// dJ/dlog sigma_s,K =  sigma_s,K chi_K^T M_K phi_K / 4pi
// M_K = (x) of 1D masses h/6 [[2,1],[1,2]]; applied as a tensor product.
template <int NN>
__device__ __forceinline__ void apply_mass(const double* h, const double in[NN], double out[NN]) {
    double t[NN];
#pragma unroll
    for (int n = 0; n < NN; ++n) t[n] = in[n];
    const int naxes = NN == 4 ? 2 : 3;
#pragma unroll
    for (int ax = 0; ax < naxes; ++ax) {
        const int st = 1 << ax;
        const double a = h[ax] / 3.0, b = h[ax] / 6.0;
        double o[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            const int m = n ^ st;
            o[n] = a * t[n] + b * t[m];
        }
#pragma unroll
        for (int n = 0; n < NN; ++n) t[n] = o[n];
    }
#pragma unroll
    for (int n = 0; n < NN; ++n) out[n] = t[n];
}

// psi, psia: [cell][ndirs][NN] for the ndirs directions of w (a part of the
// quadrature: directions of zero weight are unused slots and are skipped).
// accumulate: g_t += instead of =; g_s (with phi, chi) is written when given.
template <typename T, int NN>
__global__ void gradient_kernel(long nc, int ndirs, const double* __restrict__ w, double hx, double hy, double hz,
                                const double* __restrict__ sigma_t, const double* __restrict__ sigma_s,
                                const T* __restrict__ psi, const T* __restrict__ psia,
                                const double* __restrict__ phi, const double* __restrict__ chi,
                                double* __restrict__ gt, double* __restrict__ gs, int accumulate) {
    const double h[3] = {hx, hy, hz};
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (long)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int d = 0; d < ndirs; ++d) {
            const double wd = w[d];
            if (wd == 0.0) continue;
            double a[NN], b[NN], mb[NN];
            const T* pa = psia + (c * ndirs + d) * NN;
            const T* pb = psi + (c * ndirs + d) * NN;
#pragma unroll
            for (int n = 0; n < NN; ++n) {
                a[n] = double(pa[n]);
                b[n] = double(pb[n]);
            }
            apply_mass<NN>(h, b, mb);
            double v = 0.0;
#pragma unroll
            for (int n = 0; n < NN; ++n) v = fma(a[n], mb[n], v);
            acc = fma(wd, v, acc);
        }
        const double g = -sigma_t[c] * acc;
        gt[c] = accumulate ? gt[c] + g : g;
        if (gs) {
            double x[NN], mx[NN];
#pragma unroll
            for (int n = 0; n < NN; ++n) x[n] = phi[c * NN + n];
            apply_mass<NN>(h, x, mx);
            double v = 0.0;
#pragma unroll
            for (int n = 0; n < NN; ++n) v = fma(chi[c * NN + n], mx[n], v);
            gs[c] = sigma_s[c] * v * kInv4Pi;
        }
    }
}
template <typename T>
hipError_t launch_gradient(long nc, int nn, int ndirs, const double* w, const double* h, const double* sigma_t,
                           const double* sigma_s, const T* psi, const T* psi_adj, const double* phi,
                           const double* chi, double* g_t, double* g_s, hipStream_t st, int accumulate) {
    int blocks = (int)std::min<long>((nc + 255) / 256, 1 << 16);
    if (nn == 4)
        hipLaunchKernelGGL((gradient_kernel<T, 4>), dim3(blocks), dim3(256), 0, st, nc, ndirs, w, h[0], h[1], h[2],
                           sigma_t, sigma_s, psi, psi_adj, phi, chi, g_t, g_s, accumulate);
    else
        hipLaunchKernelGGL((gradient_kernel<T, 8>), dim3(blocks), dim3(256), 0, st, nc, ndirs, w, h[0], h[1], h[2],
                           sigma_t, sigma_s, psi, psi_adj, phi, chi, g_t, g_s, accumulate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// triangular heterogeneous DSA (Alg. 1): the thick part of the preconditioned
// residual, and the thin-only accumulation of its transport update
// ---------------------------------------------------------------------------
// bar = (a - b) on the nodes of thick cells (slot_of_cell >= 0), 0 elsewhere
__global__ void thick_diff_kernel(long nc, int nn, const int* __restrict__ slot_of_cell,
                                  const double* __restrict__ a, const double* __restrict__ b,
                                  double* __restrict__ bar) {
    const long n = nc * nn;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const long c = e / nn;
        bar[e] = slot_of_cell[c] >= 0 ? a[e] - (b ? b[e] : 0.0) : 0.0;
    }
}
// phi += z on the nodes of thin (and void) cells
__global__ void thin_add_kernel(long nc, int nn, const int* __restrict__ slot_of_cell, const double* __restrict__ z,
                                double* __restrict__ phi) {
    const long n = nc * nn;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const long c = e / nn;
        if (slot_of_cell[c] < 0) phi[e] += z[e];
    }
}
hipError_t launch_thick_diff(long nc, int nn, const int* slot_of_cell, const double* a, const double* b, double* bar,
                             hipStream_t st) {
    const int blocks = (int)std::min<long>((nc * nn + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(thick_diff_kernel, dim3(blocks), dim3(256), 0, st, nc, nn, slot_of_cell, a, b, bar);
    return hipGetLastError();
}
hipError_t launch_thin_add(long nc, int nn, const int* slot_of_cell, const double* z, double* phi, hipStream_t st) {
    const int blocks = (int)std::min<long>((nc * nn + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(thin_add_kernel, dim3(blocks), dim3(256), 0, st, nc, nn, slot_of_cell, z, phi);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// adjoint sources of the two responses
// ---------------------------------------------------------------------------
// q_adj = 4 pi r (volume detector J = sum_c r_c int_c phi)
// y = a x; y may be x
__global__ void scale_kernel(long n, double a, const double* x, double* y) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        y[e] = a * x[e];
}
// boundary data of the transposed sweep for the outflow current through a
// domain face: 1 on that face's slot of the inflow layout for every
// direction leaving through it (out: 1 or 0 per direction), 0 elsewhere
__global__ void face_data_kernel(int ndirs, long nbf, long f0, long f1, const int* __restrict__ out,
                                 double* __restrict__ data) {
    const long n = (long)ndirs * nbf;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const int d = (int)(e / nbf);
        const long f = e - (long)d * nbf;
        data[e] = (out[d] && f >= f0 && f < f1) ? 1.0 : 0.0;
    }
}
hipError_t launch_scale(long n, double a, const double* x, double* y, hipStream_t st) {
    const int blocks = (int)std::min<long>((n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(scale_kernel, dim3(blocks), dim3(256), 0, st, n, a, x, y);
    return hipGetLastError();
}
hipError_t launch_face_data(int ndirs, long nbf, long f0, long f1, const int* out, double* data, hipStream_t st) {
    const long n = (long)ndirs * nbf;
    const int blocks = (int)std::min<long>((n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(face_data_kernel, dim3(blocks), dim3(256), 0, st, ndirs, nbf, f0, f1, out, data);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Krylov vector operations (FP64), reduced in a fixed order
// ---------------------------------------------------------------------------
// part[i][blockIdx.x] = block's share of V_i . w for i < k (V: k vectors of
// length n, stride n); up to KB vectors per pass over w
constexpr int KB = 8;
__global__ void __launch_bounds__(256) multi_dot_kernel(long n, int k, const double* __restrict__ V,
                                                        const double* __restrict__ w, double* __restrict__ part) {
    __shared__ double sh[48];
    for (int i0 = 0; i0 < k; i0 += KB) {
        double acc[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) acc[i] = 0.0;
        const int nk = min(KB, k - i0);
        for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
            const double we = w[e];
#pragma unroll
            for (int i = 0; i < KB; ++i)
                if (i < nk) acc[i] = fma(V[(long)(i0 + i) * n + e], we, acc[i]);
        }
        for (int i = 0; i < nk; i += 3) {
            double a = acc[i], b = i + 1 < nk ? acc[i + 1] : 0.0, c = i + 2 < nk ? acc[i + 2] : 0.0;
            block_sum3(a, b, c, sh);
            if (threadIdx.x == 0) {
                part[(long)(i0 + i) * gridDim.x + blockIdx.x] = a;
                if (i + 1 < nk) part[(long)(i0 + i + 1) * gridDim.x + blockIdx.x] = b;
                if (i + 2 < nk) part[(long)(i0 + i + 2) * gridDim.x + blockIdx.x] = c;
            }
        }
    }
}
// out[i] = sum over blocks of part[i][.] (one workgroup per i, fixed order);
// also to pinned host memory when out_host is given
__global__ void __launch_bounds__(256) multi_dot_final_kernel(int nparts, const double* __restrict__ part,
                                                              double* __restrict__ out, double* __restrict__ out_host) {
    __shared__ double sh[48];
    double a = 0.0, b = 0.0, c = 0.0;
    const double* pi = part + (long)blockIdx.x * nparts;
    for (int e = threadIdx.x; e < nparts; e += 256) a += pi[e];
    block_sum3(a, b, c, sh);
    if (threadIdx.x == 0) {
        out[blockIdx.x] = a;
        if (out_host) out_host[blockIdx.x] = a;
    }
}
// w -= sum_i h[i] V_i (i < k)
__global__ void multi_axpy_kernel(long n, int k, const double* __restrict__ V, const double* __restrict__ h,
                                  double sign, double* __restrict__ w) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s = fma(h[i], V[(long)i * n + e], s);
        w[e] = fma(sign, s, w[e]);
    }
}
// y = a x + b y
__global__ void axpby_kernel(long n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        y[e] = fma(a, x[e], b * y[e]);
}
int krylov_blocks(long n) { return (int)std::min<long>((n + 255) / 256, 1024); }
hipError_t launch_multi_dot(long n, int k, const double* V, const double* w, double* part, double* out,
                            double* out_host, hipStream_t st) {
    const int nb = krylov_blocks(n);
    hipLaunchKernelGGL(multi_dot_kernel, dim3(nb), dim3(256), 0, st, n, k, V, w, part);
    hipLaunchKernelGGL(multi_dot_final_kernel, dim3(k), dim3(256), 0, st, nb, part, out, out_host);
    return hipGetLastError();
}
hipError_t launch_multi_axpy(long n, int k, const double* V, const double* h, double sign, double* w,
                             hipStream_t st) {
    const int blocks = (int)std::min<long>((n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(multi_axpy_kernel, dim3(blocks), dim3(256), 0, st, n, k, V, h, sign, w);
    return hipGetLastError();
}
hipError_t launch_axpby(long n, double a, const double* x, double b, double* y, hipStream_t st) {
    const int blocks = (int)std::min<long>((n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(axpby_kernel, dim3(blocks), dim3(256), 0, st, n, a, x, b, y);
    return hipGetLastError();
}

// Linear functionals of the solution, reduced deterministically:
//   out[0] = sum_c r_c int_c phi            (volume detector, r per cell)
//   out[1] = sum_{d: Omega_d.n > 0} w_d (Omega_d.n) int_face psi_d
//            (partial outflow current through one domain face)
template <typename T, int NN>
__global__ void __launch_bounds__(256) response_part_kernel(long nc, int nx, int ny, int nz, double hx, double hy,
                                                            double hz, const double* __restrict__ r,
                                                            const double* __restrict__ phi, int face, int ndirs,
                                                            const double* __restrict__ wn, const T* __restrict__ psi,
                                                            double* __restrict__ part) {
    __shared__ double sh[256];
    constexpr int DIM = NN == 4 ? 2 : 3;
    const double h[3] = {hx, hy, hz};
    double vol = DIM == 2 ? hx * hy : hx * hy * hz;
    double a = 0.0, b = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (long)gridDim.x * blockDim.x) {
        if (r && phi) {
            // int_c phi = vol / NN * sum of nodal values (Q1, exact)
            double s = 0.0;
#pragma unroll
            for (int n = 0; n < NN; ++n) s += phi[c * NN + n];
            a = fma(r[c] * vol / NN, s, a);
        }
        if (face >= 0 && psi) {
            const int ax = face >> 1, side = face & 1;
            const int pos[3] = {(int)(c % nx), (int)((c / nx) % ny), (int)(c / ((long)nx * ny))};
            const int ext[3] = {nx, ny, nz};
            if (pos[ax] == (side ? ext[ax] - 1 : 0)) {
                double area = 1.0;
                for (int o = 0; o < DIM; ++o)
                    if (o != ax) area *= h[o];
                for (int d = 0; d < ndirs; ++d) {
                    const double wd = wn[d];
                    if (wd <= 0.0) continue;
                    double s = 0.0;
#pragma unroll
                    for (int n = 0; n < NN; ++n)
                        if (((n >> ax) & 1) == side) s += double(psi[(c * ndirs + d) * NN + n]);
                    b = fma(wd * area / (NN / 2), s, b);
                }
            }
        }
    }
    double t[2] = {a, b};
    for (int k = 0; k < 2; ++k) {
        sh[threadIdx.x] = t[k];
        __syncthreads();
        for (int s2 = 128; s2 > 0; s2 >>= 1) {
            if (threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[k * gridDim.x + blockIdx.x] = sh[0];
        __syncthreads();
    }
}

template <typename T>
hipError_t launch_response(long nc, int nn, int nx, int ny, int nz, const double* h, const double* r,
                           const double* phi, int face, int ndirs, const double* wn, const T* psi, double* part,
                           int nparts, double* out, hipStream_t st) {
    if (nn == 4)
        hipLaunchKernelGGL((response_part_kernel<T, 4>), dim3(nparts), dim3(256), 0, st, nc, nx, ny, nz, h[0], h[1],
                           h[2], r, phi, face, ndirs, wn, psi, part);
    else
        hipLaunchKernelGGL((response_part_kernel<T, 8>), dim3(nparts), dim3(256), 0, st, nc, nx, ny, nz, h[0], h[1],
                           h[2], r, phi, face, ndirs, wn, psi, part);
    // final fixed-order sum of the two partial arrays (third slot unused)
    hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(256), 0, st, nparts, part, out, nullptr);
    return hipGetLastError();
}

template hipError_t launch_response<double>(long, int, int, int, int, const double*, const double*, const double*,
                                            int, int, const double*, const double*, double*, int, double*,
                                            hipStream_t);
template hipError_t launch_response<float>(long, int, int, int, int, const double*, const double*, const double*,
                                           int, int, const double*, const float*, double*, int, double*,
                                           hipStream_t);

template hipError_t launch_source<double>(long, int, const double*, const double*, const double*, const double*,
                                          double*, hipStream_t);
template hipError_t launch_source<float>(long, int, const double*, const double*, const double*, const double*,
                                         float*, hipStream_t);
template hipError_t launch_moment<double>(long, int, int, const double*, const double*, double*, int, const double*,
                                          double*, hipStream_t);
template hipError_t launch_moment<float>(long, int, int, const double*, const float*, double*, int, const double*,
                                         double*, hipStream_t);
template hipError_t launch_gradient<double>(long, int, int, const double*, const double*, const double*,
                                            const double*, const double*, const double*, const double*,
                                            const double*, double*, double*, hipStream_t, int);
template hipError_t launch_gradient<float>(long, int, int, const double*, const double*, const double*,
                                           const double*, const float*, const float*, const double*,
                                           const double*, double*, double*, hipStream_t, int);

}  // namespace sn
