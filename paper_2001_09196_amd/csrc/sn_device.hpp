// Device-side building blocks shared by the sweep kernels: per-direction
// constants and the local upwind-DG cell solve.
//
// Cell problem (Section 3.1, eq. Tmat1 at eps = 1, one Cartesian Q1 cell):
//   A u = f,  A = sum_axes |Omega_a| (mass of the other axes) (x) G_a + sigma_t M,
// with the 1D upwind block G = [[1/2, 1/2], [-1/2, 1/2]] in a frame where
// every direction component is positive.  Every direction is mapped to that
// frame by reflecting the axes along which its component is negative (node
// index a -> 1 - a), so one code path serves all octants.
//
// Multiplying by M^{-1} turns A into a Kronecker sum,
//   M^{-1} A = a_x K (x) I (x) I + a_y I (x) K (x) I + a_z I (x) I (x) K + sigma_t I,
//   a_axis = |Omega_axis| / h_axis,  K = [[3, 1], [-3, 1]],
// and K = V diag(2 + i sqrt2, 2 - i sqrt2) V^{-1} with
//   V = [[1, 1], [-1 + i sqrt2, -1 - i sqrt2]],
//   (V^{-1} b)_+ = b0/2 - i (b0 + b1) / (2 sqrt2)   (the other row is its conjugate).
// The solve is therefore: transform the right-hand side axis by axis into the
// eigenbasis, divide by a_x l_x + a_y l_y + a_z l_z + sigma_t, transform back.
// For real data the coefficients come in conjugate pairs, so only the half
// with the + eigenvalue along x is carried: 4 real numbers per 2D cell and 8
// per 3D cell, the same storage as the nodal values.
//
// The right-hand side is M^{-1} f: the volume load M (sigma_s phi + q)/4pi
// becomes the nodal values (sigma_s phi + q)/4pi, and an inflow face load
// |Omega_a| (face mass) psi_up on the a = 0 face becomes
//   +4 a_axis psi_up on node 0 and -2 a_axis psi_up on node 1 of that axis.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>

namespace sn {

struct DirInfo {
    double ax, ay, az;  // |Omega_axis| / h_axis
    double w;           // quadrature weight
    int rx, ry, rz;     // 1 if the axis is reflected (component < 0)
    int pad;
};

// reciprocal: hardware estimate refined by Newton steps
__device__ __forceinline__ double rcp(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}
__device__ __forceinline__ float rcp(float d) {
    float r = __builtin_amdgcn_rcpf(d);
    r = fmaf(r, fmaf(-d, r, 1.0f), r);
    return r;
}

// Reciprocals of two or four denominators P^2 + Q^2 of the cell solves.  In
// FP64 they come from one reciprocal of their product (one v_rcp_f64 and its
// Newton steps instead of two or four): the product of four such factors
// stays inside the double range for any cross sections and cell sizes below
// about 1e38 in magnitude.  FP32 takes each reciprocal on its own, since the
// product could leave the float range.
__device__ __forceinline__ void rcp_each(const double d[2], double r[2], std::integral_constant<int, 2>) {
    const double R = rcp(d[0] * d[1]);
    r[0] = R * d[1];
    r[1] = R * d[0];
}
__device__ __forceinline__ void rcp_each(const double d[4], double r[4], std::integral_constant<int, 4>) {
    const double d01 = d[0] * d[1], d23 = d[2] * d[3];
    const double R = rcp(d01 * d23);
    const double a = R * d23, b = R * d01;
    r[0] = a * d[1];
    r[1] = a * d[0];
    r[2] = b * d[3];
    r[3] = b * d[2];
}
template <int N>
__device__ __forceinline__ void rcp_each(const float d[N], float r[N], std::integral_constant<int, N>) {
#pragma unroll
    for (int e = 0; e < N; ++e) r[e] = rcp(d[e]);
}

template <typename T>
struct Consts {
    static constexpr T k = T(0.35355339059327376220);   // 1 / (2 sqrt 2)
    static constexpr T r2 = T(1.41421356237309504880);  // sqrt 2
};

// complex helpers on (re, im) pairs held in registers
template <typename T>
struct cpx {
    T re, im;
};

// ell^{(+)} . (c0, c1) = c0/2 - i k (c0 + c1) and ell^{(-)} . (c0, c1) = c0/2 + i k (c0 + c1)
template <typename T>
__device__ __forceinline__ void fwd_pair(cpx<T> c0, cpx<T> c1, cpx<T>& p, cpx<T>& m) {
    const T k = Consts<T>::k;
    T sr = c0.re + c1.re, si = c0.im + c1.im;
    T hr = T(0.5) * c0.re, hi = T(0.5) * c0.im;
    p.re = fma(k, si, hr);
    p.im = fma(-k, sr, hi);
    m.re = fma(-k, si, hr);
    m.im = fma(k, sr, hi);
}

// inverse along one axis: node 0 = H+ + H-,
// node 1 = (-1 + i r2) H+ + (-1 - i r2) H- = -(H+ + H-) + i r2 (H+ - H-)
template <typename T>
__device__ __forceinline__ void inv_pair(cpx<T> hp, cpx<T> hm, cpx<T>& n0, cpx<T>& n1) {
    const T r2 = Consts<T>::r2;
    T sr = hp.re + hm.re, si = hp.im + hm.im;
    T dr = hp.re - hm.re, di = hp.im - hm.im;
    n0.re = sr;
    n0.im = si;
    n1.re = fma(-r2, di, -sr);
    n1.im = fma(r2, dr, -si);
}

// H = F / (P + i Q) = F (P - i Q) / (P^2 + Q^2)
template <typename T>
__device__ __forceinline__ cpx<T> cdiv(cpx<T> f, T P, T Q, T inv) {
    cpx<T> h;
    h.re = fma(f.re, P, f.im * Q) * inv;
    h.im = fma(f.im, P, -f.re * Q) * inv;
    return h;
}

// 2D cell solve in the reflected frame. g, u: nodes a + 2b.
template <typename T>
__device__ __forceinline__ void cell_solve2(const T g[4], T ax, T ay, T sig, T u[4]) {
    const T k2 = T(2) * Consts<T>::k, r2 = Consts<T>::r2;
    // twice the x-transform (see cell_solve3)
    cpx<T> c0{g[0], -k2 * (g[0] + g[1])};   // row b = 0
    cpx<T> c1{g[2], -k2 * (g[2] + g[3])};   // row b = 1
    cpx<T> fp, fm;
    fwd_pair(c0, c1, fp, fm);
    T P = fma(T(2), ax + ay, sig);
    T Qp = r2 * (ax + ay), Qm = r2 * (ax - ay);
    T P2 = P * P;
    const T den[2] = {fma(Qp, Qp, P2), fma(Qm, Qm, P2)};
    T inv[2];
    rcp_each(den, inv, std::integral_constant<int, 2>{});
    cpx<T> hp = cdiv(fp, P, Qp, inv[0]);
    cpx<T> hm = cdiv(fm, P, Qm, inv[1]);
    cpx<T> d0, d1;
    inv_pair(hp, hm, d0, d1);
    u[0] = d0.re;
    u[1] = fma(-r2, d0.im, -d0.re);
    u[2] = d1.re;
    u[3] = fma(-r2, d1.im, -d1.re);
}

// 3D cell solve in the reflected frame. g, u: nodes a + 2b + 4c.
template <typename T>
__device__ __forceinline__ void cell_solve3(const T g[8], T ax, T ay, T az, T sig, T u[8]) {
    const T k2 = T(2) * Consts<T>::k, r2 = Consts<T>::r2;
    // Twice the x-transform of the four (b, c) pencils: every later stage is
    // linear, so the coefficients stay doubled up to the back-transform, whose
    // real part of a conjugate pair (2 Re) then needs no factor 2.  Doubling
    // is exact in binary floating point, so the values are those of the plain
    // transform; it saves the multiplications by 1/2 and by 2.
    cpx<T> c1[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        c1[p].re = g[2 * p];
        c1[p].im = -k2 * (g[2 * p] + g[2 * p + 1]);
    }
    // y-transform: for c = 0, 1 -> (e_y = +, e_y = -)
    cpx<T> yp[2], ym[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) fwd_pair(c1[2 * c], c1[2 * c + 1], yp[c], ym[c]);
    // z-transform: for e_y = +, - -> (e_z = +, e_z = -)
    cpx<T> h[4];  // index: (e_y -) * 2 + (e_z -)
    fwd_pair(yp[0], yp[1], h[0], h[1]);
    fwd_pair(ym[0], ym[1], h[2], h[3]);
    T P = fma(T(2), ax + ay + az, sig);
    T P2 = P * P;
    T Q[4] = {r2 * (ax + ay + az), r2 * (ax + ay - az), r2 * (ax - ay + az), r2 * (ax - ay - az)};
    T den[4], inv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) den[e] = fma(Q[e], Q[e], P2);
    rcp_each(den, inv, std::integral_constant<int, 4>{});
#pragma unroll
    for (int e = 0; e < 4; ++e) h[e] = cdiv(h[e], P, Q[e], inv[e]);
    // inverse z: for e_y = +, - -> nodes c = 0, 1
    cpx<T> dp[2], dm[2];
    inv_pair(h[0], h[1], dp[0], dp[1]);
    inv_pair(h[2], h[3], dm[0], dm[1]);
    // inverse y for each c -> nodes b = 0, 1 ; inverse x -> real nodes a = 0, 1
    // (node 0 = 2 Re e, node 1 = 2 Re((-1 + i r2) e); e here is already 2 e)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        cpx<T> e0, e1;
        inv_pair(dp[c], dm[c], e0, e1);
        u[4 * c + 0] = e0.re;
        u[4 * c + 1] = fma(-r2, e0.im, -e0.re);
        u[4 * c + 2] = e1.re;
        u[4 * c + 3] = fma(-r2, e1.im, -e1.re);
    }
}

// Sum over a 64-lane wave by an xor butterfly: every lane receives the same
// sum, added in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// deterministic block reduction of three sums (blockDim.x a multiple of 64,
// at most 1024; sh: at least 48 doubles): the wave sums, then the waves in
// wave order
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* sh) {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[w] = a;
        sh[16 + w] = b;
        sh[32 + w] = c;
    }
    __syncthreads();
    a = sh[0];
    b = sh[16];
    c = sh[32];
    for (int k = 1; k < nw; ++k) {
        a += sh[k];
        b += sh[16 + k];
        c += sh[32 + k];
    }
    __syncthreads();
}

}  // namespace sn
