// Upwind DG of order p = 2, 3, 4 in 2D (Q_p on the Gauss-Lobatto nodes of each
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
// The sweep runs in tile planes (sweep_hp_kernel below; sweep_hp_shfl_kernel
// at p = 4).
#include <cstdlib>

#include "../../include/sn.h"
#include "sn_device.hpp"
#include "sn_kernels.hpp"
#include "hp.hpp"

namespace sn {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;  // 1 / (4 pi)

__device__ __forceinline__ int refl(int a, int r, int P) { return r ? P - a : a; }

// Workgroup barrier that orders LDS only.  The sweep's global stores (psi)
// are never read back by the workgroup that wrote them inside a launch, so
// the barrier between cell diagonals orders only the LDS faces.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A double moved across lanes by DPP (two 32-bit moves): quad_perm CTRL
// 0x55 a broadcasts lane a of every quad, row_ror CTRL 0x120 + n gives lane l
// of a 16-lane row the value of lane (l - n) mod 16 of that row.  Every
// source lane of these patterns exists, so bound_ctrl (zero for a missing
// source) never applies; set, it spares the move that would otherwise
// initialise each destination with the old value.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int A>
__device__ __forceinline__ double quad_bcast(double v) {
    return dpp_d<0x55 * A>(v);
}
template <int M>
__device__ __forceinline__ double row_rot(double v) {
    if constexpr (M == 0) return v;
    else return dpp_d<0x120 + 4 * M>(v);
}

// entry [k][a] of a table for a lane-dependent k (compile-time a): selects
// among the rows without indexing the table by a register
template <int N>
__device__ __forceinline__ double row_pick(const double (&t)[kHpMaxN][kHpMaxN], int k, int a) {
    double v = t[0][a];
#pragma unroll
    for (int kk = 1; kk < N; ++kk) v = k == kk ? t[kk][a] : v;
    return v;
}
template <int N>
__device__ __forceinline__ double vec_pick(const double (&t)[kHpMaxN], int k) {
    double v = t[0];
#pragma unroll
    for (int kk = 1; kk < N; ++kk) v = k == kk ? t[kk] : v;
    return v;
}

// Tile-plane sweep.  The mesh is cut into TS x TS tiles in each direction's
// frame; launch t sweeps the tiles with I + J = t (frame tile indices), one
// workgroup per (direction, tile), and the launches run in order, so a tile's
// upwind tiles are complete when it starts.  Inside its tile a workgroup walks
// the cell diagonals, a barrier between diagonals.  A cell is solved by a
// group of 16 lanes, one DPP row, lane 4 j + i holding node (i, j) of the
// frame (i along x) through every stage (at p = 2 the lanes with i or j = 3
// pad the 3 x 3 group): a transform along x gathers its line from the lane's
// quad (quad_perm broadcasts), one along y from the row rotated by 4, 8 and 12
// lanes (row_ror), all VALU moves, and every lane keeps the table rows of its
// own (i, j) in registers, those of the y stages in rotation order.  Upwind
// faces inside the tile come from LDS (written one diagonal earlier, double-
// buffered by diagonal parity, indexed by the tile-local x position); across a
// tile edge from psi (an earlier launch), at the domain edge from the inflow.
// All lanes of the block walk the chunks of a diagonal in step, so the
// shuffles always run with whole waves.  Every step issues the same list of
// global accesses with no per-lane branches: the next chunk's cell data
// (loaded ahead), one load per upwind face (from psi, the inflow or, where the
// value comes from LDS or is zero, a harmless address; the selection happens
// after the load) and the psi store.  Lanes past the diagonal's end work on its
// last cell, and the lanes past the last full group of a wave repeat the last
// group's last lane, so they store values identical to that cell's own lanes.
// gfx950 counts loads and stores in one in-order counter; with the same
// accesses at every step the waits are exact instead of a full drain per step
// (measured: a wait for every outstanding access before each step's face loads).
template <int P>
__global__ void __launch_bounds__(512) sweep_hp_kernel(HpTab tb, int nx, int ny, int ndirs, long nbf, int TS,
                                                       int tdiag, int nTx, int nTy,
                                                       const DirInfo* __restrict__ dirs,
                                                       const double* __restrict__ sigt,
                                                       const double* __restrict__ sigs,
                                                       const double* __restrict__ phi, const double* __restrict__ q,
                                                       const double* __restrict__ inflow, double* __restrict__ psi) {
    constexpr int N = P + 1, NN = N * N;
    constexpr int GPW = 4;  // cell groups per wave: one 16-lane DPP row each, lane 4 j + i
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gw = lane >> 4, r = lane & 15;
    const int gid = wave * GPW + gw, ngroups = (blockDim.x >> 6) * GPW;
    // this lane's node; at p = 2 the lanes with i or j = 3 pad the 3 x 3 group:
    // they use the clamped node for their addresses, add nothing (zero
    // coefficients) and store the clamped node's value
    const int i4 = r & 3, j4 = r >> 2;
    const bool pad = i4 > P || j4 > P;
    const int i0 = min(i4, P), j0 = min(j4, P);
    const int d = blockIdx.x % ndirs;
    const int It = max(0, tdiag - (nTy - 1)) + (int)(blockIdx.x / ndirs);
    const int Jt = tdiag - It;
    const DirInfo di = dirs[d];
    const double ax = di.ax, ay = di.ay;
    const int rx = di.rx, ry = di.ry;
    // this lane's table rows
    double w1r[N], w1i[N], w2r[N], w2i[N], v1r[N], v1i[N], v2r[N], v2i[N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
        w1r[a] = row_pick<N>(tb.Wr, i0, a);
        w1i[a] = row_pick<N>(tb.Wi, i0, a);
        w2r[a] = row_pick<N>(tb.Wr, j0, a);
        w2i[a] = row_pick<N>(tb.Wi, j0, a);
        v1r[a] = row_pick<N>(tb.Vr, i0, a);
        v1i[a] = row_pick<N>(tb.Vi, i0, a);
        v2r[a] = row_pick<N>(tb.Vr, j0, a);
        v2i[a] = row_pick<N>(tb.Vi, j0, a);
    }
    // the y stages take the line's values by row rotations, the m-th bringing
    // b = (j4 - m) mod 4, so their coefficients are stored in that order (zero
    // for the padding b = 3 at p = 2)
    double w2rr[4], w2ri[4], v2rr[4], v2ri[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        double a = 0.0, b = 0.0, c = 0.0, e = 0.0;
#pragma unroll
        for (int bb = 0; bb < N; ++bb) {
            const bool hit = ((j4 - m + 4) & 3) == bb;
            a = hit ? w2r[bb] : a;
            b = hit ? w2i[bb] : b;
            c = hit ? v2r[bb] : c;
            e = hit ? v2i[bb] : e;
        }
        w2rr[m] = a;
        w2ri[m] = b;
        v2rr[m] = c;
        v2ri[m] = e;
    }
    const double zr0 = ax * vec_pick<N>(tb.lr, i0) + ay * vec_pick<N>(tb.lr, j0);
    const double zi0 = ax * vec_pick<N>(tb.li, i0) + ay * vec_pick<N>(tb.li, j0);
    const double cx = ax * vec_pick<N>(tb.c0, i0), cy = ay * vec_pick<N>(tb.c0, j0);
    const int ip = refl(i0, rx, P), jp = refl(j0, ry, P);  // this lane's node in the physical numbering
    const int n_self = ip + N * jp;
    const int n_upx = refl(P, rx, P) + N * jp;              // the x-upwind neighbour's facing node
    const int n_upy = ip + N * refl(P, ry, P);              // the y-upwind neighbour's facing node
    // the tile in frame coordinates
    const int x0 = It * TS, y0 = Jt * TS;
    const int lx = min(TS, nx - x0), ly = min(TS, ny - y0);
    // LDS faces: x [2][TS + 1][N] (the face left of local position a at a), y [2][TS][N]
    extern __shared__ double lds[];
    double* xf = lds;
    double* yf = lds + 2 * (TS + 1) * N;
    const int kend = lx + ly - 2;
    auto first_of = [&](int kk) { return max(0, kk - (ly - 1)); };
    auto last_of = [&](int kk) { return min(kk, lx - 1); };
    auto cell_of = [&](int kk, int bb, int* irp, int* jrp) {
        const int a = min(bb + gid, last_of(kk));
        *irp = a;
        *jrp = kk - a;
        const int ir = x0 + a, jr = y0 + (kk - a);
        const int i = rx ? nx - 1 - ir : ir, j = ry ? ny - 1 - jr : jr;
        return (long)j * nx + i;
    };
    // absent phi or q: read sigma_t instead and scale by zero
    const double* php = phi ? phi : sigt;
    const double* qp = q ? q : sigt;
    const double phs = phi ? 1.0 : 0.0, qs = q ? 1.0 : 0.0;
    const int phm = phi ? NN : 1, pho = phi ? n_self : 0;
    // the global upwind values of a cell (tile edge: psi of the upwind tile,
    // written by an earlier launch; domain edge: the inflow; elsewhere an
    // unused load of sigma_t)
    auto face_ptrs = [&](long cc, int a, int b, const double** px, const double** py) {
        const int ir = x0 + a, jr = y0 + b;
        const int i = rx ? nx - 1 - ir : ir, j = ry ? ny - 1 - jr : jr;
        *px = (a == 0 && ir > 0) ? psi + ((cc + (rx ? 1 : -1)) * ndirs + d) * NN + n_upx
              : (ir == 0 && inflow ? inflow + (long)d * nbf + (long)j * N + jp : sigt + cc);
        *py = (b == 0 && jr > 0) ? psi + ((cc + (ry ? nx : -nx)) * ndirs + d) * NN + n_upy
              : (jr == 0 && inflow ? inflow + (long)d * nbf + (long)ny * N + (long)i * N + ip : sigt + cc);
    };
    // A chunk: its diagonal k, first position, this lane's cell and the data
    // loaded for it, one chunk ahead of the one being solved.  Two chunk
    // slots alternate (the loop runs two steps per turn), so the loaded data
    // is used where it was loaded instead of being copied each step.  Past
    // the last diagonal a chunk keeps the previous cell and loads it again.
    struct Chunk {
        int k, base, al, bl;
        long c;
        double st, ss, qq, ph, gx, gy;
    };
    auto advance = [&](const Chunk& h, Chunk& n) {
        n.k = h.k;
        n.base = h.base + ngroups;
        if (n.base > last_of(h.k)) {
            n.k = h.k + 1;
            n.base = first_of(n.k);
        }
        n.al = h.al;
        n.bl = h.bl;
        n.c = n.k <= kend ? cell_of(n.k, n.base, &n.al, &n.bl) : h.c;
        n.st = sigt[n.c];
        n.ss = sigs[n.c];
        n.qq = qs * qp[n.c];
        n.ph = phs * php[n.c * phm + pho];
        const double *px, *py;
        face_ptrs(n.c, n.al, n.bl, &px, &py);
        n.gx = *px;
        n.gy = *py;
    };
    // solve chunk C (its data loaded), store, and pass the faces on; Cn is the
    // chunk after it (a barrier when the diagonal changes)
    auto solve = [&](const Chunk& C, const Chunk& Cn) {
        const int k = C.k, al = C.al, bl = C.bl;
        const long c = C.c;
        const double st = C.st, ss = C.ss, qq = C.qq, ph = C.ph, gx = C.gx, gy = C.gy;
        const int ir = x0 + al, jr = y0 + bl;
        const int cur = k & 1, nxt = cur ^ 1;
        double f = pad ? 0.0 : (ss * ph + qq) * kInv4Pi;
        const double lx_ = xf[(cur * (TS + 1) + al) * N + j0];
        const double ly_ = yf[(cur * TS + al) * N + i0];
        const double upx = al > 0 ? lx_ : (ir > 0 || inflow ? gx : 0.0);
        const double upy = bl > 0 ? ly_ : (jr > 0 || inflow ? gy : 0.0);
        f = pad ? 0.0 : fma(cy, upy, fma(cx, upx, f));
        // along x: T(i, j) = sum_a W[i][a] f(a, j), the quad's lanes a
        const double fq[4] = {quad_bcast<0>(f), quad_bcast<1>(f), quad_bcast<2>(f), quad_bcast<3>(f)};
        double tr = 0.0, ti = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            tr = fma(w1r[a], fq[a], tr);
            ti = fma(w1i[a], fq[a], ti);
        }
        // along y: F(i, j) = sum_b W[j][b] T(i, b), the row rotated by 4 m
        const double xr[4] = {tr, row_rot<1>(tr), row_rot<2>(tr), row_rot<3>(tr)};
        const double xi[4] = {ti, row_rot<1>(ti), row_rot<2>(ti), row_rot<3>(ti)};
        double fr = 0.0, fi = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            fr = fma(w2rr[m], xr[m], fma(-w2ri[m], xi[m], fr));
            fi = fma(w2rr[m], xi[m], fma(w2ri[m], xr[m], fi));
        }
        // U = F / (a_x lambda_i0 + a_y lambda_j0 + sigma_t)
        const double zr = zr0 + st, zi = zi0;
        const double inv = rcp(zr * zr + zi * zi);
        const double ur = (fr * zr + fi * zi) * inv, ui = (fi * zr - fr * zi) * inv;
        // back along x: T2(i, j) = sum_k V[i][k] U(k, j)
        const double uq[4] = {quad_bcast<0>(ur), quad_bcast<1>(ur), quad_bcast<2>(ur), quad_bcast<3>(ur)};
        const double vq[4] = {quad_bcast<0>(ui), quad_bcast<1>(ui), quad_bcast<2>(ui), quad_bcast<3>(ui)};
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int kk = 0; kk < N; ++kk) {
            sr = fma(v1r[kk], uq[kk], fma(-v1i[kk], vq[kk], sr));
            si = fma(v1r[kk], vq[kk], fma(v1i[kk], uq[kk], si));
        }
        // back along y: u(i, j) = Re sum_l V[j][l] T2(i, l)
        const double yr[4] = {sr, row_rot<1>(sr), row_rot<2>(sr), row_rot<3>(sr)};
        const double yi[4] = {si, row_rot<1>(si), row_rot<2>(si), row_rot<3>(si)};
        double u = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) u = fma(v2rr[m], yr[m], fma(-v2ri[m], yi[m], u));
        if constexpr (P == 2) {
            // padding lanes take the value of their clamped node: lane i = 3 from
            // lane 2 of its quad, then row j = 3 from row 2 (rotation by 4)
            const double ux = dpp_d<0xA4>(u);  // quad_perm (0, 1, 2, 2)
            u = i4 > P ? ux : u;
            const double uy = row_rot<1>(u);
            u = j4 > P ? uy : u;
        }
        psi[(c * ndirs + d) * NN + n_self] = u;
        if (i0 == P) xf[(nxt * (TS + 1) + al + 1) * N + j0] = u;
        if (j0 == P) yf[(nxt * TS + al) * N + i0] = u;
        if (Cn.k != k) lds_barrier();
    };
    Chunk A, B;
    A.k = 0;
    A.base = 0;
    A.c = cell_of(0, 0, &A.al, &A.bl);
    {
        A.st = sigt[A.c];
        A.ss = sigs[A.c];
        A.qq = qs * qp[A.c];
        A.ph = phs * php[A.c * phm + pho];
        const double *px, *py;
        face_ptrs(A.c, A.al, A.bl, &px, &py);
        A.gx = *px;
        A.gy = *py;
    }
    for (;;) {
        advance(A, B);
        solve(A, B);
        if (B.k > kend) break;
        advance(B, A);
        solve(B, A);
        if (A.k > kend) break;
    }
}

// The same tile-plane sweep for p = 4, whose 25 nodes do not fit a 16-lane
// DPP row.  A cell is solved by a group of (p + 1)^2 lanes, lane
// g0 + i + (p + 1) j of the wave holding node (i, j) of the frame, two groups
// per wave; the 14 lanes past the second group repeat that group's last lane
// (same node, same values, same stores).  A transform along x gathers the
// p + 1 values of the lane's line from lanes g0 + a + (p + 1) j, one along y
// from lanes g0 + i + (p + 1) b, through a 64-slot LDS exchange area of the
// wave: each lane writes its (complex) value once and reads the p + 1 it
// needs (one 8- or 16-byte read each, against two to four 4-byte lane
// permutes per value).  The LDS operations of one wave execute in order, so
// a stage's write comes after every read of the stage before.  Cell data is
// loaded two chunks ahead (one at p = 2, 3: measured on the 256^2 S8 mesh,
// two ahead gives 2.70 -> 2.51 ms at p = 4 but 1.17 -> 1.22 ms at p = 3).
// The rest (tile planes, LDS faces inside a tile, uniform global accesses)
// is as in sweep_hp_kernel.
template <int P>
__global__ void __launch_bounds__(512) sweep_hp_shfl_kernel(HpTab tb, int nx, int ny, int ndirs, long nbf, int TS,
                                                            int tdiag, int nTx, int nTy,
                                                            const DirInfo* __restrict__ dirs,
                                                            const double* __restrict__ sigt,
                                                            const double* __restrict__ sigs,
                                                            const double* __restrict__ phi,
                                                            const double* __restrict__ q,
                                                            const double* __restrict__ inflow,
                                                            double* __restrict__ psi) {
    constexpr int N = P + 1, NN = N * N;
    constexpr int GPW = 64 / NN;  // cell groups per wave
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gw = min(lane / NN, GPW - 1), r = min(lane - gw * NN, NN - 1);
    const int gid = wave * GPW + gw, ngroups = (blockDim.x >> 6) * GPW;
    const int g0 = gw * NN;
    const int i0 = r % N, j0 = r / N;
    const int d = blockIdx.x % ndirs;
    const int It = max(0, tdiag - (nTy - 1)) + (int)(blockIdx.x / ndirs);
    const int Jt = tdiag - It;
    const DirInfo di = dirs[d];
    const double ax = di.ax, ay = di.ay;
    const int rx = di.rx, ry = di.ry;
    // this lane's table rows
    double w1r[N], w1i[N], w2r[N], w2i[N], v1r[N], v1i[N], v2r[N], v2i[N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
        w1r[a] = row_pick<N>(tb.Wr, i0, a);
        w1i[a] = row_pick<N>(tb.Wi, i0, a);
        w2r[a] = row_pick<N>(tb.Wr, j0, a);
        w2i[a] = row_pick<N>(tb.Wi, j0, a);
        v1r[a] = row_pick<N>(tb.Vr, i0, a);
        v1i[a] = row_pick<N>(tb.Vi, i0, a);
        v2r[a] = row_pick<N>(tb.Vr, j0, a);
        v2i[a] = row_pick<N>(tb.Vi, j0, a);
    }
    const double zr0 = ax * vec_pick<N>(tb.lr, i0) + ay * vec_pick<N>(tb.lr, j0);
    const double zi0 = ax * vec_pick<N>(tb.li, i0) + ay * vec_pick<N>(tb.li, j0);
    const double cx = ax * vec_pick<N>(tb.c0, i0), cy = ay * vec_pick<N>(tb.c0, j0);
    const int ip = refl(i0, rx, P), jp = refl(j0, ry, P);  // this lane's node in the physical numbering
    const int n_self = ip + N * jp;
    const int n_upx = refl(P, rx, P) + N * jp;              // the x-upwind neighbour's facing node
    const int n_upy = ip + N * refl(P, ry, P);              // the y-upwind neighbour's facing node
    // the tile in frame coordinates
    const int x0 = It * TS, y0 = Jt * TS;
    const int lx = min(TS, nx - x0), ly = min(TS, ny - y0);
    // LDS faces: x [2][TS + 1][N] (the face left of local position a at a), y [2][TS][N];
    // then the exchange areas, 64 complex slots per wave
    extern __shared__ double lds[];
    double* xf = lds;
    double* yf = lds + 2 * (TS + 1) * N;
    typedef double cx2 __attribute__((ext_vector_type(2)));
    cx2* xch = reinterpret_cast<cx2*>(lds + (2 * (TS + 1) + 2 * TS) * N) + wave * 64;
    const int kend = lx + ly - 2;
    auto first_of = [&](int kk) { return max(0, kk - (ly - 1)); };
    auto last_of = [&](int kk) { return min(kk, lx - 1); };
    auto cell_of = [&](int kk, int bb, int* irp, int* jrp) {
        const int a = min(bb + gid, last_of(kk));
        *irp = a;
        *jrp = kk - a;
        const int ir = x0 + a, jr = y0 + (kk - a);
        const int i = rx ? nx - 1 - ir : ir, j = ry ? ny - 1 - jr : jr;
        return (long)j * nx + i;
    };
    // absent phi or q: read sigma_t instead and scale by zero
    const double* php = phi ? phi : sigt;
    const double* qp = q ? q : sigt;
    const double phs = phi ? 1.0 : 0.0, qs = q ? 1.0 : 0.0;
    const int phm = phi ? NN : 1, pho = phi ? n_self : 0;
    // the global upwind values of a cell (tile edge: psi of the upwind tile,
    // written by an earlier launch; domain edge: the inflow; elsewhere an
    // unused load of sigma_t)
    auto face_ptrs = [&](long cc, int a, int b, const double** px, const double** py) {
        const int ir = x0 + a, jr = y0 + b;
        const int i = rx ? nx - 1 - ir : ir, j = ry ? ny - 1 - jr : jr;
        *px = (a == 0 && ir > 0) ? psi + ((cc + (rx ? 1 : -1)) * ndirs + d) * NN + n_upx
              : (ir == 0 && inflow ? inflow + (long)d * nbf + (long)j * N + jp : sigt + cc);
        *py = (b == 0 && jr > 0) ? psi + ((cc + (ry ? nx : -nx)) * ndirs + d) * NN + n_upy
              : (jr == 0 && inflow ? inflow + (long)d * nbf + (long)ny * N + (long)i * N + ip : sigt + cc);
    };
    // the line slots of this lane: along x (a, j0) and along y (i0, b)
    const int sx = g0 + N * j0, sy = g0 + i0;
    // A chunk: its diagonal k, first position, this lane's cell and the data
    // loaded for it.  Chunks are loaded two ahead of the one being solved
    // (cell data is read-only here and the upwind psi comes from earlier
    // launches), so a load has two steps to arrive.  Three chunk slots rotate
    // over a three-step loop, so the loaded data is used where it was loaded.
    // Past the last diagonal a chunk keeps the previous cell and loads it
    // again.
    struct Chunk {
        int k, base, al, bl;
        long c;
        double st, ss, qq, ph, gx, gy;
    };
    auto load = [&](Chunk& h) {
        h.st = sigt[h.c];
        h.ss = sigs[h.c];
        h.qq = qs * qp[h.c];
        h.ph = phs * php[h.c * phm + pho];
        const double *px, *py;
        face_ptrs(h.c, h.al, h.bl, &px, &py);
        h.gx = *px;
        h.gy = *py;
    };
    auto advance = [&](const Chunk& h, Chunk& n) {
        n.k = h.k;
        n.base = h.base + ngroups;
        if (n.base > last_of(h.k)) {
            n.k = h.k + 1;
            n.base = first_of(n.k);
        }
        n.al = h.al;
        n.bl = h.bl;
        n.c = n.k <= kend ? cell_of(n.k, n.base, &n.al, &n.bl) : h.c;
        load(n);
    };
    // solve chunk C0 (its data loaded), store, and pass the faces on; C1 is the
    // chunk after it (a barrier when the diagonal changes)
    auto solve = [&](const Chunk& C0, const Chunk& C1) {
        const int k = C0.k, al = C0.al, bl = C0.bl;
        const long c = C0.c;
        const double st = C0.st, ss = C0.ss, qq = C0.qq, ph = C0.ph, gx = C0.gx, gy = C0.gy;
        const int ir = x0 + al, jr = y0 + bl;
        const int cur = k & 1, nxt = cur ^ 1;
        double f = (ss * ph + qq) * kInv4Pi;
        const double lx_ = xf[(cur * (TS + 1) + al) * N + j0];
        const double ly_ = yf[(cur * TS + al) * N + i0];
        const double upx = al > 0 ? lx_ : (ir > 0 || inflow ? gx : 0.0);
        const double upy = bl > 0 ? ly_ : (jr > 0 || inflow ? gy : 0.0);
        f = fma(cx, upx, f);
        f = fma(cy, upy, f);
        // along x: T(i0, j0) = sum_a W[i0][a] f(a, j0)
        xch[lane].x = f;
        __builtin_amdgcn_wave_barrier();
        double tr = 0.0, ti = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            const double fa = xch[sx + a].x;
            tr = fma(w1r[a], fa, tr);
            ti = fma(w1i[a], fa, ti);
        }
        __builtin_amdgcn_wave_barrier();
        // along y: F(i0, j0) = sum_b W[j0][b] T(i0, b)
        xch[lane] = cx2{tr, ti};
        __builtin_amdgcn_wave_barrier();
        double fr = 0.0, fi = 0.0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const cx2 t = xch[sy + N * b];
            fr = fma(w2r[b], t.x, fma(-w2i[b], t.y, fr));
            fi = fma(w2r[b], t.y, fma(w2i[b], t.x, fi));
        }
        __builtin_amdgcn_wave_barrier();
        // U = F / (a_x lambda_i0 + a_y lambda_j0 + sigma_t)
        const double zr = zr0 + st, zi = zi0;
        const double inv = rcp(zr * zr + zi * zi);
        const double ur = (fr * zr + fi * zi) * inv, ui = (fi * zr - fr * zi) * inv;
        // back along x: T2(i0, j0) = sum_k V[i0][k] U(k, j0)
        xch[lane] = cx2{ur, ui};
        __builtin_amdgcn_wave_barrier();
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int kk = 0; kk < N; ++kk) {
            const cx2 t = xch[sx + kk];
            sr = fma(v1r[kk], t.x, fma(-v1i[kk], t.y, sr));
            si = fma(v1r[kk], t.y, fma(v1i[kk], t.x, si));
        }
        __builtin_amdgcn_wave_barrier();
        // back along y: u(i0, j0) = Re sum_l V[j0][l] T2(i0, l)
        xch[lane] = cx2{sr, si};
        __builtin_amdgcn_wave_barrier();
        double u = 0.0;
#pragma unroll
        for (int l = 0; l < N; ++l) {
            const cx2 t = xch[sy + N * l];
            u = fma(v2r[l], t.x, fma(-v2i[l], t.y, u));
        }
        __builtin_amdgcn_wave_barrier();
        psi[(c * ndirs + d) * NN + n_self] = u;
        if (i0 == P) xf[(nxt * (TS + 1) + al + 1) * N + j0] = u;
        if (j0 == P) yf[(nxt * TS + al) * N + i0] = u;
        if (C1.k != k) lds_barrier();
    };
    Chunk A, B, C;
    A.k = 0;
    A.base = 0;
    A.c = cell_of(0, 0, &A.al, &A.bl);
    load(A);
    advance(A, B);
    for (;;) {
        advance(B, C);
        solve(A, B);
        if (B.k > kend) break;
        advance(C, A);
        solve(B, C);
        if (C.k > kend) break;
        advance(A, B);
        solve(C, A);
        if (A.k > kend) break;
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
    // 16 x 16 tiles (smaller meshes: one tile per axis of the mesh's size;
    // SN_HP_TILE in the environment overrides the 16, at most 64).  Measured
    // on the 256^2 S8 mesh, order 2 / 3: tiles of 8 1.28 / 1.30 ms, 12 1.27 /
    // 1.29, 16 1.18 / 1.18, 24 1.42 / 1.63.  Enough waves for a tile's longest
    // diagonal, at most 8 (longer diagonals are walked in chunks).
    int tile = 16;
    if (const char* e = std::getenv("SN_HP_TILE")) tile = std::max(4, std::min(64, std::atoi(e)));
    const int TS = std::min(tile, std::max(nx, ny));
    const int nTx = (nx + TS - 1) / TS, nTy = (ny + TS - 1) / TS;
    const int n1 = tb.p + 1;
    // cell groups per wave: 16-lane DPP groups at p = 2, 3; two 25-lane groups at p = 4
    const int gpw = tb.p == 4 ? 64 / (n1 * n1) : 4;
    const int waves = std::max(1, std::min(8, (std::min(TS, std::min(nx, ny)) + gpw - 1) / gpw));
    // faces; at p = 4 also the waves' exchange areas (64 complex slots each)
    const size_t lds = (size_t)(2 * (TS + 1) + 2 * TS) * n1 * sizeof(double) +
                       (tb.p == 4 ? (size_t)waves * 64 * 2 * sizeof(double) : 0);
    for (int t = 0; t <= nTx + nTy - 2; ++t) {
        const int ntiles = std::min(t, nTx - 1) - std::max(0, t - (nTy - 1)) + 1;
        const dim3 grid((unsigned)(ntiles * ndirs));
        if (tb.p == 2)
            hipLaunchKernelGGL(sweep_hp_kernel<2>, grid, dim3(64 * waves), lds, st, tb, nx, ny, ndirs, nbf, TS, t, nTx,
                               nTy, dirs, sigt, sigs, phi, q, inflow, psi);
        else if (tb.p == 3)
            hipLaunchKernelGGL(sweep_hp_kernel<3>, grid, dim3(64 * waves), lds, st, tb, nx, ny, ndirs, nbf, TS, t, nTx,
                               nTy, dirs, sigt, sigs, phi, q, inflow, psi);
        else
            hipLaunchKernelGGL(sweep_hp_shfl_kernel<4>, grid, dim3(64 * waves), lds, st, tb, nx, ny, ndirs, nbf, TS, t,
                               nTx, nTy, dirs, sigt, sigs, phi, q, inflow, psi);
    }
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
    } else if (tb.p == 3) {
        if (op == SN_DIFFUSION_SIP) SN_HA(3, SN_DIFFUSION_SIP);
        else if (op == SN_DIFFUSION_NIP) SN_HA(3, SN_DIFFUSION_NIP);
        else SN_HA(3, SN_DIFFUSION_MNIP);
    } else {
        if (op == SN_DIFFUSION_SIP) SN_HA(4, SN_DIFFUSION_SIP);
        else if (op == SN_DIFFUSION_NIP) SN_HA(4, SN_DIFFUSION_NIP);
        else SN_HA(4, SN_DIFFUSION_MNIP);
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
    else if (nn == 16)
        hipLaunchKernelGGL(hp_spmv_kernel<16>, dim3(nb), dim3(256), 0, st, nthick, blk, col, x, b, y);
    else
        hipLaunchKernelGGL(hp_spmv_kernel<25>, dim3(nb), dim3(256), 0, st, nthick, blk, col, x, b, y);
    return hipGetLastError();
}

hipError_t launch_hp_block_inverse(int nn, int nthick, const double* blk, double* binv, int* bad, hipStream_t st) {
    if (nthick == 0) return hipSuccess;
    const int nb = blocks_of(nthick, 64);
    if (nn == 9)
        hipLaunchKernelGGL(hp_block_inverse_kernel<9>, dim3(nb), dim3(64), 0, st, nthick, blk, binv, bad);
    else if (nn == 16)
        hipLaunchKernelGGL(hp_block_inverse_kernel<16>, dim3(nb), dim3(64), 0, st, nthick, blk, binv, bad);
    else
        hipLaunchKernelGGL(hp_block_inverse_kernel<25>, dim3(nb), dim3(64), 0, st, nthick, blk, binv, bad);
    return hipGetLastError();
}

hipError_t launch_hp_block_apply(int nn, int nthick, const double* binv, const double* v, double* z, hipStream_t st) {
    if (nthick == 0) return hipSuccess;
    const int nb = blocks_of((long)nthick * nn, 256);
    if (nn == 9)
        hipLaunchKernelGGL(hp_block_apply_kernel<9>, dim3(nb), dim3(256), 0, st, nthick, binv, v, z);
    else if (nn == 16)
        hipLaunchKernelGGL(hp_block_apply_kernel<16>, dim3(nb), dim3(256), 0, st, nthick, binv, v, z);
    else
        hipLaunchKernelGGL(hp_block_apply_kernel<25>, dim3(nb), dim3(256), 0, st, nthick, binv, v, z);
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
    else if (tb.p == 3)
        hipLaunchKernelGGL(hp_rhs_kernel<3>, dim3(nb), dim3(256), 0, st, tb, nthick, hx, hy, thick_cell, sigma_t,
                           sigma_s, mass_kind, phi_old, phi_si, b);
    else
        hipLaunchKernelGGL(hp_rhs_kernel<4>, dim3(nb), dim3(256), 0, st, tb, nthick, hx, hy, thick_cell, sigma_t,
                           sigma_s, mass_kind, phi_old, phi_si, b);
    return hipGetLastError();
}

hipError_t launch_hp_band(int nn, int nthick, const double* blk, const int* col, int kl, int ldb, double* band,
                          hipStream_t st) {
    if (nthick == 0) return hipSuccess;
    const int nb = blocks_of((long)nthick * nn, 256);
    if (nn == 9)
        hipLaunchKernelGGL(hp_band_kernel<9>, dim3(nb), dim3(256), 0, st, nthick, blk, col, kl, ldb, band);
    else if (nn == 16)
        hipLaunchKernelGGL(hp_band_kernel<16>, dim3(nb), dim3(256), 0, st, nthick, blk, col, kl, ldb, band);
    else
        hipLaunchKernelGGL(hp_band_kernel<25>, dim3(nb), dim3(256), 0, st, nthick, blk, col, kl, ldb, band);
    return hipGetLastError();
}

}  // namespace sn
