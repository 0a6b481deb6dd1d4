// Transport sweeps (Section 1 and Section 2.2, eq. psi): for every direction d
// and every cell in upwind order, solve the upwind-DG cell problem with the
// already-computed upwind face values.  The local solve is sn::cell_solve2/3.
//
// 2D (latency bound: the dependency chain is nx + ny - 1 cells long):
//   one workgroup per direction; lane r of wave w owns local row 64 w + r and
//   walks along x, skewed by its row index, so that at step t it works on
//   column t - row.  The x inflow of a cell is the previous cell of the same
//   lane (registers); the y inflow is the top face of the row below, taken
//   from lane r - 1 by a DPP wave shift, or from the previous wave through
//   an LDS ring (one barrier per B2D steps).  Rows beyond ROWS2D are processed
//   in chunks, one launch per chunk, chained through a y-face buffer.
//
// 3D (throughput bound): tiles of TX x 4 x 4 cells in the reflected frame of
//   each direction; one wave per (tile, group of four directions with the
//   same reflection); lane (jy, kz, k) owns the
//   x-pencil (jy, kz) of a 4 x 4 pencil block for four directions and walks
//   along x skewed by jy + kz, taking its y inflow from lane - 1 and its z
//   inflow from lane - 4 by DPP row shifts.  Tiles on one diagonal plane I + J + K = p are independent, so
//   each plane is one launch; tile faces travel through face buffers in the
//   reflected frame (slot 0 of each buffer holds the domain inflow).
//
// Node order in memory is global (a + 2b + 4c); in the reflected frame node
// n_local = n_global ^ M with M = rx + 2 ry + 4 rz, a compile-time constant
// of each kernel body.
#include <type_traits>
#include <utility>

#include "sn_kernels.hpp"

namespace sn {

// v of lane - 1 across the wave; lane 0 receives `old`
__device__ __forceinline__ double wave_shr1_old(double v, double old) {
    const long long x = __double_as_longlong(v), y = __double_as_longlong(old);
    int lo = (int)(x & 0xffffffffLL), hi = (int)(x >> 32);
    int olo = (int)(y & 0xffffffffLL), ohi = (int)(y >> 32);
    lo = __builtin_amdgcn_update_dpp(olo, lo, 0x138, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(ohi, hi, 0x138, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float wave_shr1_old(float v, float old) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x138, 0xF, 0xF, false));
}

// ---------------------------------------------------------------------------
// face-buffer initialisation from the domain inflow (or zero)
// ---------------------------------------------------------------------------
// inflow layout per direction (global frame): x face ((k*ny + j)*F + b + 2c),
// y face ((k*nx + i)*F + a + 2c), z face ((j*nx + i)*F + a + 2b).
template <typename T>
__global__ void init_faces_kernel(int dim, int nx, int ny, int nz, int ndirs, const DirInfo* __restrict__ dirs,
                                  int transpose, const double* __restrict__ inflow, long nbf, T* __restrict__ xf,
                                  long xstride, T* __restrict__ yf, long ystride, T* __restrict__ zf,
                                  long zstride) {
    const int F = dim == 2 ? 2 : 4;
    const long nxf = (long)ny * nz, nyf = (long)nx * nz, nzf = (long)nx * ny;
    const long per = dim == 3 ? nxf : nxf + nyf;  // 3D: x faces only (y and z: init_yz_faces_kernel)
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long total = per * ndirs;
    for (; idx < total; idx += (long)gridDim.x * blockDim.x) {
        int d = (int)(idx / per);
        long f = idx % per;
        DirInfo di = dirs[d];
        int rx = di.rx ^ transpose, ry = di.ry ^ transpose, rz = (dim == 3) ? (di.rz ^ transpose) : 0;
        const double* in = inflow ? inflow + (long)d * nbf : nullptr;
        if (f < nxf) {  // x face, local (kl, jl)
            int jl = (int)(f % ny), kl = (int)(f / ny);
            int j = ry ? ny - 1 - jl : jl, k = rz ? nz - 1 - kl : kl;
            for (int t = 0; t < F; ++t) {
                int b = (t & 1) ^ ry, c = ((t >> 1) & 1) ^ rz;
                double v = in ? in[((long)k * ny + j) * F + b + 2 * c] : 0.0;
                xf[d * xstride + f * F + t] = T(v);
            }
        } else if (f < nxf + nyf) {  // y face, local (kl, il)
            long g = f - nxf;
            int il = (int)(g % nx), kl = (int)(g / nx);
            int i = rx ? nx - 1 - il : il, k = rz ? nz - 1 - kl : kl;
            for (int t = 0; t < F; ++t) {
                int a = (t & 1) ^ rx, c = ((t >> 1) & 1) ^ rz;
                double v = in ? in[nxf * F + ((long)k * nx + i) * F + a + 2 * c] : 0.0;
                yf[d * ystride + g * F + t] = T(v);
            }
        } else {  // z face, local (jl, il)
            long g = f - nxf - nyf;
            int il = (int)(g % nx), jl = (int)(g / nx);
            int i = rx ? nx - 1 - il : il, j = ry ? ny - 1 - jl : jl;
            for (int t = 0; t < 4; ++t) {
                int a = (t & 1) ^ rx, b = ((t >> 1) & 1) ^ ry;
                double v = in ? in[(nxf + nyf) * 4 + ((long)j * nx + i) * 4 + a + 2 * b] : 0.0;
                zf[d * zstride + g * 4 + t] = T(v);
            }
        }
    }
}

// The boundary face slots of the 3D y and z faces (yface_slot layout): the y
// half of every tile with J = 0 and the z half of every tile with K = 0, from
// the inflow (zero where inflow is null, the direction slot is empty or the
// position lies outside the tile or the mesh).
template <typename T>
__global__ void init_yz_faces_kernel(int nx, int ny, int nz, int TX, int nTx, int nTy, int nTz, int ngroups,
                                     const int* __restrict__ groups, const DirInfo* __restrict__ dirs, int transpose,
                                     const double* __restrict__ inflow, long nbf, T* __restrict__ yz) {
    const long nxf = (long)ny * nz, nyf = (long)nx * nz;
    const int slots = TX + 3;
    const long side_y = (long)nTx * nTz, side_z = (long)nTx * nTy;  // boundary tiles per group
    const long per_group = (side_y + side_z) * slots * 64;
    const long total = per_group * ngroups;
    const long ntiles = (long)nTx * nTy * nTz;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int g = (int)(idx / per_group);
        long r = idx - (long)g * per_group;
        const int v = (int)(r & 63);
        r >>= 6;
        const int q = (int)(r % slots);
        const long bt = r / slots;
        const bool yside = bt < side_y;
        int I, J, K;
        if (yside) {
            I = (int)(bt / nTz);
            K = (int)(bt % nTz);
            J = 0;
        } else {
            I = (int)((bt - side_y) / nTy);
            J = (int)((bt - side_y) % nTy);
            K = 0;
        }
        const int kd = v >> 4, kq = (v >> 2) & 3, t = v & 3;
        const int d = groups[6 * g + kd];
        const int i0 = I * TX, len = min(TX, nx - i0);
        const int ir = q - kq;
        double val = 0.0;
        if (inflow && d >= 0 && ir >= 0 && ir < len) {
            const DirInfo di = dirs[d];
            const int rx = di.rx ^ transpose, ry = di.ry ^ transpose, rz = di.rz ^ transpose;
            const int il = i0 + ir;
            const int i = rx ? nx - 1 - il : il;
            const double* in = inflow + (long)d * nbf;
            if (yside) {
                const int kl = K * 4 + kq;
                if (kl < nz) {
                    const int k = rz ? nz - 1 - kl : kl;
                    const int a = (t & 1) ^ rx, c = ((t >> 1) & 1) ^ rz;
                    val = in[nxf * 4 + ((long)k * nx + i) * 4 + a + 2 * c];
                }
            } else {
                const int jl = J * 4 + kq;
                if (jl < ny) {
                    const int j = ry ? ny - 1 - jl : jl;
                    const int a = (t & 1) ^ rx, b = ((t >> 1) & 1) ^ ry;
                    val = in[(nxf + nyf) * 4 + ((long)j * nx + i) * 4 + a + 2 * b];
                }
            }
        }
        const long tl = ((long)I * nTy + J) * nTz + K;
        yz[(((long)g * ntiles + tl) * slots + q) * YZ_SLOT + (yside ? 0 : YZ_SLOT / 2) + v] = T(val);
    }
}

// ---------------------------------------------------------------------------
// vector loads and stores
// ---------------------------------------------------------------------------
template <typename T>
struct Vec4 {
    T v[4];
};

template <typename T>
__device__ __forceinline__ Vec4<T> load4(const T* p) {
    Vec4<T> r;
    if constexpr (sizeof(T) == 8) {
        const double2* q = reinterpret_cast<const double2*>(p);
        double2 a = q[0], b = q[1];
        r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
    } else {
        float4 a = *reinterpret_cast<const float4*>(p);
        r.v[0] = a.x; r.v[1] = a.y; r.v[2] = a.z; r.v[3] = a.w;
    }
    return r;
}

template <typename T>
__device__ __forceinline__ void store4(T* p, T a0, T a1, T a2, T a3) {
    if constexpr (sizeof(T) == 8) {
        double2* q = reinterpret_cast<double2*>(p);
        q[0] = make_double2(a0, a1);
        q[1] = make_double2(a2, a3);
    } else {
        *reinterpret_cast<float4*>(p) = make_float4(a0, a1, a2, a3);
    }
}

// ---------------------------------------------------------------------------
// 2D diagonal-major input layout
// ---------------------------------------------------------------------------
// For the quadrant with reflection (rx, ry), local cell (il, jl) of the
// reflected frame lies on diagonal il + jl.  A wave owns the 64 rows
// jl = 64 b + l (l = lane) of one row block b and at a given step works on
// one diagonal of it, so each block is stored as a parallelogram
// [s][l], s = il + l in [0, nx + 63): every load of a wave is one contiguous
// run instead of one cache line per lane, and only the two 64 x 64 ramp
// triangles are padding (entries off the mesh are zero).
// out: [4 quadrants][ceil(ny / 64) blocks][nx + 63][64][nn].
template <typename T>
__global__ void skew2d_kernel(int nx, int ny, int nn, const T* __restrict__ in, T* __restrict__ out) {
    const long ns = (long)nx + 63;
    const long nb = (ny + 63) / 64;
    const long per = nb * ns * 64;
    const long total = 4 * per;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        const int q = (int)(idx / per);
        const long e = idx - q * per;
        const int l = (int)(e & 63);
        const long bs = e >> 6;
        const int b = (int)(bs / ns), sd = (int)(bs - (long)b * ns);
        const int il = sd - l, jl = 64 * b + l;
        T* o = out + idx * nn;
        if (il >= 0 && il < nx && jl < ny) {
            const int i = (q & 1) ? nx - 1 - il : il;
            const int j = (q & 2) ? ny - 1 - jl : jl;
            const T* src = in + ((long)j * nx + i) * nn;
            for (int n = 0; n < nn; ++n) o[n] = src[n];
        } else {
            for (int n = 0; n < nn; ++n) o[n] = T(0);
        }
    }
}

// Source of the 2D sweep written straight into the diagonal-major arrays:
// the source (sigma_s f + q) / 4pi of cell c from its four flux values f,
// written to the cell's place in the diagonal-major arrays of all four
// quadrants
template <typename T>
__device__ __forceinline__ void put_source_skew2d(int nx, int ny, long c, double sigs, double qc, const double f[4],
                                                  T* __restrict__ out) {
    const long ns = (long)nx + 63;
    const long per = (long)((ny + 63) / 64) * ns * 64;
    const int i = (int)(c % nx), j = (int)(c / nx);
    T v[4];
    for (int n = 0; n < 4; ++n) v[n] = T((sigs * f[n] + qc) * 0.07957747154594766788);  // 1 / 4pi
    for (int qd = 0; qd < 4; ++qd) {
        const int il = (qd & 1) ? nx - 1 - i : i;
        const int jl = (qd & 2) ? ny - 1 - j : j;
        const int l = jl & 63;
        T* o = out + (qd * per + ((long)(jl >> 6) * ns + il + l) * 64 + l) * 4;
        for (int n = 0; n < 4; ++n) o[n] = v[n];
    }
}

// s = (sigma_s (phi - phi_prev) + q) / 4pi per node (one thread per cell),
// stored at the cell's position in each quadrant's layout.  Only on-mesh
// entries are written; the padding of the arrays is zeroed once when they
// are allocated.
template <typename T>
__global__ void source_skew2d_kernel(int nx, int ny, const double* __restrict__ sigma_s,
                                     const double* __restrict__ phi, const double* __restrict__ phi_prev,
                                     const double* __restrict__ q, T* __restrict__ out) {
    const long nc = (long)nx * ny;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (long)gridDim.x * blockDim.x) {
        double f[4];
        for (int n = 0; n < 4; ++n) {
            f[n] = phi ? phi[c * 4 + n] : 0.0;
            if (phi_prev) f[n] -= phi_prev[c * 4 + n];
        }
        put_source_skew2d<T>(nx, ny, c, sigma_s[c], q ? q[c] : 0.0, f, out);
    }
}

// 2D source iteration: the DSA's final update phi_out = phi_SI + P x fused
// with the next iteration's FP64 sweep source from phi_out (one kernel and
// one launch fewer between the solve and the next sweep)
__global__ void scatter_source_skew2d_kernel(int nx, int ny, const int* __restrict__ slot_of_cell,
                                             const double* __restrict__ phi_si, const double* __restrict__ x,
                                             const double* __restrict__ sigma_s, const double* __restrict__ q,
                                             double* __restrict__ phi_out, double* __restrict__ out) {
    const long nc = (long)nx * ny;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (long)gridDim.x * blockDim.x) {
        const int s = slot_of_cell[c];
        double f[4];
        for (int n = 0; n < 4; ++n) {
            f[n] = phi_si[c * 4 + n];
            if (s >= 0) f[n] += x[(long)s * 4 + n];
            phi_out[c * 4 + n] = f[n];
        }
        put_source_skew2d<double>(nx, ny, c, sigma_s[c], q ? q[c] : 0.0, f, out);
    }
}

// ---------------------------------------------------------------------------
// 2D pipelined sweep
// ---------------------------------------------------------------------------
// Inputs of one cell for one lane, loaded ahead of use.
template <typename T>
struct In2 {
    Vec4<T> s;
    T sig, yb0, yb1;
};

// The LDS buffers reach the sweep bodies as plain pointers; these casts give
// them back the LDS address space, so that the compiler emits LDS
// instructions (ds_read / ds_write) rather than flat ones, which wait on both
// the memory and the LDS counters.
template <typename T>
using lds_t = __attribute__((address_space(3))) T;
using dvec2 = double __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ lds_t<T>* as_lds(T* p) {
    return (lds_t<T>*)p;
}

// Pipeline constants of the 2D sweep: the input prefetch ring depth, and the
// number of steps between workgroup barriers (also the unroll of the step
// loop).  Wave w runs B2D w steps behind the plain diagonal schedule, so the
// top row of wave w - 1 produces the value that the bottom row of wave w
// needs B2D + 1 steps before it is needed.  The values travel through a ring
// of 2 B2D LDS slots; with one barrier per B2D steps, every window of B2D
// consecutive steps holds exactly one barrier, which orders each write before
// its read (done one step early, to hide the LDS latency) and each read
// before the slot is rewritten.
constexpr int R2D = 4;
constexpr int B2D = 8;
static_assert(B2D % R2D == 0, "the prefetch ring must wrap at chunk boundaries");

// f(integral_constant<int, K>) for K = 0, 1, ... in order
template <typename F, int... K>
__device__ __forceinline__ void unroll_seq(F&& f, std::integer_sequence<int, K...>) {
    (f(std::integral_constant<int, K>{}), ...);
}

// LDS of one 2D sweep workgroup.
template <typename T>
struct Lds2 {
    // FP64: double-buffered psi stage, see sweep2d_wave
    T stage[sizeof(T) == 8 ? 2 : 1][ROWS2D][4];
    // y outflow of the top row of each wave, one slot per step
    T ring[2 * B2D][ROWS2D / 64][2];
    // every lane writes the ring; the lanes below the top one write here (one
    // pair per lane, moved by the same slot offset), so the write needs no
    // lane mask
    T discard[64 + (2 * B2D - 1) * (ROWS2D / 64)][2];
};

// Roles of a wave in the 2D sweep: the bottom wave takes its y inflow from
// the chunk's inflow row in memory, the others from the wave below through
// the LDS ring; the top wave of a chunk that has a chunk above also writes
// the y outflow of its top row to memory.
enum { W2_FIRST = 0, W2_MID = 1, W2_TOPOUT = 2 };

// One wave of the 2D sweep.  Lane l owns row r = 64 w + l of the chunk and,
// at step t, cell il = t - r - B2D w of it.  The wave is busy only in its
// window of LEN steps starting at ts = (64 + B2D) w, in which it reads
// diagonal k = t - ts of its row block, a contiguous run of the
// diagonal-major arrays; outside the window it only takes part in the
// barriers.  Cells outside the row (il < 0 or il >= nx) are computed on
// padding and discarded: their y outflow reaches only lanes that are outside
// their row as well, their x outflow is not kept before the row starts, and
// their psi stores are masked.
// In FP64 the four psi values of a lane (32 bytes) go through a
// double-buffered LDS stage so that two lanes write the two 16-byte halves
// of one cell's block (one cache line per cell per store instruction instead
// of one per lane); the write-out of step k happens during step k + 1,
// behind its arithmetic.  Store addresses move by a fixed stride per step.
template <typename T, int M, int ROLE>
__device__ __forceinline__ void sweep2d_wave(int nx, int ny, int ndirs, int d, T ax, T ay,
                                             const T* __restrict__ sigq, const T* __restrict__ srcq,
                                             const T* __restrict__ xf, const T* __restrict__ yin_buf,
                                             T* __restrict__ yout_buf, int row0, int nrows, T* __restrict__ psi,
                                             Lds2<T>* L, int wave, int nw) {
    constexpr int rx = M & 1, ry = (M >> 1) & 1;
    constexpr int PR = ROWS2D / 64;  // ring pairs per slot
    const int lane = threadIdx.x & 63;
    const int r = wave * 64 + lane;
    const bool rowok = r < nrows;
    const int jl = row0 + min(r, nrows - 1);
    const int j = ry ? ny - 1 - jl : jl;
    const int ns = nx + 63;
    const int LEN = (ns + 1 + B2D - 1) / B2D * B2D;  // >= ns + 1: the last step writes out psi
    const int ts = wave * (64 + B2D);
    const int NT = (nw - 1) * (64 + B2D) + LEN;
    // this wave's row block in the diagonal-major arrays (uniform) and the lane's column
    const long blk = (long)((row0 >> 6) + wave) * ns;
    const T* sbase = srcq + blk * 256;
    const T* gbase = sigq + blk * 64;
    T xin0 = xf[(long)jl * 2 + 0];
    T xin1 = xf[(long)jl * 2 + 1];
    T yo0 = T(0), yo1 = T(0);
    T rin0 = T(0), rin1 = T(0);  // y inflow of lane 0 from the wave below, read one step early
    const lds_t<T>* rd = as_lds(&L->ring[0][max(wave - 1, 0)][0]);
    lds_t<T>* wr = lane == 63 ? as_lds(&L->ring[0][wave][0]) : as_lds(&L->discard[lane][0]);
    if constexpr (ROLE != W2_FIRST) {
        for (int b = 0; b + 1 < ts / B2D; ++b) __syncthreads();
        // the value for step ts, written by wave - 1 at step ts - 1 - B2D
        const int sl = (ts - 1 - B2D) & (2 * B2D - 1);
        rin0 = rd[sl * PR * 2 + 0];
        rin1 = rd[sl * PR * 2 + 1];
        __syncthreads();
    }
    auto fetch = [&](int k, In2<T>& v) {
        v.s = load4(sbase + (long)k * 256 + lane * 4);
        v.sig = gbase[(long)k * 64 + lane];
        if constexpr (ROLE == W2_FIRST) {
            const int c = min(k, nx - 1);
            v.yb0 = yin_buf[(long)c * 2 + 0];
            v.yb1 = yin_buf[(long)c * 2 + 1];
        }
    };
    // psi store addresses at k = 0, moved by sgn_step per step; a store is
    // done when (unsigned)(k - v) < nx (v = a huge negative for rows past nrows)
    const long dstep = (long)ndirs * 4;
    const long sgn_step = rx ? -dstep : dstep;
    constexpr int OFF = -(1 << 30);
    T* wp0;
    T* wp1;
    int v0, v1;
    const lds_t<T>* st0 = nullptr;
    const lds_t<T>* st1 = nullptr;
    if constexpr (sizeof(T) == 8) {
        // lane pair (2 q, 2 q + 1) stores the halves o = lane & 1 of cell q =
        // 32 h + lane / 2 of the wave (step k writes out the cells of step k - 1)
        auto half = [&](int h, T*& wp, int& v, const lds_t<T>*& sp) {
            const int q = 32 * h + (lane >> 1), o = lane & 1, rq = wave * 64 + q;
            const int jq0 = row0 + min(rq, nrows - 1);
            const int jq = ry ? ny - 1 - jq0 : jq0;
            const long i0 = rx ? (long)(nx + q) : (long)(-1 - q);
            wp = psi + ((long)jq * nx * ndirs + d) * 4 + 2 * o + i0 * dstep;
            v = rq < nrows ? 1 + q : OFF;
            sp = as_lds(&L->stage[0][rq][2 * o]);
        };
        half(0, wp0, v0, st0);
        half(1, wp1, v1, st1);
    } else {
        const long i0 = rx ? (long)(nx - 1 + lane) : (long)(-lane);
        wp0 = psi + ((long)j * nx * ndirs + d) * 4 + i0 * dstep;
        v0 = rowok ? lane : OFF;
        wp1 = nullptr;
        v1 = OFF;
    }
    lds_t<T>* stw = as_lds(&L->stage[0][r][0]);
    const T ax4 = T(4) * ax, ax2 = T(2) * ax, ay4 = T(4) * ay, ay2 = T(2) * ay;
    // step k of the window (slot base sb = (ts + k - kk) & B2D, kk = k mod B2D);
    // FULL: every lane of the wave is inside its row at this step and at the
    // previous one (no store masks, no hold of the x inflow)
    auto step = [&](int k, int sb, auto kkc, auto fullc, In2<T>& use, In2<T>& fill) {
        constexpr int kk = decltype(kkc)::value;
        constexpr bool FULL = decltype(fullc)::value;
        fetch(k + R2D - 1, fill);
        dvec2 prev0{}, prev1{};
        if constexpr (sizeof(T) == 8) {
            constexpr int par = (kk + 1) & 1;  // stage buffer of step k - 1
            prev0 = *reinterpret_cast<const lds_t<dvec2>*>(st0 + par * ROWS2D * 4);
            prev1 = *reinterpret_cast<const lds_t<dvec2>*>(st1 + par * ROWS2D * 4);
        }
        // y inflow: the lane below (DPP); lane 0 keeps the DPP's old value,
        // the wave below's top row (ring) or the chunk's inflow row
        const T old0 = ROLE == W2_FIRST ? use.yb0 : rin0;
        const T old1 = ROLE == W2_FIRST ? use.yb1 : rin1;
        const T yi0 = wave_shr1_old(yo0, old0), yi1 = wave_shr1_old(yo1, old1);
        if constexpr (ROLE != W2_FIRST) {
            // the value for step k + 1, written by wave - 1 B2D steps ago
            const int sl = (sb ^ B2D) + kk;
            rin0 = rd[sl * PR * 2 + 0];
            rin1 = rd[sl * PR * 2 + 1];
        }
        T g[4], u[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) g[n] = use.s.v[n ^ M];
        // x inflow face (a' = 0), y inflow face (b' = 0)
        g[0] = fma(ax4, xin0, g[0]);
        g[1] = fma(-ax2, xin0, g[1]);
        g[2] = fma(ax4, xin1, g[2]);
        g[3] = fma(-ax2, xin1, g[3]);
        g[0] = fma(ay4, yi0, g[0]);
        g[2] = fma(-ay2, yi0, g[2]);
        g[1] = fma(ay4, yi1, g[1]);
        g[3] = fma(-ay2, yi1, g[3]);
        cell_solve2(g, ax, ay, use.sig, u);
        if constexpr (FULL) {
            xin0 = u[1];
            xin1 = u[3];
        } else {
            const bool started = k >= lane;  // il >= 0: keep the row's x inflow until then
            xin0 = started ? u[1] : xin0;
            xin1 = started ? u[3] : xin1;
        }
        yo0 = u[2];
        yo1 = u[3];
        if constexpr (sizeof(T) == 8) {
            // the unconditional stage write consumes the solve, so the solve
            // stays ahead of the write-out of the previous step
            constexpr int par = kk & 1;
            lds_t<dvec2>* sw = reinterpret_cast<lds_t<dvec2>*>(stw + par * ROWS2D * 4);
            sw[0] = dvec2{u[0 ^ M], u[1 ^ M]};
            sw[1] = dvec2{u[2 ^ M], u[3 ^ M]};
            if (FULL || (unsigned)(k - v0) < (unsigned)nx) *reinterpret_cast<dvec2*>(wp0) = prev0;
            if (FULL || (unsigned)(k - v1) < (unsigned)nx) *reinterpret_cast<dvec2*>(wp1) = prev1;
            wp0 += sgn_step;
            wp1 += sgn_step;
        } else {
            if (FULL || (unsigned)(k - v0) < (unsigned)nx) store4(wp0, u[0 ^ M], u[1 ^ M], u[2 ^ M], u[3 ^ M]);
            wp0 += sgn_step;
        }
        if constexpr (ROLE == W2_TOPOUT) {
            // lane 63 of the top wave is the chunk's top row (the chunk is full)
            if (lane == 63 && (unsigned)(k - 63) < (unsigned)nx) {
                yout_buf[(long)(k - 63) * 2 + 0] = yo0;
                yout_buf[(long)(k - 63) * 2 + 1] = yo1;
            }
        }
        const int slw = sb + kk;
        wr[slw * PR * 2 + 0] = yo0;
        wr[slw * PR * 2 + 1] = yo1;
    };
    In2<T> sl[R2D];
#pragma unroll
    for (int k = 0; k + 1 < R2D; ++k) fetch(k, sl[k]);
    // one chunk of B2D steps; step k uses ring slot k % R2D and refills the
    // slot of step k + R2D - 1 (B2D is a multiple of R2D)
    auto chunk = [&](int k0, auto fullc) {
        const int sb = (ts + k0) & B2D;
        unroll_seq(
            [&](auto kc) {
                constexpr int kk = decltype(kc)::value;
                step(k0 + kk, sb, kc, fullc, sl[kk % R2D], sl[(kk + R2D - 1) % R2D]);
            },
            std::make_integer_sequence<int, B2D>{});
        __syncthreads();
    };
    // chunks [64, kf) have every lane inside its row (il = k - lane in
    // [0, nx) at k and at k - 1) when the wave's rows are all in the chunk
    const int kf = (wave + 1) * 64 <= nrows ? max(64, nx / B2D * B2D) : 0;
    for (int k0 = 0; k0 < LEN; k0 += B2D) {
        if (k0 >= 64 && k0 < kf) chunk(k0, std::true_type{});
        else chunk(k0, std::false_type{});
    }
    for (int t = ts + LEN; t < NT; t += B2D) __syncthreads();
}

// blockIdx.x: position in dir_order (directions of one quadrant are placed
// on the same XCDs, whose L2 then holds that quadrant's arrays); one launch
// per row chunk.  psi: [cell][pstride][4], direction index d (or, with local,
// the workgroup's position in dir_order).  sigskew / srcskew: the diagonal-major arrays of the four
// quadrants (skew2d_kernel layout).
template <typename T>
__global__ void __launch_bounds__(ROWS2D) sweep2d_kernel(int nx, int ny, int ndirs, const DirInfo* __restrict__ dirs,
                                                       const int* __restrict__ dir_order,
                                                       int transpose, const T* __restrict__ sigskew,
                                                       const T* __restrict__ srcskew, const T* __restrict__ xf,
                                                       long xstride, T* __restrict__ ybuf, long ystride, int chunk,
                                                       int nchunk, int row0, int nrows, T* __restrict__ psi,
                                                       int pstride, int local) {
    __shared__ __align__(16) Lds2<T> L;
    const int d = dir_order[blockIdx.x];
    // direction index of this workgroup in psi: the global one, or (local)
    // its position in dir_order, for a psi holding only those directions
    const int dpsi = local ? (int)blockIdx.x : d;
    const DirInfo di = dirs[d];
    const int m = (di.rx ^ transpose) | ((di.ry ^ transpose) << 1);
    const T ax = T(di.ax), ay = T(di.ay);
    const long per = (long)((ny + 63) / 64) * (nx + 63) * 64;
    const T* sq = sigskew + m * per;
    const T* cq = srcskew + m * per * 4;
    const T* xfd = xf + d * xstride;
    const T* yin = ybuf + d * ystride + (long)chunk * nx * 2;
    T* yout = (chunk + 1 < nchunk) ? ybuf + d * ystride + (long)(chunk + 1) * nx * 2 : nullptr;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = (nrows + 63) / 64;
#define SN_WAVE2(MM, RR) \
    sweep2d_wave<T, MM, RR>(nx, ny, pstride, dpsi, ax, ay, sq, cq, xfd, yin, yout, row0, nrows, psi, &L, wave, nw)
#define SN_CASE2(MM)                                      \
    case MM:                                              \
        if (wave == 0) SN_WAVE2(MM, W2_FIRST);            \
        else if (yout && wave == nw - 1) SN_WAVE2(MM, W2_TOPOUT); \
        else SN_WAVE2(MM, W2_MID);                        \
        break;
    switch (m) {
        SN_CASE2(0)
        SN_CASE2(1)
        SN_CASE2(2)
        SN_CASE2(3)
    }
#undef SN_CASE2
#undef SN_WAVE2
}

// ---------------------------------------------------------------------------
// 3D tile-plane sweep
// ---------------------------------------------------------------------------
// Lane layout: lane = p + 16 k, pencil p = jy + 4 kz of a 4 x 4 block of
// x-pencils, k = one of four directions that share the reflection M.  The
// y-upwind pencil is lane - 1 and the z-upwind pencil lane - 4, both inside
// the same 16-lane DPP row, so the face values move with row_shr DPP moves.
// The four lanes of one pencil read the same cell (one cache line serves four
// directions) and write its four consecutive directions of psi (contiguous).
template <typename T>
struct Vec8 {
    T v[8];
};

template <typename T>
__device__ __forceinline__ Vec8<T> load8(const T* p) {
    Vec8<T> r;
    Vec4<T> a = load4(p), b = load4(p + 4);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        r.v[n] = a.v[n];
        r.v[n + 4] = b.v[n];
    }
    return r;
}

// v of lane - SHIFT within the 16-lane row (row_shr DPP); lanes without a
// source inside the row receive 0 and take their value from a face buffer
template <int SHIFT>
__device__ __forceinline__ double row_shr(double v) {
    const long long x = __double_as_longlong(v);
    int lo = (int)(x & 0xffffffffLL), hi = (int)(x >> 32);
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x110 + SHIFT, 0xF, 0xF, true);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x110 + SHIFT, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int SHIFT>
__device__ __forceinline__ float row_shr(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + SHIFT, 0xF, 0xF, true));
}

template <typename T>
struct In3 {
    Vec8<T> s;
    T sig;
    Vec4<T> y, z;  // y- and z-face inflow (lanes on the tile's y = 0 / z = 0 side)
};

// Sums over the four direction rows of a pencil of eight values v[0..7],
// reduce-scattered: lane (p, k) receives the sums of nodes nb and nb + 1,
// nb = 2 (k >> 1) + 4 (k & 1).  The first permlane16 swap pairs rows 0-1 and
// 2-3, exchanging nodes 4..7 of the even row for nodes 0..3 of the odd row,
// so an even row keeps partial sums of nodes 0..3 and an odd row of 4..7;
// the permlane32 swap then pairs the two halves the same way.  Every sum is
// (v0 + v1) + (v2 + v3) over the rows, in a fixed order.  (The gfx950
// permlane swaps exchange the odd rows of their first operand with the even
// rows of the second, and the upper half of the first with the lower half of
// the second.)
__device__ __forceinline__ double swap_sum16(double a, double b) {
    const unsigned long long x = (unsigned long long)__double_as_longlong(a);
    const unsigned long long y = (unsigned long long)__double_as_longlong(b);
    const auto l = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)y, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap((unsigned)(x >> 32), (unsigned)(y >> 32), false, false);
    return __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0])) +
           __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
}
__device__ __forceinline__ double swap_sum32(double a, double b) {
    const unsigned long long x = (unsigned long long)__double_as_longlong(a);
    const unsigned long long y = (unsigned long long)__double_as_longlong(b);
    const auto l = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)y, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap((unsigned)(x >> 32), (unsigned)(y >> 32), false, false);
    return __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0])) +
           __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
}
__device__ __forceinline__ void rows_sum8(const double v[8], double& r0, double& r1) {
    double c[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) c[n] = swap_sum16(v[n], v[n + 4]);
    r0 = swap_sum32(c[0], c[2]);
    r1 = swap_sum32(c[1], c[3]);
}

// fused sweep + moment: steps per workgroup barrier
constexpr int RF = 4;

// The tile's source and sigma_t, staged in LDS once per workgroup: every wave
// of a block sweeps the same cells (one reflection class, different
// directions), so the per-step loads of the waves become LDS reads of one
// copy, loaded with contiguous runs (a pencil's cells are consecutive in
// memory).  Layout [x][pencil][SRCP] in the reflected frame, nodes in memory
// order; the pencil stride is padded by 16 bytes so that the 16 pencils of
// one x fall on different LDS bank groups.
// Only the FP64 kernels stage (measured: FP64 -4% psi sweep, -5% fused; the
// FP32 fused sweep was 6% slower, so FP32 loads its inputs directly).
constexpr int TXMAX = 32;  // longest tile along x
template <typename T>
constexpr bool staged_tile() {
    return sizeof(T) == 8;
}
template <typename T>
constexpr int src_pencil() {
    return 8 + 16 / (int)sizeof(T);
}
template <typename T>
struct TileIn {
    static constexpr int NX = staged_tile<T>() ? TXMAX : 1;
    T s[NX][16][src_pencil<T>()];
    T sig[NX][16];
};
template <typename T>
__device__ __forceinline__ const lds_t<T>* as_lds(const T* p) {
    return (const lds_t<T>*)p;
}
// all threads of the block take part; the caller synchronises afterwards
template <typename T>
__device__ __forceinline__ void stage_tile(int nx, int ny, int nz, int m, int I, int J, int K, int TX,
                                           const T* __restrict__ sigt, const T* __restrict__ src, TileIn<T>* t) {
    const int rx = m & 1, ry = (m >> 1) & 1, rz = (m >> 2) & 1;
    const int i0 = I * TX, len = min(TX, nx - i0);
    const int ilo = rx ? nx - i0 - len : i0;  // lowest x of the tile's cells in memory
    lds_t<T>* ts = as_lds(&t->s[0][0][0]);
    lds_t<T>* tg = as_lds(&t->sig[0][0]);
    const int per = len * 8;
    for (int e = threadIdx.x; e < 16 * per; e += blockDim.x) {
        const int q = e / per, r = e - q * per;
        const int xm = r >> 3, n = r & 7;  // position in the pencil's memory run
        const int qjl = J * 4 + (q & 3), qkl = K * 4 + (q >> 2);
        T v = T(0);
        if (qjl < ny && qkl < nz) {
            const int qj = ry ? ny - 1 - qjl : qjl, qk = rz ? nz - 1 - qkl : qkl;
            v = src[(((long)qk * ny + qj) * nx + ilo + xm) * 8 + n];
        }
        const int ir = rx ? len - 1 - xm : xm;
        ts[(ir * 16 + q) * src_pencil<T>() + n] = v;
    }
    for (int e = threadIdx.x; e < 16 * len; e += blockDim.x) {
        const int q = e / len, xm = e - q * len;
        const int qjl = J * 4 + (q & 3), qkl = K * 4 + (q >> 2);
        T v = T(0);
        if (qjl < ny && qkl < nz) {
            const int qj = ry ? ny - 1 - qjl : qjl, qk = rz ? nz - 1 - qkl : qkl;
            v = sigt[((long)qk * ny + qj) * nx + ilo + xm];
        }
        const int ir = rx ? len - 1 - xm : xm;
        tg[ir * 16 + q] = v;
    }
}



// The psi stage of a wave: 16 pencil blocks of four directions x eight values
// each, a block padded by 16 bytes.  Lane (pencil p, direction k) writes its
// eight values at p * STAGE_PENCIL + 8 k; unpadded, the blocks of consecutive
// pencils lie 256 (FP64) or 128 (FP32) bytes apart and the eight lanes of one
// LDS pass all hit the same four banks (an eight-way conflict on every write;
// measured at C5: bank-conflict cycles five times the LDS-active cycles).
// With the padding the eight lanes fall on eight distinct bank groups.
template <typename T>
constexpr int stage_pencil() {
    return 32 + 16 / (int)sizeof(T);
}
template <typename T>
constexpr int stage_elems() {
    return 16 * stage_pencil<T>();
}

// FUSED = false: psi is stored.  FUSED = true (source iteration): psi is not
// stored; every step the lanes' w_d psi (FP64) is summed over the four
// directions of a pencil (rows_sum8), the 16 pencil sums of each wave go to an
// LDS ring red[2 RF][waves][16][8], and every RF steps, after a workgroup
// barrier, the workgroup adds the waves' sums in wave order and stores the
// octant's share of phi for those cells (each cell is visited once per
// octant, so plain stores suffice and the result does not depend on timing).
// Face stores of the branching body: raw buffer stores from the wave's face
// slot base, every lane every step; a lane with nothing to store gets offset
// 0x80000000, outside the resource's range, and the hardware drops its store.
// With no store inside a per-lane branch the compiler counts the step's
// memory operations exactly.  The base must be the same for the whole wave
// (it is read from the first lane).
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t face_rsrc(const T* base) {
    const unsigned long long a = (unsigned long long)base;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void*)(((unsigned long long)hi << 32) | lo), 0, 0x7fffffff,
                                             0x00020000);
}
template <typename T>
__device__ __forceinline__ void face_store4(__amdgpu_buffer_rsrc_t r, unsigned off, T a0, T a1, T a2, T a3) {
    if constexpr (sizeof(T) == 8) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b128(d2{a0, a1}, r, (int)off, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b128(d2{a2, a3}, r, (int)(off + 16u), 0, 0);
    } else {
        typedef float f4 __attribute__((ext_vector_type(4)));
        __builtin_amdgcn_raw_buffer_store_b128(f4{a0, a1, a2, a3}, r, (int)off, 0, 0);
    }
}

template <typename T, int M, bool FUSED = false>
__device__ __forceinline__ void sweep3d_body(int nx, int ny, int nz, int ndirs, int d, bool dok, T ax, T ay, T az,
                                             int I, int J, int K, int TX, int nTx, int nTy, int nTz,
                                             const TileIn<T>* tin, const T* __restrict__ sigt,
                                             const T* __restrict__ src, T* __restrict__ xf, T* __restrict__ yzt,
                                             T* __restrict__ psi, int d0, int nvalid, T* __restrict__ stg,
                                             double wgt = 0.0, double* __restrict__ red = nullptr,
                                             double* __restrict__ phio = nullptr, int nwaves = 0) {
    constexpr int rx = M & 1, ry = (M >> 1) & 1, rz = (M >> 2) & 1;
    const int lane = threadIdx.x & 63;
    const int jy = lane & 3, kz = (lane >> 2) & 3;
    const int jl = J * 4 + jy, kl = K * 4 + kz;
    const bool pen = dok && jl < ny && kl < nz;
    const int jc = min(jl, ny - 1), kc = min(kl, nz - 1);
    const int j = ry ? ny - 1 - jc : jc, k = rz ? nz - 1 - kc : kc;
    const int i0 = I * TX;
    const int len = min(TX, nx - i0);
    T xin[4], yo[4], zo[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        xin[t] = T(0);
        yo[t] = T(0);
        zo[t] = T(0);
    }
    if (pen) {
        Vec4<T> x = load4(xf + (((long)I * nz + kl) * ny + jl) * 4);
#pragma unroll
        for (int t = 0; t < 4; ++t) xin[t] = x.v[t];
    }
    const long rowbase = ((long)k * ny + j) * nx;
    // Addresses are formed from per-lane bases at the tile's first cell
    // (position ir = 0 along the pencil) plus a multiple of the step, so the
    // step loop does no 64-bit index arithmetic.  cdir: cells per step in
    // memory along x.
    constexpr int cdir = rx ? -1 : 1;
    const int skew = jy + kz;  // lane's pencil lags the tile's first pencil by skew steps
    // this lane's pencil in the LDS tile (FP64), or its cells in memory (FP32)
    const lds_t<T>* tsrc = as_lds(&tin->s[0][lane & 15][0]);
    const lds_t<T>* tsig = as_lds(&tin->sig[0][lane & 15]);
    const long c0 = rowbase + (rx ? nx - 1 - i0 : i0);
    const T* src0 = src + c0 * 8;
    const T* sig0 = sigt + c0;
    // y/z face inflow of the lane's cell at position ir of its pencil: slot
    // ir + kz (y) or ir + jy (z) of the tile's face slots (yface_slot)
    const int kd = lane >> 4;
    const T* yin0 = yzt + kz * YZ_SLOT + (kd * 4 + kz) * 4;
    const T* zin0 = yzt + jy * YZ_SLOT + YZ_SLOT / 2 + (kd * 4 + jy) * 4;
    // The source, sigma_t and the y/z face inflow of the next cell are loaded
    // one step ahead.  The face values of this tile were written by earlier
    // launches (the upwind tiles) and no tile of this launch writes them, so
    // they can be read at any time.  Every lane loads its face pieces, not
    // only the lanes on the tile's near sides that use them: yin0 does not
    // depend on jy nor zin0 on kz, so the other lanes read the same addresses
    // (no extra traffic), and slot kz + irc (or jy + irc) <= TX + 2 lies in
    // the tile's TX + 3 slots of its group, which the face buffer holds for
    // every group slot.  With the loads outside per-lane branches the
    // compiler counts them exactly instead of draining every access before
    // each use (C5 fused sweep: FP64 9.32 -> 8.38 ms, FP32 6.03 -> 5.57 ms,
    // bit-identical).
    auto fetch = [&](int ir, In3<T>& v) {
        const int irc = min(max(ir, 0), len - 1);
        if constexpr (!staged_tile<T>()) {
            v.s = load8(src0 + cdir * irc * 8);
            v.sig = sig0[cdir * irc];
        } else if constexpr (FUSED) {
            const lds_t<T>* sp = tsrc + irc * (16 * src_pencil<T>());
#pragma unroll
            for (int n = 0; n < 8; ++n) v.s.v[n] = sp[n];
            v.sig = tsig[irc * 16];
        }
        v.y = load4(yin0 + irc * YZ_SLOT);
        v.z = load4(zin0 + irc * YZ_SLOT);
    };
    // face outflow of the tile's top pencils (position il = i0 + s - skew at
    // step s) and of the last cell of each pencil
    const bool ystore = pen && jy == 3 && J + 1 < nTy;
    const bool zstore = pen && kz == 3 && K + 1 < nTz;
    const bool xstore = pen && I + 1 < nTx;
    // outflow at step s into slot s - 3 of the downstream tiles (J + 1: nTz
    // tiles on, K + 1: the next tile); the pointers are formed at step 0 and
    // used from step 3 on
    // (byte offsets from yzt, at most 1023 tiles x 35 slots x 1 KiB: below 2^31)
    const __amdgpu_buffer_rsrc_t rfz = face_rsrc<T>(yzt);
    const unsigned yob = (unsigned)((((long)nTz * (TX + 3) - 3) * YZ_SLOT + (kd * 4 + kz) * 4) * sizeof(T));
    const unsigned zob = (unsigned)(((long)TX * YZ_SLOT + YZ_SLOT / 2 + (kd * 4 + jy) * 4) * sizeof(T));
    constexpr unsigned kSlotBytes = YZ_SLOT * sizeof(T);
    T* xout = xf + (((long)(I + 1) * nz + kl) * ny + jl) * 4;
    // psi write-out through the LDS stage (nvalid > 0): pass it of the wave
    // covers the 64 consecutive 16-byte pieces it * 64 + lane of the 16
    // pencils' blocks of nvalid * 8 values; wsk: the pencil's skew (a huge
    // value where the lane has no piece), woff: the piece's LDS offset, wp:
    // its address at the current step, moved by wstride per step
    constexpr int CH = 16 / sizeof(T);  // values per 16-byte piece
    constexpr int NIT = 8 / CH;         // passes for four directions
    const long wstride = (long)cdir * ndirs * 8;
    int wsk[NIT], woff[NIT];
    T* wp[NIT];
    if constexpr (!FUSED) {
        const int per = nvalid * 8 / CH;  // pieces per pencil block
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int id = it * 64 + lane;
            wsk[it] = 1 << 29;
            woff[it] = 0;
            wp[it] = psi;
            if (nvalid > 0 && id < 16 * per) {
                const int q = id / per, o = id - q * per;
                const int qy = q & 3, qz = q >> 2;
                const int qjl = J * 4 + qy, qkl = K * 4 + qz;
                if (qjl < ny && qkl < nz) {
                    const int qj = ry ? ny - 1 - qjl : qjl;
                    const int qk = rz ? nz - 1 - qkl : qkl;
                    const long qc0 = ((long)qk * ny + qj) * nx + (rx ? nx - 1 - i0 : i0);
                    wsk[it] = qy + qz;
                    woff[it] = q * stage_pencil<T>() + o * CH;
                    wp[it] = psi + (qc0 * ndirs + d0) * 8 + o * CH - (long)(qy + qz) * wstride;
                }
            }
        }
    }
    const T ax4 = T(4) * ax, ax2 = T(2) * ax, ay4 = T(4) * ay, ay2 = T(2) * ay, az4 = T(4) * az, az2 = T(2) * az;
    const int nsteps = len + 6;
    auto step = [&](int s, In3<T>& use, In3<T>& fill) {
        const int ir = s - skew;
        fetch(ir + 1, fill);
        T yi[4], zi[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            yi[t] = row_shr<1>(yo[t]);
            zi[t] = row_shr<4>(zo[t]);
        }
        const bool active = pen && ir >= 0 && ir < len;
        double acc[8];
        if constexpr (FUSED) {
#pragma unroll
            for (int n = 0; n < 8; ++n) acc[n] = 0.0;
        }
        if (active) {
            const int il = i0 + ir;
            if (jy == 0) {
#pragma unroll
                for (int t = 0; t < 4; ++t) yi[t] = use.y.v[t];
            }
            if (kz == 0) {
#pragma unroll
                for (int t = 0; t < 4; ++t) zi[t] = use.z.v[t];
            }
            const int i = rx ? nx - 1 - il : il;
            const long c = rowbase + i;
            T g[8], u[8], sg;
            if constexpr (staged_tile<T>() && !FUSED) {
                // psi kernel: read from the LDS tile when used, not a step
                // ahead, which keeps the source out of the prefetch registers
                // (three waves per SIMD fit, so two workgroups per CU)
                const lds_t<T>* sp = tsrc + ir * (16 * src_pencil<T>());
#pragma unroll
                for (int n = 0; n < 8; ++n) g[n] = sp[n ^ M];
                sg = tsig[ir * 16];
            } else {
#pragma unroll
                for (int n = 0; n < 8; ++n) g[n] = use.s.v[n ^ M];
                sg = use.sig;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                // x face: local nodes (0, t) += 4 ax xin, (1, t) -= 2 ax xin ; t = b + 2c
                const int nx0 = 2 * t;
                g[nx0] = fma(ax4, xin[t], g[nx0]);
                g[nx0 + 1] = fma(-ax2, xin[t], g[nx0 + 1]);
                // y face: t = a + 2c -> nodes a + 4c (b = 0) and a + 2 + 4c (b = 1)
                const int ny0 = (t & 1) + 4 * (t >> 1);
                g[ny0] = fma(ay4, yi[t], g[ny0]);
                g[ny0 + 2] = fma(-ay2, yi[t], g[ny0 + 2]);
                // z face: t = a + 2b -> nodes t (c = 0) and t + 4 (c = 1)
                g[t] = fma(az4, zi[t], g[t]);
                g[t + 4] = fma(-az2, zi[t], g[t + 4]);
            }
            cell_solve3(g, ax, ay, az, sg, u);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                xin[t] = u[2 * t + 1];
                yo[t] = u[(t & 1) + 2 + 4 * (t >> 1)];
                zo[t] = u[t + 4];
            }
            T o[8];
#pragma unroll
            for (int n = 0; n < 8; ++n) o[n] = u[n ^ M];
            if constexpr (FUSED) {
#pragma unroll
                for (int n = 0; n < 8; ++n) acc[n] = wgt * (double)o[n];
            } else if (nvalid > 0) {
                // staged: this lane's eight values go to LDS slot (pencil, k)
                lds_t<T>* sp = as_lds(stg) + (lane & 15) * stage_pencil<T>() + (lane >> 4) * 8;
#pragma unroll
                for (int n = 0; n < 8; ++n) sp[n] = o[n];
            } else {
                T* pp = psi + (c * ndirs + d) * 8;
                store4(pp, o[0], o[1], o[2], o[3]);
                store4(pp + 4, o[4], o[5], o[6], o[7]);
            }
        }
        face_store4<T>(rfz, active && ystore ? yob + (unsigned)s * kSlotBytes : 0x80000000u, yo[0], yo[1], yo[2],
                       yo[3]);
        face_store4<T>(rfz, active && zstore ? zob + (unsigned)s * kSlotBytes : 0x80000000u, zo[0], zo[1], zo[2],
                       zo[3]);
        if constexpr (FUSED) {
            const int wave = threadIdx.x >> 6;
            lds_t<double>* rs = as_lds(red) + ((s % (2 * RF)) * nwaves + wave) * 128;
            double r0, r1;
            rows_sum8(acc, r0, r1);
            {
                const int kr = lane >> 4;
                *reinterpret_cast<lds_t<dvec2>*>(rs + (lane & 15) * 8 + 2 * (kr >> 1) + 4 * (kr & 1)) =
                    dvec2{r0, r1};
            }
            if ((s + 1) % RF == 0 || s == nsteps - 1) {
                // a barrier ordering LDS only: the waves exchange nothing
                // else inside a launch
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                __builtin_amdgcn_s_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                // the steps sb .. s of this batch: 128 (pencil, node) sums each
                const int sb = s - s % RF;
                const int nwork = (s - sb + 1) * 128;
                // (the block is nwaves waves: blockDim.x would be a load from
                // the dispatch packet, and its wait would drain every access in
                // flight)
                for (int id = threadIdx.x; id < nwork; id += nwaves * 64) {
                    const int sj = sb + (id >> 7), q = (id >> 3) & 15, n = id & 7;
                    const lds_t<double>* rq = as_lds(red) + (sj % (2 * RF)) * nwaves * 128 + q * 8 + n;
                    double sum = 0.0;
                    for (int w = 0; w < nwaves; ++w) sum += rq[w * 128];
                    const int qy = q & 3, qz = q >> 2;
                    const int qjl = J * 4 + qy, qkl = K * 4 + qz;
                    const int qir = sj - (qy + qz);
                    if (qjl < ny && qkl < nz && qir >= 0 && qir < len) {
                        const int qil = i0 + qir;
                        const int qi = rx ? nx - 1 - qil : qil;
                        const int qj = ry ? ny - 1 - qjl : qjl;
                        const int qk = rz ? nz - 1 - qkl : qkl;
                        phio[(((long)qk * ny + qj) * nx + qi) * 8 + n] = sum;
                    }
                }
            }
        } else if (nvalid > 0) {
            // Write the staged psi of the 16 pencils: pencil q's block is the
            // nvalid consecutive directions d0.. of its current cell, nvalid*8
            // contiguous values, and consecutive lanes write consecutive
            // 16-byte pieces of it, so neighbouring lanes store neighbouring
            // bytes.  LDS operations of one wave execute in order, so the
            // reads below see this step's writes.
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                if ((unsigned)(s - wsk[it]) < (unsigned)len) {
                    const lds_t<T>* sp = as_lds(stg) + woff[it];
                    // psi is written once per sweep and not read back by this
                    // kernel: nontemporal stores keep it from displacing the
                    // face and source data in the caches
                    if constexpr (sizeof(T) == 8) {
                        typedef double d2v __attribute__((ext_vector_type(2)));
                        typedef __attribute__((address_space(3))) d2v lds_d2v;
                        __builtin_nontemporal_store(*reinterpret_cast<const lds_d2v*>(sp),
                                                    reinterpret_cast<d2v*>(wp[it]));
                    } else {
                        typedef float f4v __attribute__((ext_vector_type(4)));
                        typedef __attribute__((address_space(3))) f4v lds_f4v;
                        __builtin_nontemporal_store(*reinterpret_cast<const lds_f4v*>(sp),
                                                    reinterpret_cast<f4v*>(wp[it]));
                    }
                }
                wp[it] += wstride;
            }
            __builtin_amdgcn_wave_barrier();
        }
    };
    In3<T> s0, s1;
    fetch(-skew, s0);
    for (int s = 0; s < nsteps; s += 2) {
        step(s, s0, s1);
        if (s + 1 < nsteps) step(s + 1, s1, s0);
    }
    // the x outflow of the pencil's last cell, which xin holds after its row
    if (xstore) store4(xout, xin[0], xin[1], xin[2], xin[3]);
}

// ---------------------------------------------------------------------------
// 3D psi sweep without branches around memory operations
// ---------------------------------------------------------------------------
// In sweep3d_body the face loads and every store sit inside per-lane
// conditions (the lane's cell is inside the tile at this step, it is a face
// lane, its psi piece is valid).  gfx950 counts loads and stores in one
// in-order counter (vmcnt), and across such branches the compiler cannot tell
// how many operations a step issued, so each step waits for all of them
// (s_waitcnt vmcnt(0)): the face inflow of a step waited for the previous
// step's psi and face stores to be acknowledged.  Measured at C5 (FP64): the
// psi sweep takes 8.7 ms with the face loads left out against 15.4 ms with
// them.  This body issues the same fixed list of memory operations at every
// step, so the counts are exact and a step waits only for what it uses:
//   * one 16-byte face piece per lane is loaded two steps ahead: the y and z
//     face inflow of the wave's four directions for that step (FP64: 64
//     pieces; FP32: 32, the other lanes idle), then moved through a small LDS
//     area to the lanes on the tile's y = 0 and z = 0 sides;
//   * the y and z face outflow of the step goes the opposite way: the lanes on
//     the tile's far sides put it in the LDS area and every lane stores one
//     piece;
//   * psi pieces go out through the LDS stage as in sweep3d_body;
//   * the x face is loaded before the loop and stored after it.
// Loads and stores use raw buffer resources with a wave-uniform base and a
// per-lane byte offset; a lane with nothing to load or store gets the offset
// kOOB, outside the resource's range, and the hardware's range check turns
// the load into zeros and drops the store without touching memory.  The
// faces of a direction are one block (x, y, z regions) so that a single
// resource from the wave's first direction covers both faces of its four
// directions; valid offsets stay below 2^31 bytes (checked on the host,
// SweepGeom::buf), and each wave's directions must be consecutive.
constexpr unsigned kOOB = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, 0x00020000);
}
template <typename T>
struct Piece;  // a 16-byte piece of T values
template <>
struct Piece<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Piece<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <typename T>
using piece_t = typename Piece<T>::type;
template <typename T>
using lds_piece_t = __attribute__((address_space(3))) piece_t<T>;
// Cache policy (the aux operand: bit 0 sc0, bit 1 nt, bit 4 sc1).  psi is
// written once and never read back in the sweep: nontemporal (2).  A face
// piece is written once and read once, by the downstream tile in the next
// plane's launch: stores at device scope (sc1, 16) and nontemporal loads (2),
// so that neither keeps face lines in L2 beside the tile's source and sigma_t.
// Measured at C5 against default caching on both, A/B in one process: FP64
// 9.31 -> 8.53 ms, FP32 6.80 -> 6.27 ms (the loads give most of the FP64 gain).
constexpr int kPsiStore = 2, kFaceStore = 16, kFaceLoad = 2;
template <typename T, int AUX>
__device__ __forceinline__ void buf_store_piece(__amdgpu_buffer_rsrc_t r, unsigned off, piece_t<T> v) {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, AUX);
}
template <typename T>
__device__ __forceinline__ piece_t<T> buf_load_piece(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, kFaceLoad);
}
template <typename T>
constexpr int face_pieces() {  // 16-byte pieces per four face values
    return (int)sizeof(T) / 4;
}
template <typename T>
constexpr int face_stage_elems() {  // the face area of a wave: 64 pieces
    return 64 * 16 / (int)sizeof(T);
}

// rf: face resource at the wave's first direction's face block (fstride
// elements per direction; y and z regions at yoff and zoff within a block);
// xd: this lane's direction's x-face region.  rpsi: psi resource at the
// tile's lowest cell (cell_base) and the wave's first psi direction.  slots:
// bit k set when the wave's direction slot k is used.
template <typename T, int M>
__device__ __forceinline__ void sweep3d_body_buf(int nx, int ny, int nz, int pstride, unsigned slots, bool dok, T ax,
                                                 T ay, T az, int I, int J, int K, int TX, int nTx, int nTy, int nTz,
                                                 const TileIn<T>* tin, const T* __restrict__ sigt,
                                                 const T* __restrict__ src, T* __restrict__ xd,
                                                 __amdgpu_buffer_rsrc_t rf, __amdgpu_buffer_rsrc_t rpsi,
                                                 long cell_base, int nvalid,
                                                 T* __restrict__ stg, T* __restrict__ fstg) {
    constexpr int rx = M & 1, ry = (M >> 1) & 1, rz = (M >> 2) & 1;
    constexpr int sz = (int)sizeof(T);
    constexpr int CH = 16 / sz;                  // values per 16-byte piece
    constexpr int NIT = 8 / CH;                  // psi passes for four directions
    constexpr int NPK = face_pieces<T>();        // pieces per four face values
    constexpr int NYP = 16 * NPK;                // y-face pieces of a step (z: as many)
    const int lane = threadIdx.x & 63;
    const int jy = lane & 3, kz = (lane >> 2) & 3, kd = lane >> 4;
    const int jl = J * 4 + jy, kl = K * 4 + kz;
    const bool pen = dok && jl < ny && kl < nz;
    const int jc = min(jl, ny - 1), kc = min(kl, nz - 1);
    const int j = ry ? ny - 1 - jc : jc, k = rz ? nz - 1 - kc : kc;
    const int i0 = I * TX;
    const int len = min(TX, nx - i0);
    const int skew = jy + kz;
    T xin[4], yo[4], zo[4];
    {
        const Vec4<T> x = load4(xd + (((long)I * nz + kc) * ny + jc) * 4);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            xin[t] = x.v[t];
            yo[t] = T(0);
            zo[t] = T(0);
        }
    }
    constexpr int cdir = rx ? -1 : 1;
    const long rowbase = ((long)k * ny + j) * nx;
    const long c0 = rowbase + (rx ? nx - 1 - i0 : i0);
    const T* src0 = src + c0 * 8;
    const T* sig0 = sigt + c0;
    const lds_t<T>* tsrc = as_lds(&tin->s[0][lane & 15][0]);
    const lds_t<T>* tsig = as_lds(&tin->sig[0][lane & 15]);
    // The face piece of this lane: piece q of the y face (q < NYP) or of the
    // z face, for direction slot fk and side position fq (the kz of a y-face
    // lane, the jy of a z-face lane), half fh of the four values.  The lane on
    // the near side that receives it lags the tile's first pencil by fq steps,
    // the far-side lane that sends it by fq + 3.
    const bool isy = lane < NYP, isz = !isy && lane < 2 * NYP;
    const int fqq = isy ? lane : lane - NYP;
    const int fk = fqq / (4 * NPK), fq = (fqq / NPK) & 3, fh = fqq % NPK;
    const bool fslot = (isy || isz) && ((slots >> (fk & 3)) & 1u);
    const bool fin_ok = fslot && (isy ? K * 4 + fq < nz : J * 4 + fq < ny);
    const bool fout_ok = fslot && (isy ? (J + 1 < nTy && K * 4 + fq < nz) : (K + 1 < nTz && J * 4 + fq < ny));
    // Face slots (yface_slot): the receiving lane takes slot s at step s, and
    // the sending lane writes slot s - 3 of the downstream tile (J + 1: nTz
    // tiles on, K + 1: the next tile) at step s; piece `lane` of a slot is
    // this lane's piece.  Offsets in bytes from the tile's first slot.
    constexpr unsigned SLOTB = YZ_SLOT * sz;
    const unsigned fin0 = (unsigned)lane * 16u;
    const unsigned fout0 = (unsigned)((isy ? nTz : 1) * (TX + 3) - 3) * SLOTB + (unsigned)lane * 16u;
    auto fin_off = [&](int s) {
        const int ir = s - fq;
        return (fin_ok && (unsigned)ir < (unsigned)len) ? fin0 + (unsigned)s * SLOTB : kOOB;
    };
    auto fout_off = [&](int s) {
        const int ir = s - fq - 3;
        return (fout_ok && (unsigned)ir < (unsigned)len) ? fout0 + (unsigned)s * SLOTB : kOOB;
    };
    // this lane's four y- and z-face values in the face area
    lds_t<T>* fa = as_lds(fstg);
    const int ypos = (kd * 4 + kz) * NPK * CH, zpos = (NYP + (kd * 4 + jy) * NPK) * CH;
    // psi pieces: pass it of the wave writes 16-byte piece it * 64 + lane of
    // the 16 pencils' blocks of nvalid * 8 values; its byte offset from the
    // psi resource base at step 0 (32-bit wrap-around arithmetic: at every
    // step where the piece is written the true offset lies in [0, 2^31)),
    // moved by wsb per step; wsk: the pencil's skew (huge: no piece)
    const int wsb = cdir * pstride * 8 * sz;
    int wsk[NIT], woff[NIT];
    unsigned wofs[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int id = it * 64 + lane;
        const int per = nvalid * 8 / CH;
        wsk[it] = 1 << 29;
        woff[it] = 0;
        wofs[it] = 0;
        if (id < 16 * per) {
            const int q = id / per, o = id - q * per;
            const int qy = q & 3, qz = q >> 2;
            const int qjl = J * 4 + qy, qkl = K * 4 + qz;
            if (qjl < ny && qkl < nz) {
                const int qj = ry ? ny - 1 - qjl : qjl;
                const int qk = rz ? nz - 1 - qkl : qkl;
                const long qc0 = ((long)qk * ny + qj) * nx + (rx ? nx - 1 - i0 : i0);
                wsk[it] = qy + qz;
                woff[it] = q * stage_pencil<T>() + o * CH;
                wofs[it] = (unsigned)(((qc0 - cell_base) * pstride * 8 + o * CH) * sz - (long)(qy + qz) * wsb);
            }
        }
    }
    const T ax4 = T(4) * ax, ax2 = T(2) * ax, ay4 = T(4) * ay, ay2 = T(2) * ay, az4 = T(4) * az, az2 = T(2) * az;
    const int nsteps = len + 6;
    lds_t<T>* stw = as_lds(stg) + (lane & 15) * stage_pencil<T>() + (lane >> 4) * 8;
    struct Src {
        Vec8<T> s;
        T sig;
    };
    auto fetch = [&](int ir, Src& v) {
        if constexpr (!staged_tile<T>()) {
            const int irc = min(max(ir, 0), len - 1);
            v.s = load8(src0 + cdir * irc * 8);
            v.sig = sig0[cdir * irc];
        }
    };
    // fin: this step's face inflow piece, loaded two steps earlier; refilled
    // here with the piece of step s + 2
    auto step = [&](int s, piece_t<T>& fin, Src& use, Src& fill) {
        const int ir = s - skew;
        fetch(ir + 1, fill);
        *reinterpret_cast<lds_piece_t<T>*>(fa + lane * CH) = fin;
        fin = buf_load_piece<T>(rf, fin_off(s + 2));
        __builtin_amdgcn_wave_barrier();
        T yi[4], zi[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            // the moves are made by every lane and only then selected (the
            // empty asm keeps the compiler from turning the selects into
            // branches around the moves)
            T ys = row_shr<1>(yo[t]), zs = row_shr<4>(zo[t]);
            asm volatile("" : "+v"(ys), "+v"(zs));
            yi[t] = jy == 0 ? fa[ypos + t] : ys;
            zi[t] = kz == 0 ? fa[zpos + t] : zs;
        }
        const bool active = pen && ir >= 0 && ir < len;
        const int irl = min(max(ir, 0), len - 1);
        T g[8], u[8], sg;
        if constexpr (staged_tile<T>()) {
            const lds_t<T>* sp = tsrc + irl * (16 * src_pencil<T>());
#pragma unroll
            for (int n = 0; n < 8; ++n) g[n] = sp[n ^ M];
            sg = tsig[irl * 16];
        } else {
#pragma unroll
            for (int n = 0; n < 8; ++n) g[n] = use.s.v[n ^ M];
            sg = use.sig;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int nx0 = 2 * t;
            g[nx0] = fma(ax4, xin[t], g[nx0]);
            g[nx0 + 1] = fma(-ax2, xin[t], g[nx0 + 1]);
            const int ny0 = (t & 1) + 4 * (t >> 1);
            g[ny0] = fma(ay4, yi[t], g[ny0]);
            g[ny0 + 2] = fma(-ay2, yi[t], g[ny0 + 2]);
            g[t] = fma(az4, zi[t], g[t]);
            g[t + 4] = fma(-az2, zi[t], g[t + 4]);
        }
        cell_solve3(g, ax, ay, az, sg, u);
        // x inflow: the tile's until the lane's first cell, then each cell's
        // outflow, held after the last cell for the store after the loop
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            xin[t] = active ? u[2 * t + 1] : xin[t];
            yo[t] = u[(t & 1) + 2 + 4 * (t >> 1)];
            zo[t] = u[t + 4];
        }
#pragma unroll
        for (int n = 0; n < 8; ++n) stw[n] = u[n ^ M];
        // the staged psi of the 16 pencils: LDS operations of one wave execute
        // in order, so the reads below see this step's writes
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const bool ok = (unsigned)(s - wsk[it]) < (unsigned)len;
            const piece_t<T> v = *reinterpret_cast<const lds_piece_t<T>*>(as_lds(stg) + woff[it]);
            buf_store_piece<T, kPsiStore>(rpsi, ok ? wofs[it] + (unsigned)(s * wsb) : kOOB, v);
        }
        // face outflow: far-side lanes into the face area (after this step's
        // reads of it), one piece per lane out
        if (jy == 3) {
#pragma unroll
            for (int t = 0; t < 4; ++t) fa[ypos + t] = yo[t];
        }
        if (kz == 3) {
#pragma unroll
            for (int t = 0; t < 4; ++t) fa[zpos + t] = zo[t];
        }
        __builtin_amdgcn_wave_barrier();
        const piece_t<T> fo = *reinterpret_cast<const lds_piece_t<T>*>(fa + lane * CH);
        buf_store_piece<T, kFaceStore>(rf, fout_off(s), fo);
        __builtin_amdgcn_wave_barrier();
    };
    Src s0, s1;
    fetch(-skew, s0);
    // The pieces of steps 0 and 1, each followed by PAD stores with offset
    // kOOB (dropped by the range check).  The wait for a piece inside the
    // loop is set for every way into it, the first turn included, so the
    // pieces loaded here must be followed by at least as many operations as
    // in the loop (a step issues NIT psi stores, one face store and, FP32, its
    // three source loads); otherwise every step would wait for the previous
    // step's stores.  The scheduling barriers keep this order.
    constexpr int PAD = NIT + 4;
    piece_t<T> f0 = buf_load_piece<T>(rf, fin_off(0));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < PAD; ++i) buf_store_piece<T, 0>(rf, kOOB + 16u * i, piece_t<T>{});
    __builtin_amdgcn_sched_barrier(0);
    piece_t<T> f1 = buf_load_piece<T>(rf, fin_off(1));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < PAD; ++i) buf_store_piece<T, 0>(rf, kOOB + 16u * (PAD + i), piece_t<T>{});
    __builtin_amdgcn_sched_barrier(0);
    // an even number of steps, so that the loop has no exit between its two
    // steps (such an exit makes the wait at the top of the loop cover every
    // store again); the extra step, when there is one, has every lane
    // outside its row and stores nothing
    const int nsteps2 = (nsteps + 1) & ~1;
    for (int s = 0; s < nsteps2; s += 2) {
        step(s, f0, s0, s1);
        step(s + 1, f1, s1, s0);
    }
    if (pen && I + 1 < nTx) store4(xd + (((long)(I + 1) * nz + kl) * ny + jl) * 4, xin[0], xin[1], xin[2], xin[3]);
}

// blockIdx.x: tile of the plane; blockIdx.y: reflection class; wave w of the
// block: direction group w of that class (four directions, -1 = unused slot).
// The waves of a block read the same cells' source and sigma_t, which one
// compute unit's L1 then serves to all of them.
// The compiler is told to schedule for three waves per SIMD, so that two
// six-wave workgroups share a CU.  Measured at C5: FP32 11.0 -> 9.4 ms against
// the default schedule for four or more waves; FP64 16.0 -> 15.7 ms against
// two waves per SIMD.
constexpr int PSI3D_WAVES = 3;
template <typename T, bool BUF>
__global__ void __launch_bounds__(384) __attribute__((amdgpu_waves_per_eu(PSI3D_WAVES, PSI3D_WAVES)))
sweep3d_kernel(int nx, int ny, int nz, int ndirs,
                                                      const DirInfo* __restrict__ dirs, int transpose,
                                                      const int* __restrict__ groups, int groups_per_class,
                                                      int cls0, int pstride, int local,
                                                      const T* __restrict__ sigt, const T* __restrict__ src,
                                                      T* __restrict__ xf, long xstride, T* __restrict__ yz, int TX,
                                                      int nTx, int nTy, int nTz, const int* __restrict__ tiles,
                                                      T* __restrict__ psi) {
    __shared__ __align__(16) T stage[6][stage_elems<T>()];
    __shared__ __align__(16) TileIn<T> tin;
    // (wave-uniform for the compiler, so that the group's values below and
    // the buffer resources built from them live in scalar registers)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int tile = tiles[blockIdx.x];
    const int I = tile & 1023, J = (tile >> 10) & 1023, K = (tile >> 20) & 1023;
    // reflection of the class, from its first direction (always valid)
    const int cls = cls0 + (int)blockIdx.y;
    const int mc = groups[6 * cls * groups_per_class];
    const DirInfo dm = dirs[mc];
    const int m = (dm.rx ^ transpose) | ((dm.ry ^ transpose) << 1) | ((dm.rz ^ transpose) << 2);
    if constexpr (staged_tile<T>()) {
        stage_tile<T>(nx, ny, nz, m, I, J, K, TX, sigt, src, &tin);
        __syncthreads();
    }
    const int grp = cls * groups_per_class + wave;
    const int* gi = groups + 6 * grp;
    const int d = gi[lane >> 4];
    const int m0 = __builtin_amdgcn_readfirstlane(gi[0]);  // first direction of the group (-1: empty slot)
    if (m0 < 0) return;              // empty group slot: the whole wave leaves
    // consecutive directions d0 .. d0 + nvalid - 1 of psi: psi goes out
    // through the LDS stage; otherwise (nvalid = 0) every lane stores its own
    // values.  With local, psi holds only this class's directions, in group
    // order (group w, slot k -> 4 w + k), which are always consecutive.
    const int d0 = __builtin_amdgcn_readfirstlane(local ? 4 * wave : gi[4]);
    const int nvalid = __builtin_amdgcn_readfirstlane(local ? gi[5] : (gi[4] >= 0 ? gi[5] : 0));
    const bool dok = d >= 0;
    const int dd = dok ? d : m0;
    const int dpsi = local ? 4 * wave + (lane >> 4) : dd;
    const DirInfo di = dirs[dd];
    const T ax = T(di.ax), ay = T(di.ay), az = T(di.az);
    T* xd = xf + dd * xstride;
    // this group's face slots of this tile
    T* yzt = yz + ((long)grp * nTx * nTy * nTz + ((long)I * nTy + J) * nTz + K) * (TX + 3) * YZ_SLOT;
    if constexpr (BUF) {
        // wave-uniform resources: the group's face slots of the tile, psi
        // from the tile's lowest cell in memory and the wave's first psi
        // direction
        __shared__ __align__(16) T fstage[6][face_stage_elems<T>()];
        const int i0 = I * TX, len = min(TX, nx - i0);
        const int rxm = m & 1, rym = (m >> 1) & 1, rzm = (m >> 2) & 1;
        const int jn = min(J * 4 + 4, ny) - J * 4, kn = min(K * 4 + 4, nz) - K * 4;
        const long imin = rxm ? nx - i0 - len : i0;
        const long jmin = rym ? ny - J * 4 - jn : J * 4;
        const long kmin = rzm ? nz - K * 4 - kn : K * 4;
        const long cell_base = (kmin * ny + jmin) * nx + imin;
        const __amdgpu_buffer_rsrc_t rf = buf_rsrc(yzt);
        const __amdgpu_buffer_rsrc_t rpsi = buf_rsrc(psi + (cell_base * pstride + d0) * 8);
        const unsigned slots = (unsigned)__builtin_amdgcn_readfirstlane(
            (gi[0] >= 0 ? 1 : 0) | (gi[1] >= 0 ? 2 : 0) | (gi[2] >= 0 ? 4 : 0) | (gi[3] >= 0 ? 8 : 0));
#define SN_CASEB(MM)                                                                                               \
    case MM:                                                                                                       \
        sweep3d_body_buf<T, MM>(nx, ny, nz, pstride, slots, dok, ax, ay, az, I, J, K, TX, nTx, nTy, nTz, &tin, sigt, \
                                src, xd, rf, rpsi, cell_base, nvalid, stage[wave],                                 \
                                fstage[wave]);                                                                     \
        break;
        switch (m) {
            SN_CASEB(0)
            SN_CASEB(1)
            SN_CASEB(2)
            SN_CASEB(3)
            SN_CASEB(4)
            SN_CASEB(5)
            SN_CASEB(6)
            SN_CASEB(7)
        }
#undef SN_CASEB
        return;
    }
#define SN_CASE(MM)                                                                                               \
    case MM:                                                                                                      \
        sweep3d_body<T, MM>(nx, ny, nz, pstride, dpsi, dok, ax, ay, az, I, J, K, TX, nTx, nTy, nTz, &tin, sigt,   \
                            src, xd, yzt, psi, d0, nvalid, stage[wave]);                                          \
        break;
    switch (m) {
        SN_CASE(0)
        SN_CASE(1)
        SN_CASE(2)
        SN_CASE(3)
        SN_CASE(4)
        SN_CASE(5)
        SN_CASE(6)
        SN_CASE(7)
    }
#undef SN_CASE
}

// Fused sweep + moment (source iteration): as sweep3d_kernel, but psi is not
// stored; phio receives, per reflection class (octant) blockIdx.y, that
// octant's share sum_d w_d psi_d of phi ([class][cell][8], FP64).  Every wave
// of the block takes part in the block-wide reductions, including waves of
// empty direction groups (their lanes contribute zero).
template <typename T>
__global__ void __launch_bounds__(384) sweep3d_flux_kernel(int nx, int ny, int nz, int ndirs,
                                                           const DirInfo* __restrict__ dirs, const double* __restrict__ w,
                                                           int transpose, const int* __restrict__ groups,
                                                           int groups_per_class, int cls0,
                                                           const T* __restrict__ sigt,
                                                           const T* __restrict__ src, T* __restrict__ xf, long xstride,
                                                           T* __restrict__ yz, int TX, int nTx, int nTy, int nTz,
                                                           const int* __restrict__ tiles, double* __restrict__ phioct) {
    __shared__ __align__(16) double red[2 * RF * 6 * 128];
    __shared__ __align__(16) TileIn<T> tin;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int cls = cls0 + (int)blockIdx.y;
    const int grp = cls * groups_per_class + wave;
    const int* gi = groups + 6 * grp;
    const int d = gi[lane >> 4];
    const int mc = groups[6 * cls * groups_per_class];  // first direction of the class (valid)
    const bool dok = d >= 0;
    const int dd = dok ? d : mc;
    const int tile = tiles[blockIdx.x];
    const int I = tile & 1023, J = (tile >> 10) & 1023, K = (tile >> 20) & 1023;
    const DirInfo dm = dirs[mc];
    const int m = (dm.rx ^ transpose) | ((dm.ry ^ transpose) << 1) | ((dm.rz ^ transpose) << 2);
    if constexpr (staged_tile<T>()) {
        stage_tile<T>(nx, ny, nz, m, I, J, K, TX, sigt, src, &tin);
        __syncthreads();
    }
    const DirInfo di = dirs[dd];
    const T ax = T(di.ax), ay = T(di.ay), az = T(di.az);
    const double wgt = dok ? w[dd] : 0.0;
    T* xd = xf + dd * xstride;
    T* yzt = yz + ((long)grp * nTx * nTy * nTz + ((long)I * nTy + J) * nTz + K) * (TX + 3) * YZ_SLOT;
    double* po = phioct + (long)cls * nx * ny * nz * 8;
#define SN_CASEF(MM)                                                                                             \
    case MM:                                                                                                     \
        sweep3d_body<T, MM, true>(nx, ny, nz, ndirs, dd, dok, ax, ay, az, I, J, K, TX, nTx, nTy, nTz, &tin, sigt, \
                                  src, xd, yzt, nullptr, -1, 0, nullptr, wgt, red, po, groups_per_class);         \
        break;
    switch (m) {
        SN_CASEF(0)
        SN_CASEF(1)
        SN_CASEF(2)
        SN_CASEF(3)
        SN_CASEF(4)
        SN_CASEF(5)
        SN_CASEF(6)
        SN_CASEF(7)
    }
#undef SN_CASEF
}

// phi = sum over the classes of phioct (fixed order), or phi += that sum
// RES: also the residual partial sums (phi - ref)^2, phi^2, ref^2 per block
template <bool RES>
__global__ void __launch_bounds__(256) octant_sum_kernel(long n, int ncls, const double* __restrict__ phioct,
                                                         double* __restrict__ phi, int accumulate,
                                                         const double* __restrict__ ref,
                                                         double* __restrict__ part) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < ncls; ++c) s += phioct[c * n + i];
        const double v = accumulate ? phi[i] + s : s;
        phi[i] = v;
        if constexpr (RES) {
            const double y = ref[i], e = v - y;
            s0 = fma(e, e, s0);
            s1 = fma(v, v, s1);
            s2 = fma(y, y, s2);
        }
    }
    if constexpr (RES) {
        __shared__ double sh[768];
        block_sum3(s0, s1, s2, sh);
        if (threadIdx.x == 0) {
            part[blockIdx.x] = s0;
            part[gridDim.x + blockIdx.x] = s1;
            part[2 * gridDim.x + blockIdx.x] = s2;
        }
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// the streams st[1..ns) of a split start after the work queued so far on st[0]
static hipError_t split_fork(const StreamSplit& sp, int ns) {
    hipError_t e = hipEventRecord(sp.fork, sp.st[0]);
    for (int k = 1; k < ns && e == hipSuccess; ++k) e = hipStreamWaitEvent(sp.st[k], sp.fork, 0);
    return e;
}
// st[0] continues after the work queued on st[1..ns)
static hipError_t split_join(const StreamSplit& sp, int ns) {
    hipError_t e = hipSuccess;
    for (int k = 1; k < ns && e == hipSuccess; ++k) {
        e = hipEventRecord(sp.join[k], sp.st[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(sp.st[0], sp.join[k], 0);
    }
    return e;
}

template <typename T>
hipError_t launch_init_faces(const SweepGeom& g, const DirInfo* dirs, int transpose, const double* inflow,
                             T* xf, T* yf, T* zf, hipStream_t st) {
    long per = (long)g.ny * g.nz + (g.dim == 3 ? 0 : (long)g.nx * g.nz);
    long total = per * g.ndirs;
    int blocks = (int)std::min<long>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(init_faces_kernel<T>, dim3(blocks), dim3(256), 0, st, g.dim, g.nx, g.ny, g.nz, g.ndirs, dirs,
                       transpose, inflow, g.nbf, xf, g.xstride, yf, g.ystride, zf, g.zstride);
    if (g.dim == 3) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int ngroups = g.nclasses * g.groups_per_class;
        const long ny_t = (long)ngroups * ((long)g.nTx * g.nTz + (long)g.nTx * g.nTy) * (g.TX + 3) * 64;
        const int yb = (int)std::min<long>((ny_t + 255) / 256, 65536);
        // yf: the y/z face slots
        hipLaunchKernelGGL(init_yz_faces_kernel<T>, dim3(yb), dim3(256), 0, st, g.nx, g.ny, g.nz, g.TX, g.nTx, g.nTy,
                           g.nTz, ngroups, g.groups, dirs, transpose, inflow, g.nbf, yf);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep(const SweepGeom& g, const DirInfo* dirs, int transpose, const T* sigt, const T* src, T* xf,
                        T* yf, T* zf, const int* tiles, const int* plane_off, T* psi, T* sink, hipStream_t st,
                        const SweepPart* part, const StreamSplit* split) {
    const SweepPart all{0, g.dim == 2 ? g.ndirs : g.nclasses, g.ndirs, 0, g.groups};
    const SweepPart& pp = part ? *part : all;
    if (g.dim == 2) {
        for (int ch = 0; ch < g.nchunk; ++ch) {
            int row0 = ch * ROWS2D;
            int nrows = std::min(ROWS2D, g.ny - row0);
            int nw = (nrows + 63) / 64;
            hipLaunchKernelGGL(sweep2d_kernel<T>, dim3(pp.count), dim3(64 * nw), 0, st, g.nx, g.ny, g.ndirs, dirs,
                               pp.order2d, transpose, sigt, src, xf, g.xstride, yf, g.ystride, ch, g.nchunk, row0,
                               nrows, psi, pp.pstride, pp.local);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    // a class split over several streams only for full sweeps
    const int ns = (!part && split) ? std::min(split->n, pp.count) : 1;
    hipError_t e;
    if (ns > 1 && (e = split_fork(*split, ns)) != hipSuccess) return e;
    for (int p = 0; p < g.nplanes; ++p) {
        int nt = plane_off[p + 1] - plane_off[p];
        for (int k = 0; k < ns; ++k) {
            const int c0 = pp.first + k * pp.count / ns, c1 = pp.first + (k + 1) * pp.count / ns;
            hipStream_t sk = ns > 1 ? split->st[k] : st;
            if (g.buf)
                hipLaunchKernelGGL((sweep3d_kernel<T, true>), dim3(nt, c1 - c0), dim3(64 * g.groups_per_class), 0,
                                   sk, g.nx, g.ny, g.nz, g.ndirs, dirs, transpose, g.groups, g.groups_per_class, c0,
                                   pp.pstride, pp.local, sigt, src, xf, g.xstride, yf, g.TX,
                                   g.nTx, g.nTy, g.nTz, tiles + plane_off[p], psi);
            else
                hipLaunchKernelGGL((sweep3d_kernel<T, false>), dim3(nt, c1 - c0), dim3(64 * g.groups_per_class), 0,
                                   sk, g.nx, g.ny, g.nz, g.ndirs, dirs, transpose, g.groups, g.groups_per_class, c0,
                                   pp.pstride, pp.local, sigt, src, xf, g.xstride, yf, g.TX,
                                   g.nTx, g.nTy, g.nTz, tiles + plane_off[p], psi);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    if (ns > 1) return split_join(*split, ns);
    return hipSuccess;
}

template <typename T>
hipError_t launch_skew2d(int nx, int ny, int nn, const T* in, T* out, hipStream_t st) {
    const long total = 4L * ((ny + 63) / 64) * (nx + 63) * 64;
    const int blocks = (int)std::min<long>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(skew2d_kernel<T>, dim3(blocks), dim3(256), 0, st, nx, ny, nn, in, out);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_source_skew2d(int nx, int ny, const double* sigma_s, const double* phi, const double* phi_prev,
                                const double* q, T* out, hipStream_t st) {
    const long nc = (long)nx * ny;
    const int blocks = (int)std::min<long>((nc + 255) / 256, 65536);
    hipLaunchKernelGGL(source_skew2d_kernel<T>, dim3(blocks), dim3(256), 0, st, nx, ny, sigma_s, phi, phi_prev, q,
                       out);
    return hipGetLastError();
}
hipError_t launch_scatter_source_skew2d(int nx, int ny, const int* slot_of_cell, const double* phi_si,
                                       const double* x, const double* sigma_s, const double* q, double* phi_out,
                                       double* out, hipStream_t st) {
    const long nc = (long)nx * ny;
    const int blocks = (int)std::min<long>((nc + 255) / 256, 65536);
    hipLaunchKernelGGL(scatter_source_skew2d_kernel, dim3(blocks), dim3(256), 0, st, nx, ny, slot_of_cell, phi_si,
                       x, sigma_s, q, phi_out, out);
    return hipGetLastError();
}
template hipError_t launch_source_skew2d<double>(int, int, const double*, const double*, const double*,
                                                 const double*, double*, hipStream_t);
template hipError_t launch_source_skew2d<float>(int, int, const double*, const double*, const double*, const double*,
                                                float*, hipStream_t);
template hipError_t launch_skew2d<double>(int, int, int, const double*, double*, hipStream_t);
template hipError_t launch_skew2d<float>(int, int, int, const float*, float*, hipStream_t);

template <typename T>
hipError_t launch_sweep_flux3d(const SweepGeom& g, const DirInfo* dirs, const double* w, int transpose,
                               const T* sigt, const T* src, T* xf, T* yf, T* zf, const int* tiles,
                               const int* plane_off, double* phioct, double* phi, int accumulate,
                               const double* ref, double* part, hipStream_t st, const StreamSplit* split) {
    const int ns = split ? std::min(split->n, g.nclasses) : 1;
    hipError_t e;
    if (ns > 1 && (e = split_fork(*split, ns)) != hipSuccess) return e;
    for (int p = 0; p < g.nplanes; ++p) {
        int nt = plane_off[p + 1] - plane_off[p];
        for (int k = 0; k < ns; ++k) {
            const int c0 = k * g.nclasses / ns, c1 = (k + 1) * g.nclasses / ns;
            hipLaunchKernelGGL((sweep3d_flux_kernel<T>), dim3(nt, c1 - c0), dim3(64 * g.groups_per_class), 0,
                               ns > 1 ? split->st[k] : st, g.nx, g.ny, g.nz, g.ndirs, dirs, w, transpose, g.groups,
                               g.groups_per_class, c0, sigt, src, xf, g.xstride, yf, g.TX,
                               g.nTx, g.nTy, g.nTz, tiles + plane_off[p], phioct);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    if (ns > 1 && (e = split_join(*split, ns)) != hipSuccess) return e;
    const long nc = (long)g.nx * g.ny * g.nz, n = nc * 8;
    const int blocks = octant_sum_blocks(nc);
    if (ref)
        hipLaunchKernelGGL(octant_sum_kernel<true>, dim3(blocks), dim3(256), 0, st, n, g.nclasses, phioct, phi,
                           accumulate, ref, part);
    else
        hipLaunchKernelGGL(octant_sum_kernel<false>, dim3(blocks), dim3(256), 0, st, n, g.nclasses, phioct, phi,
                           accumulate, ref, part);
    return hipGetLastError();
}
template hipError_t launch_sweep_flux3d<double>(const SweepGeom&, const DirInfo*, const double*, int, const double*,
                                                const double*, double*, double*, double*, const int*, const int*,
                                                double*, double*, int, const double*, double*, hipStream_t,
                                                const StreamSplit*);
template hipError_t launch_sweep_flux3d<float>(const SweepGeom&, const DirInfo*, const double*, int, const float*,
                                               const float*, float*, float*, float*, const int*, const int*,
                                               double*, double*, int, const double*, double*, hipStream_t,
                                               const StreamSplit*);

template hipError_t launch_init_faces<double>(const SweepGeom&, const DirInfo*, int, const double*, double*, double*,
                                              double*, hipStream_t);
template hipError_t launch_init_faces<float>(const SweepGeom&, const DirInfo*, int, const double*, float*, float*,
                                             float*, hipStream_t);
template hipError_t launch_sweep<double>(const SweepGeom&, const DirInfo*, int, const double*, const double*,
                                         double*, double*, double*, const int*, const int*, double*, double*,
                                         hipStream_t, const SweepPart*, const StreamSplit*);
template hipError_t launch_sweep<float>(const SweepGeom&, const DirInfo*, int, const float*, const float*, float*,
                                        float*, float*, const int*, const int*, float*, float*, hipStream_t,
                                        const SweepPart*, const StreamSplit*);

}  // namespace sn
