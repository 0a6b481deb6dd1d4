// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "sn_device.hpp"

namespace sn {

// Geometry of one sweep: mesh, direction count and the tiling / chunking the
// sweep kernels use (see sweep.hip).
// rows per 2D sweep workgroup (one lane per row, 8 waves)
constexpr int ROWS2D = 512;

struct SweepGeom {
    int dim, nx, ny, nz, ndirs;
    long nbf;          // boundary-face nodes per direction in the inflow layout
    int TX;            // 3D tile length along x
    int nTx, nTy, nTz; // 3D tile counts (tiles are TX x 4 x 4 cells)
    int nclasses;      // 3D: reflection classes with at least one direction
    int groups_per_class;  // 3D: direction groups of four per class (max over classes)
    const int* groups; // 3D: device [nclasses * groups_per_class][6]: four direction ids (-1 = empty),
                       //     the first id if the valid ids are consecutive (else -1), the valid count;
                       // 2D: device [ndirs] direction of each workgroup (XCD-aware order)
    int nplanes;       // 3D tile-diagonal planes
    int buf;           // 3D psi sweep: the variant without branches around memory operations (buffer loads
                       //     and stores with range-checked offsets); needs every direction group consecutive
                       //     and the byte offsets of one tile's psi below 2^31
    int nchunk;        // 2D row chunks of at most ROWS2D rows
    long xstride, ystride, zstride;  // per-direction face-buffer sizes (elements); 3D: x only (y and z faces
                                     // are kept in tile slots, yz_face_elems)
};

template <typename T>
hipError_t launch_init_faces(const SweepGeom& g, const DirInfo* dirs, int transpose, const double* inflow, T* xf,
                             T* yf, T* zf, hipStream_t st);
// 2D: sigt and src are the diagonal-major arrays of launch_skew2d; 3D: per cell.
// sink: scratch of sink_elems(g) elements (unused)
// A part of the directions to sweep (nullptr: all of them, psi [cell][ndirs][nn]).
// 3D: the reflection classes first .. first + count - 1; 2D: the count
// directions order2d[0 .. count - 1].  psi: [cell][pstride][nn]; local = 0:
// a direction's global index, local = 1: its position in the part (3D:
// 4 * group + slot within its class).
// 3D y and z face data, in tile slots: for direction group g (class * groups
// per class + wave) and tile t = (I nTy + J) nTz + K, TX + 3 slots of
// YZ_SLOT values.  Slot q holds, for the group's four direction slots kd and
// the four positions kq across the face, the four y-face values (first half,
// [kd][kq][4]) and z-face values (second half) entering the cell at position
// q - kq of the tile along x (kq: the kz of a y face, the jy of a z face).
// The upstream tile writes slot q of its downstream neighbour at step q + 3
// of its sweep and the tile reads it at step q, so a wave's face data of one
// step is contiguous.  Faces on the domain boundary (J = 0 for y, K = 0 for z)
// hold the inflow.  x faces: per direction, [I][kl][jl][4] in the reflected
// frame.
constexpr int YZ_SLOT = 128;
inline long yz_face_elems(int ngroups, int nTx, int nTy, int nTz, int TX) {
    return (long)ngroups * nTx * nTy * nTz * (TX + 3) * YZ_SLOT;
}

// Streams over which the reflection classes of a full 3D sweep are split: the
// classes [k ncls / n, (k + 1) ncls / n) go to st[k], and the plane launches
// are issued plane by plane across the streams, so that a class group starts
// its next plane as soon as its own launch is done instead of waiting for the
// slowest tile of every class.  st[0] is the caller's stream; the others wait
// for an event recorded on it before the sweep, and it waits for theirs after
// (classes touch disjoint psi and face data).  n = 1: st[0] only.
constexpr int MAX_SPLIT = 4;
constexpr int SPLIT_DEFAULT = 2;
struct StreamSplit {
    int n;
    hipStream_t st[MAX_SPLIT];
    hipEvent_t fork, join[MAX_SPLIT];
};
struct SweepPart {
    int first, count, pstride, local;
    const int* order2d;
};
template <typename T>
hipError_t launch_sweep(const SweepGeom& g, const DirInfo* dirs, int transpose, const T* sigt, const T* src, T* xf,
                        T* yf, T* zf, const int* tiles, const int* plane_off, T* psi, T* sink, hipStream_t st,
                        const SweepPart* part = nullptr, const StreamSplit* split = nullptr);
inline long sink_elems(const SweepGeom&) { return 1; }
// 3D fused sweep + moment (source iteration): psi is not stored; phioct
// (workspace [nclasses][ncells][8]) receives each octant's share of phi, then
// phi = (accumulate ? phi : 0) + sum over the octants in a fixed order.
// ref != nullptr: residual partial sums as in launch_moment, part[3][octant_sum_blocks(ncells)]
// (at most 4096 blocks: the residual's partial sums are reduced afterwards by
// one workgroup, and 3 x 65536 of them made that reduction the tail of the
// DSA's first kernel at 128^3)
inline int octant_sum_blocks(long nc) { return (int)std::min<long>((nc * 8 + 255) / 256, 4096); }
template <typename T>
hipError_t launch_sweep_flux3d(const SweepGeom& g, const DirInfo* dirs, const double* w, int transpose,
                               const T* sigt, const T* src, T* xf, T* yf, T* zf, const int* tiles,
                               const int* plane_off, double* phioct, double* phi, int accumulate,
                               const double* ref, double* part, hipStream_t st,
                               const StreamSplit* split = nullptr);
// per-cell array [ncells][nn] -> four quadrant diagonal-major arrays
// [4][ceil(ny / 64)][nx + 63][64][nn] (2D sweep input layout)
template <typename T>
hipError_t launch_skew2d(int nx, int ny, int nn, const T* in, T* out, hipStream_t st);
// the 2D sweep source (sigma_s (phi - phi_prev) + q) / 4pi written straight
// into the diagonal-major layout (only on-mesh entries; padding stays zero)
template <typename T>
hipError_t launch_source_skew2d(int nx, int ny, const double* sigma_s, const double* phi, const double* phi_prev,
                                const double* q, T* out, hipStream_t st);
// phi_out = phi_si + P x (x: thick-slot values, slot_of_cell -1 for others)
// and the FP64 diagonal-major sweep source of phi_out (2D, four quadrants)
hipError_t launch_scatter_source_skew2d(int nx, int ny, const int* slot_of_cell, const double* phi_si,
                                       const double* x, const double* sigma_s, const double* q, double* phi_out,
                                       double* out, hipStream_t st);
// (plus SKEW2D_TAIL zero diagonals after the last block: the sweep's
// prefetch runs up to that far past a block's last diagonal)
constexpr int SKEW2D_TAIL = 16;
inline long skew2d_elems(int nx, int ny, int nn) {
    return (4L * ((ny + 63) / 64) * (nx + 63) + SKEW2D_TAIL) * 64 * nn;
}

// scalar-flux kernels (flux.hip)
template <typename T>
hipError_t launch_source(long nc, int nn, const double* sigma_s, const double* phi, const double* phi_prev,
                         const double* q, T* src, hipStream_t st);
// ref != nullptr: also the residual partial sums of (phi - ref)^2, phi^2,
// ref^2 over the written phi, part[3][moment_blocks(nc)]
inline int moment_blocks(long nc) { return (int)std::min<long>((4 * nc + 255) / 256, 1 << 16); }
template <typename T>
hipError_t launch_moment(long nc, int nn, int ndirs, const double* w, const T* psi, double* phi, int accumulate,
                         const double* ref, double* part, hipStream_t st);
// partial sums of (a-b)^2, a^2, b^2 over n doubles; out[3] on device
hipError_t launch_residual(long n, const double* a, const double* b, double* partials, int nparts, double* out,
                           hipStream_t st);
// the final reduction of nparts such partial sums into out[3] (device) and,
// if out_host != nullptr, into pinned host memory
hipError_t launch_residual_final(int nparts, const double* partials, double* out, double* out_host,
                                 hipStream_t st);
// gradient contraction over the ndirs directions of psi / psi_adj
// ([cell][ndirs][nn], weights w, zero weight = unused slot); accumulate:
// g_t += ...; g_s is written when not NULL
template <typename T>
hipError_t launch_gradient(long nc, int nn, int ndirs, const double* w, const double* h, const double* sigma_t,
                           const double* sigma_s, const T* psi, const T* psi_adj, const double* phi,
                           const double* chi, double* g_t, double* g_s, hipStream_t st, int accumulate = 0);
// Alg. 1: bar = a - b (b may be NULL) on thick cells, 0 elsewhere; phi += z on thin cells
hipError_t launch_thick_diff(long nc, int nn, const int* slot_of_cell, const double* a, const double* b, double* bar,
                             hipStream_t st);
hipError_t launch_thin_add(long nc, int nn, const int* slot_of_cell, const double* z, double* phi, hipStream_t st);
// adjoint sources: y = a x; face data [ndirs][nbf] = 1 on [f0, f1) for directions with out[d] != 0
hipError_t launch_scale(long n, double a, const double* x, double* y, hipStream_t st);
hipError_t launch_face_data(int ndirs, long nbf, long f0, long f1, const int* out, double* data, hipStream_t st);
// Krylov vector operations: out[i] = V_i . w (i < k, V: k vectors of n, part:
// k * krylov_blocks(n) scratch, out_host: pinned copy or NULL);
// w += sign * sum_i h[i] V_i; y = a x + b y
int krylov_blocks(long n);
hipError_t launch_multi_dot(long n, int k, const double* V, const double* w, double* part, double* out,
                            double* out_host, hipStream_t st);
hipError_t launch_multi_axpy(long n, int k, const double* V, const double* h, double sign, double* w,
                             hipStream_t st);
hipError_t launch_axpby(long n, double a, const double* x, double b, double* y, hipStream_t st);

// out[0] = sum_c r_c int_c phi; out[1] = outflow partial current through `face`
// (wn[d] = w_d Omega_d.n for outgoing directions, else 0); part: 3*nparts scratch
template <typename T>
hipError_t launch_response(long nc, int nn, int nx, int ny, int nz, const double* h, const double* r,
                           const double* phi, int face, int ndirs, const double* wn, const T* psi, double* part,
                           int nparts, double* out, hipStream_t st);

// fixed device scratch of the entry points that allocate nothing (noalloc.hip):
// NOALLOC_SCRATCH_DOUBLES doubles per device, shared by every call on that
// device; noalloc_scratch returns its device address on the current device
constexpr long NOALLOC_SCRATCH_DOUBLES = 16384;
hipError_t noalloc_scratch(double** out);

// heterogeneous DSA (dsa.hip)
struct DsaGeom {
    int dim, nx, ny, nz, nn;
    double h[3];
    double kappa0[3];  // (1/8pi) sum_d w_d |Omega_d,axis|
    int nthick;
};

hipError_t launch_thick_flags(long nc, const double* sigma_s, double eta, int* flags, int* block_sums, int nblk,
                              hipStream_t st);
hipError_t launch_thick_scan(int nblk, int* block_sums, int* total, hipStream_t st);
hipError_t launch_thick_scatter(long nc, const int* flags, const int* block_sums, int* slot_of_cell,
                                int* thick_cell, hipStream_t st);
// words per thick cell of the stored block-Jacobi inverse (upper triangle)
template <int NN>
constexpr int bj_entries() {
    return NN * (NN + 1) / 2;
}
inline int bj_entries_of(int nn) {
    return nn * (nn + 1) / 2;
}
hipError_t launch_block_jacobi(const DsaGeom& g, const int* thick_cell, const int* slot_of_cell,
                               const double* sigma_t, const double* sigma_s, double* binv, hipStream_t st);
// nonsymmetric diffusion forms (op = 1 NIP, 2 mNIP): full inverse of the
// diagonal blocks (nn * nn words per thick cell, element-major; *bad set for
// a singular block or, with mNIP, sigma_t <= 0 at a thick cell or its
// neighbour), w = D B^{-1} v or w = b - D B^{-1} v (binv = nullptr: B = I),
// x = B^{-1} u, and the
// thick right-hand side b = coef M (phi_si - phi_old)
hipError_t launch_block_inverse_full(const DsaGeom& g, int op, const int* thick_cell, const int* nbr,
                                     const double* sigma_t, const double* sigma_s, double* binv, int* bad,
                                     hipStream_t st);
hipError_t launch_nip_apply(const DsaGeom& g, int op, const int* thick_cell, const int* nbr, const double* sigma_t,
                            const double* sigma_s, const double* binv, const double* v, const double* b, double* w,
                            hipStream_t st);
hipError_t launch_full_block_apply(const DsaGeom& g, const double* binv, const double* u, double* x, hipStream_t st);
// Exact thick solve by band LU (any form): half width in cells into *w
// (atomic max, zero it first), band assembly (lu zeroed first, row i at
// lu[i ldb + j - i + kl]), factorisation and solve by one workgroup each.
// The solve needs n <= 8192 (the vector in LDS) and kl + ku <= 1023 (one
// row of a column per thread).
constexpr long kBandSolveMaxN = 8192;
constexpr int kBandMaxWidth = 1023;
hipError_t launch_band_width(const DsaGeom& g, const int* nbr, int* w, hipStream_t st);
hipError_t launch_band_assemble(const DsaGeom& g, int op, const int* thick_cell, const int* nbr,
                                const double* sigma_t, const double* sigma_s, int kl, int ldb, double* lu,
                                hipStream_t st);
hipError_t launch_band_factor(long n, int kl, int ku, int ldb, double* lu, int* piv, int* bad, hipStream_t st);
hipError_t launch_band_solve(long n, int kl, int ku, int ldb, const double* lu, const int* piv, const double* b,
                             double* x, hipStream_t st);
hipError_t launch_dsa_rhs_vec(const DsaGeom& g, const int* thick_cell, const double* sigma_t, const double* sigma_s,
                              int mass_kind, const double* phi_old, const double* phi_si, double* b, hipStream_t st);

struct CgScalars {
    double rz[2];   // r.z of the current iterate, slot = iteration parity
    double bb, rr;  // ||b||^2 and the latest ||r||^2
    int done, iters, breakdown, pad;
};

// warm start of the CG from its previous solution xp: w = D xp and the
// partials of xp.b, xp.w (part: 2 * nparts)
hipError_t launch_dsa_warm(const DsaGeom& g, const int* thick_cell, const int* nbr, const double* sigma_t,
                           const double* sigma_s, int mass_kind, const double* phi_old, const double* phi_si,
                           const double* xp, double* w, double* part, int nparts, hipStream_t st);
// right-hand side and CG start (x = 0, or x = alpha x with the warm-start
// partials wpart and w = D x); partials r.z, r.r, b.b in part (3 * nparts);
// also resets s and, given res_part, reduces res_nparts source-iteration
// residual partials into res_out (device) and res_host (pinned host memory)
hipError_t launch_dsa_rhs(const DsaGeom& g, const int* thick_cell, const double* sigma_t, const double* sigma_s,
                          int mass_kind, const double* phi_old, const double* phi_si, const double* binv,
                          double* x, double* r, double* z, double* p, double* part, int nparts, int bj,
                          CgScalars* s, const double* res_part, int res_nparts, double* res_out, double* res_host,
                          const double* w, const double* wpart, hipStream_t st);
hipError_t launch_neighbour_table(const DsaGeom& g, const int* thick_cell, const int* slot_of_cell, int* nbr,
                                  hipStream_t st);
// CG iteration `it` in two kernels.  apply: the stop test (at it = maxit
// only the test), then p = z + beta p_old and q = D p; update (it < maxit):
// x, r and, with bj = 1, z = B^{-1} r (bj = 0: the caller computes z and the
// r.z partials, multigrid V-cycle, after the update).  p0/p1 alternate by
// parity.  When the solve stops or breaks down, block 0 also writes the
// stop fields into s_host (pinned host memory, may be nullptr).
hipError_t launch_cg_apply(const DsaGeom& g, const int* thick_cell, const int* nbr, const double* sigma_t,
                           const double* sigma_s, const double* z, double* p0, double* p1, double* q,
                           double* part_a, double* part_b, int nparts, CgScalars* s, CgScalars* s_host, double rtol,
                           int maxit, int it, hipStream_t st);
hipError_t launch_cg_update(const DsaGeom& g, const double* binv, double* x, double* r, double* z, double* p0,
                            double* p1, const double* q, double* part_a, double* part_b, int nparts, CgScalars* s,
                            CgScalars* s_host, int it, int bj, hipStream_t st);
// the stop test of iteration it (>= 1) on the ||r||^2 partials of part_b
// (from the update of iteration it - 1), made ahead of the multigrid V-cycle
hipError_t launch_cg_test(const double* part_b, int nparts, CgScalars* s, CgScalars* s_host, double rtol,
                          int maxit, int it, hipStream_t st);

hipError_t launch_dsa_scatter(long nc, int nn, const int* slot_of_cell, const double* phi_si, const double* x,
                              double* phi_out, hipStream_t st);
hipError_t launch_sip_apply(const DsaGeom& g, const int* thick_cell, const int* slot_of_cell,
                            const double* sigma_t, const double* sigma_s, const double* u, double* y,
                            hipStream_t st);

// geometric multigrid hierarchy on the device: level 0 is the DG system;
// vertex levels 1 .. L hold one value per active vertex (level 1 = the
// vertices of the thick cells in increasing vertex order) with a 3^dim-point
// stencil (offset index o = sum_d (o_d + 1) 3^d); the per-unknown tables of a level
// are stored offset-major ([o][unknown], [q][unknown]) so that consecutive
// lanes read consecutive words
constexpr int MG_MAXL = 20;
struct MgDev {
    int L, dim, ns;        // coarsest level, dimension, stencil size 3^dim
    int n[MG_MAXL];        // unknowns of each level
    long vo[MG_MAXL];      // offset of level l in the per-unknown arrays (b, x, y, r)
    long so[MG_MAXL];      // offset of level l in coef, nbr, chl (ns per unknown)
    long po[MG_MAXL];      // offset of level l in par, pw (2^dim per unknown; levels < L)
    const double* coef;    // stencil coefficients [ns][unknown]
    const int* nbr;        // stencil neighbours [ns][unknown] or -1
    const int* chl;        // level l >= 2: fine unknowns at 2C + o of level l - 1, [ns][unknown] or -1
    const int* par;        // coarse parents (level l + 1) of each unknown [2^dim][unknown] or -1
    const double* pw;      // interpolation weights of the parents
    const int* vnodes;     // level 1: DG indices (slot * nn + node) at each vertex [2^dim][n1] or -1
    const int* nodev;      // level-1 vertex of each DG node [nthick * nn]
    double* b;
    double* x;
    double* y;
    double* r;
    const double* ainv;    // dense inverse of the level-L operator [n_L][n_L]
    double omega;          // Jacobi damping on the vertex levels
};
// level-1 stencil by probing: coef[w][o] of P^T D_ff P (x0, y0: DG scratch)
hipError_t launch_vmg_probe(const DsaGeom& g, const int* thick_cell, const int* slot_of_cell,
                            const double* sigma_t, const double* sigma_s, const MgDev& m, int nvx, int nvy,
                            const long* vpos, double* x0, double* y0, double* coef, hipStream_t st);
hipError_t launch_mg_vcycle(const DsaGeom& g, const int* thick_cell, const int* nbr, const double* sigma_t,
                            const double* sigma_s, const double* binv, const double* r, double* z0, double* res0,
                            double* z, const MgDev& m, int lc, double omega0, double* part, int nparts,
                            const CgScalars* s, hipStream_t st);

}  // namespace sn
