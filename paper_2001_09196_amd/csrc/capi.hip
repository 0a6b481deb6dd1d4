// C ABI (include/sn.h): context management, argument validation and the
// host-side control of source iteration.  Every arithmetic step of the path
// runs in the kernels of sweep.hip, flux.hip and dsa.hip; the host only
// launches them, reads the residual scalars once per iteration and the CG
// status once per batch of CG iterations.
#include <chrono>
#include <cstdarg>
#include <memory>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sn.h"
#include "sn_kernels.hpp"
#include "hp.hpp"
#include "mg_host.hpp"

using namespace sn;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return fail(SN_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    // grows only; returns 0 or an SN error code
    int ensure(size_t count) {
        if (count <= n && p) return 0;
        release();
        if (count == 0) count = 1;
        hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            return fail(SN_ERR_NOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
        }
        n = count;
        return 0;
    }
};

constexpr double kPi = 3.14159265358979323846;

}  // namespace

struct sn_context {
    sn_mesh mesh{};
    int nn = 4;
    long nc = 0;
    int ndirs = 0;
    long nbf = 0;
    double eta = 1.0;
    hipStream_t stream = nullptr;
    StreamSplit split{};  // 3D full sweeps: reflection classes over split.n streams (st[0] = stream)
    std::vector<DirInfo> hdirs;
    std::vector<double> hw, omega;
    DevBuf<double> wn;
    DevBuf<DirInfo> dirs;
    DevBuf<double> w, sigt, sigs;
    DevBuf<float> sigt32;
    // thick set and diffusion preconditioner
    int nthick = 0;
    DevBuf<int> flags, blocksums, total, slot, thick;
    DevBuf<double> binv;
    DsaGeom dg{};
    int nparts = 1;
    DevBuf<double> cx, cr, cz, cp, cp1, cq, parta, partb;
    DevBuf<int> nbr;
    DevBuf<CgScalars> scal;
    int cg_hint = 8, cg_hint2 = 8;  // CG iterations of the last two solves
    // 2D source iteration, FP64 form: the DSA's final update also wrote the
    // next sweep's source (srcskew64) from phi = src_tok_phi and
    // q = src_tok_q; the next sweep then skips its source kernel
    bool src_tok = false;
    const double* src_tok_phi = nullptr;
    const double* src_tok_q = nullptr;
    // pinned host copies of the device scalars (async read-back) and the
    // event that marks the latest residual copy
    struct HostScalars {
        double r3[4];
        CgScalars cs;
    };
    HostScalars* hpin = nullptr;
    hipEvent_t res_ev = nullptr, cg_ev = nullptr;
    // geometric multigrid hierarchy (built on first use)
    bool mg_ready = false;
    int mg_lc = 1, mg_levels = 0;
    double mg_omega0 = 0.8;
    MgDev mg{};
    DevBuf<double> mg_coef, mg_pw, mg_b, mg_x, mg_y, mg_r, mg_ainv, cz0, cres;
    DevBuf<int> mg_nbr, mg_chl, mg_par, mg_vnodes, mg_nodev;
    // sweep
    SweepGeom sg{};
    DevBuf<int> tiles, groups;
    std::vector<int> plane_off;
    DevBuf<double> xf64, yf64, zf64, src64, sink64, sigskew64, srcskew64;
    DevBuf<float> xf32, yf32, zf32, src32, sink32, sigskew32, srcskew32;
    // source iteration workspace
    DevBuf<double> psi64, phisi, phitmp, phiprev, rpart, res3, phioct, fpart;
    DevBuf<float> psi32;
    int nrpart = 1;
    // Face buffers of each precision hold the inflow of the last
    // initialisation (slot 0 is never overwritten by a sweep).  Within one
    // source-iteration call, where the inflow array does not change, a sweep
    // with the same inflow pointer and transpose flag skips the
    // initialisation.
    struct FaceKey {
        const double* inflow = nullptr;
        int transpose = 0;
        bool valid = false;
    };
    FaceKey fkey[2];  // [FP64, FP32]
    bool face_reuse = false;
    // direction parts for sweeps that keep only some directions' psi (the
    // adjoint contraction and the face response): 3D one reflection class
    // (octant) each, 2D one quadrant each; part_dirs[p][l] = global direction
    // of local index l (-1: unused slot), part_w = [part][part_stride] weights
    std::vector<SweepPart> parts;
    std::vector<std::vector<int>> part_dirs;
    int part_stride = 0;
    DevBuf<int> order2d_parts, face_out;
    DevBuf<double> part_w, part_wn, psi_a, psi_b;
    // triangular DSA (Alg. 1): the iterate before the thick update, the thick
    // part of the preconditioned residual and its transport update
    DevBuf<double> phiold, phibar, zeta;
    // Krylov solve: basis V [m + 1][n], preconditioned basis Z [m][n], work
    // vectors, the zero vector, dot products and their pinned host copy
    DevBuf<double> kv, kz, kw, kb, kzero, kdot, kpart;
    double* kdot_host = nullptr;
    // GMRES inner solve of the nonsymmetric diffusion forms: full inverse
    // diagonal blocks of form binvf_op (-1: none yet), basis [restart + 1][nf],
    // dot products and their pinned copy, the singular-block flag
    DevBuf<double> binvf, gv, gdot, gpart, gb, gu, gz;
    DevBuf<int> gbad;
    double* gdot_host = nullptr;
    int binvf_op = -1;
    // order p >= 2 (2D): the tables, the thick block rows of form hblk_op
    // (-1: none yet) and their columns, and a copy of dg with the Q1 node
    // count (for the neighbour-table and band-width kernels, which only use
    // the dimension)
    int order = 1;
    HpTab hp{};
    DevBuf<double> hblk;
    DevBuf<int> hcol;
    int hblk_op = -1;
    DsaGeom dg4{};
    // exact thick solve: band LU factors of form band_op (-1: none yet)
    DevBuf<double> band;
    DevBuf<int> bpiv;
    int band_op = -1, band_kl = 0, band_ku = 0, band_ldb = 0;
    int sweeps = 0;  // transport sweeps (all directions) since the last reset
    // device address of the fixed scratch of the entry points that allocate
    // nothing on this context's device (NULL if its lookup failed)
    double* noalloc = nullptr;
    hipError_t noalloc_err = hipSuccess;
    // optional event timing of the sweep kernels and of the DSA solves
    int timing = 0;
    std::vector<hipEvent_t> evpool;
    size_t evused = 0;
    std::vector<std::pair<size_t, size_t>> sweep_ev, dsa_ev;
};

namespace {

// next event of the pool, recorded on the context stream (nullptr if disabled)
int record_event(sn_context* ctx, size_t* idx) {
    if (ctx->evused == ctx->evpool.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        ctx->evpool.push_back(e);
    }
    *idx = ctx->evused++;
    HIPCHK(hipEventRecord(ctx->evpool[*idx], ctx->stream));
    return 0;
}

int check_mesh(const sn_mesh* m) {
    if (!m) return fail(SN_ERR_INVALID, "mesh is NULL");
    if (m->dim != 2 && m->dim != 3) return fail(SN_ERR_INVALID, "dim must be 2 or 3 (got %d)", m->dim);
    if (m->nx <= 0 || m->ny <= 0 || m->nz <= 0) return fail(SN_ERR_INVALID, "cell counts must be positive");
    if (m->dim == 2 && m->nz != 1) return fail(SN_ERR_INVALID, "2D mesh needs nz = 1");
    if (!(m->hx > 0) || !(m->hy > 0) || (m->dim == 3 && !(m->hz > 0)) || !std::isfinite(m->hx) ||
        !std::isfinite(m->hy) || !std::isfinite(m->hz))
        return fail(SN_ERR_INVALID, "cell widths must be positive and finite");
    long nc = (long)m->nx * m->ny * m->nz;
    if (nc > (1L << 31) - 1) return fail(SN_ERR_UNSUPPORTED, "more than 2^31 - 1 cells");
    if (m->order < 0 || m->order > 4) return fail(SN_ERR_INVALID, "order must be 0..4 (got %d)", m->order);
    if (m->order >= 2 && m->dim != 2) return fail(SN_ERR_UNSUPPORTED, "order %d is built for 2D only", m->order);
    return 0;
}

long inflow_size(const sn_mesh* m) {
    if (m->order >= 2) return (long)(m->order + 1) * (m->nx + m->ny);
    if (m->dim == 2) return 2L * m->ny + 2L * m->nx;
    return 4L * ((long)m->ny * m->nz + (long)m->nx * m->nz + (long)m->nx * m->ny);
}

// The sweep's face buffers.  3D: x faces per direction in xf, the y/z face
// slots of every direction group and tile in yf; 2D: x and y per direction.
template <typename T>
struct Faces {
    T *x, *y, *z;
};
template <typename T>
int face_views(sn_context* ctx, DevBuf<T>& xf, DevBuf<T>& yf, DevBuf<T>& zf, Faces<T>* f) {
    const SweepGeom& g = ctx->sg;
    int rc;
    if (g.dim == 3) {
        if ((rc = xf.ensure((size_t)g.xstride * g.ndirs))) return rc;
        if ((rc = yf.ensure((size_t)yz_face_elems(g.nclasses * g.groups_per_class, g.nTx, g.nTy, g.nTz, g.TX))))
            return rc;
        *f = Faces<T>{xf.p, yf.p, nullptr};
        return 0;
    }
    if ((rc = xf.ensure((size_t)g.xstride * g.ndirs))) return rc;
    if ((rc = yf.ensure((size_t)g.ystride * g.ndirs))) return rc;
    if ((rc = zf.ensure(1))) return rc;
    *f = Faces<T>{xf.p, yf.p, zf.p};
    return 0;
}

template <typename T>
int init_faces(sn_context* ctx, const double* inflow, int transpose, const Faces<T>& f) {
    sn_context::FaceKey& k = ctx->fkey[sizeof(T) == 8 ? 0 : 1];
    if (ctx->face_reuse && k.valid && k.inflow == inflow && k.transpose == transpose) return 0;
    HIPCHK(launch_init_faces<T>(ctx->sg, ctx->dirs.p, transpose, inflow, f.x, f.y, f.z, ctx->stream));
    k.inflow = inflow;
    k.transpose = transpose;
    k.valid = true;
    return 0;
}

// the 2D diagonal-major source array, allocated with zero padding
template <typename T>
int ensure_skew(sn_context* ctx, DevBuf<T>& srcskew) {
    const size_t ne = (size_t)skew2d_elems(ctx->sg.nx, ctx->sg.ny, 4);
    const bool fresh = srcskew.n < ne || !srcskew.p;
    int rc;
    if ((rc = srcskew.ensure(ne))) return rc;
    if (fresh) HIPCHK(hipMemsetAsync(srcskew.p, 0, ne * sizeof(T), ctx->stream));  // padding stays zero
    return 0;
}

template <typename T>
int sweep_impl(sn_context* ctx, const double* phi, const double* phi_prev, const double* q, const double* inflow,
               int transpose, T* psi, DevBuf<T>& xf, DevBuf<T>& yf, DevBuf<T>& zf, DevBuf<T>& src, DevBuf<T>& sink,
               const T* sigt, DevBuf<T>& srcskew, const T* sigskew, const SweepPart* part = nullptr) {
    const SweepGeom& g = ctx->sg;
    int rc;
    Faces<T> f;
    if ((rc = face_views(ctx, xf, yf, zf, &f))) return rc;
    if ((rc = sink.ensure((size_t)sink_elems(g)))) return rc;
    const T* sweep_src;
    const T* sweep_sig = sigt;
    if (g.dim == 2) {
        if ((rc = ensure_skew(ctx, srcskew))) return rc;
        const bool ready = std::is_same<T, double>::value && ctx->src_tok && ctx->src_tok_phi == phi &&
                           ctx->src_tok_q == q && !phi_prev;
        ctx->src_tok = false;
        if (!ready)
            HIPCHK(launch_source_skew2d<T>(g.nx, g.ny, ctx->sigs.p, phi, phi_prev, q, srcskew.p, ctx->stream));
        sweep_src = srcskew.p;
        sweep_sig = sigskew;
    } else {
        if ((rc = src.ensure((size_t)ctx->nc * ctx->nn))) return rc;
        HIPCHK(launch_source<T>(ctx->nc, ctx->nn, ctx->sigs.p, phi, phi_prev, q, src.p, ctx->stream));
        sweep_src = src.p;
    }
    if ((rc = init_faces<T>(ctx, inflow, transpose, f))) return rc;
    size_t e0 = 0, e1 = 0;
    if (ctx->timing && (rc = record_event(ctx, &e0))) return rc;
    HIPCHK(launch_sweep<T>(g, ctx->dirs.p, transpose, sweep_sig, sweep_src, f.x, f.y, f.z, ctx->tiles.p,
                           ctx->plane_off.data(), psi, sink.p, ctx->stream, part, &ctx->split));
    if (!part) ++ctx->sweeps;
    if (ctx->timing) {
        if ((rc = record_event(ctx, &e1))) return rc;
        ctx->sweep_ev.emplace_back(e0, e1);
    }
    return 0;
}

// psi = L^{-1} or L^{-T} of the load of (sigma_s (phi - phi_prev) + q)/4pi plus the inflow
int do_sweep(sn_context* ctx, const double* phi, const double* phi_prev, const double* q, const double* inflow,
             int transpose, sn_precision prec, void* psi, const SweepPart* part = nullptr) {
    if (prec == SN_FP64)
        return sweep_impl<double>(ctx, phi, phi_prev, q, inflow, transpose, (double*)psi, ctx->xf64, ctx->yf64,
                                  ctx->zf64, ctx->src64, ctx->sink64, ctx->sigt.p, ctx->srcskew64, ctx->sigskew64.p,
                                  part);
    return sweep_impl<float>(ctx, phi, phi_prev, q, inflow, transpose, (float*)psi, ctx->xf32, ctx->yf32, ctx->zf32,
                             ctx->src32, ctx->sink32, ctx->sigt32.p, ctx->srcskew32, ctx->sigskew32.p, part);
}

// res_ref != nullptr: also the residual partial sums against res_ref into
// ctx->fpart (moment_blocks(nc) blocks)
int do_moment(sn_context* ctx, const void* psi, sn_precision prec, double* phi, int accumulate = 0,
              const double* res_ref = nullptr) {
    if (prec == SN_FP64)
        HIPCHK(launch_moment<double>(ctx->nc, ctx->nn, ctx->ndirs, ctx->w.p, (const double*)psi, phi, accumulate,
                                     res_ref, ctx->fpart.p, ctx->stream));
    else
        HIPCHK(launch_moment<float>(ctx->nc, ctx->nn, ctx->ndirs, ctx->w.p, (const float*)psi, phi, accumulate,
                                    res_ref, ctx->fpart.p, ctx->stream));
    return 0;
}

// 3D fused sweep + moment in precision T: phi_out (+)= sum_d w_d psi_d, psi not stored
template <typename T>
int sweep_flux3d_impl(sn_context* ctx, const double* phi, const double* phi_prev, const double* q,
                      const double* inflow, int transpose, double* phi_out, int accumulate, DevBuf<T>& xf,
                      DevBuf<T>& yf, DevBuf<T>& zf, DevBuf<T>& src, const T* sigt, const double* res_ref) {
    const SweepGeom& g = ctx->sg;
    int rc;
    Faces<T> f;
    if ((rc = face_views(ctx, xf, yf, zf, &f))) return rc;
    if ((rc = src.ensure((size_t)ctx->nc * ctx->nn))) return rc;
    if ((rc = ctx->phioct.ensure((size_t)g.nclasses * ctx->nc * 8))) return rc;
    HIPCHK(launch_source<T>(ctx->nc, ctx->nn, ctx->sigs.p, phi, phi_prev, q, src.p, ctx->stream));
    if ((rc = init_faces<T>(ctx, inflow, transpose, f))) return rc;
    size_t e0 = 0, e1 = 0;
    if (ctx->timing && (rc = record_event(ctx, &e0))) return rc;
    HIPCHK(launch_sweep_flux3d<T>(g, ctx->dirs.p, ctx->w.p, transpose, sigt, src.p, f.x, f.y, f.z, ctx->tiles.p,
                                  ctx->plane_off.data(), ctx->phioct.p, phi_out, accumulate, res_ref, ctx->fpart.p,
                                  ctx->stream, &ctx->split));
    ++ctx->sweeps;
    if (ctx->timing) {
        if ((rc = record_event(ctx, &e1))) return rc;
        ctx->sweep_ev.emplace_back(e0, e1);
    }
    return 0;
}

// phi_out (+)= sum_d w_d L_d^{-1}(...) for source iteration: in 3D the fused
// kernels (psi never reaches memory); in 2D a psi-writing sweep into the
// context's psi workspace followed by the moment.  res_ref != nullptr: the
// last kernel also writes the residual partial sums of phi_out against
// res_ref into ctx->fpart; returns their block count in *res_nparts.
int do_sweep_flux(sn_context* ctx, const double* phi, const double* phi_prev, const double* q, const double* inflow,
                  int transpose, sn_precision prec, double* phi_out, int accumulate, const double* res_ref = nullptr,
                  int* res_nparts = nullptr) {
    int rc;
    if (res_ref) {
        const int nb = std::max(moment_blocks(ctx->nc), octant_sum_blocks(ctx->nc));
        if ((rc = ctx->fpart.ensure(3 * (size_t)nb))) return rc;
        *res_nparts = ctx->mesh.dim == 3 ? octant_sum_blocks(ctx->nc) : moment_blocks(ctx->nc);
    }
    if (ctx->mesh.dim == 3) {
        if (prec == SN_FP64)
            return sweep_flux3d_impl<double>(ctx, phi, phi_prev, q, inflow, transpose, phi_out, accumulate,
                                             ctx->xf64, ctx->yf64, ctx->zf64, ctx->src64, ctx->sigt.p, res_ref);
        return sweep_flux3d_impl<float>(ctx, phi, phi_prev, q, inflow, transpose, phi_out, accumulate, ctx->xf32,
                                        ctx->yf32, ctx->zf32, ctx->src32, ctx->sigt32.p, res_ref);
    }
    const size_t npsi = (size_t)ctx->nc * ctx->ndirs * ctx->nn;
    void* psi;
    if (prec == SN_FP64) {
        if ((rc = ctx->psi64.ensure(npsi))) return rc;
        psi = ctx->psi64.p;
    } else {
        if ((rc = ctx->psi32.ensure(npsi))) return rc;
        psi = ctx->psi32.p;
    }
    if ((rc = do_sweep(ctx, phi, phi_prev, q, inflow, transpose, prec, psi))) return rc;
    return do_moment(ctx, psi, prec, phi_out, accumulate, res_ref);
}

// phi_out = phi_si + P_T delta; returns an SN code; fills stats
double env_double(const char* name, double dflt) {
    const char* e = std::getenv(name);
    return e ? std::atof(e) : dflt;
}

// Inverse of a symmetric positive definite matrix (row-major, n x n) by
// Cholesky factorisation; returns false if a pivot is not positive.
bool spd_inverse(int n, std::vector<double>& a, std::vector<double>& inv) {
    for (int j = 0; j < n; ++j) {
        double d = a[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        a[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double v = a[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) v -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
            a[(size_t)i * n + j] = v / d;
        }
    }
    inv.assign((size_t)n * n, 0.0);
    std::vector<double> y(n);
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < n; ++i) {  // L y = e_c
            double v = i == c ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= a[(size_t)i * n + k] * y[k];
            y[i] = v / a[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {  // L^T x = y
            double v = y[i];
            for (int k = i + 1; k < n; ++k) v -= a[(size_t)k * n + i] * inv[(size_t)k * n + c];
            inv[(size_t)i * n + c] = v / a[(size_t)i * n + i];
        }
    }
    return true;
}

// Multigrid hierarchy for the thick-region operator.  Level 1: the vertices
// of the thick cells (continuous Q1), stencil P^T D_ff P by probing on the
// device.  Coarser levels (host, sums in a fixed order): every other vertex,
// (bi/tri)linear interpolation, Galerkin stencils, until at most 256 unknowns
// remain; that operator is inverted densely.
int mg_setup(sn_context* c) {
    const DsaGeom& g = c->dg;
    const int nt = g.nthick, dim = g.dim, nn = c->nn, nch = 1 << dim, ns = dim == 2 ? 9 : 27;
    int rc;
    std::vector<MgLevelHost> lv(2);
    MgLevelHost& l1 = lv[1];
    l1.nvx = g.nx + 1;
    l1.nvy = g.ny + 1;
    l1.nvz = dim == 3 ? g.nz + 1 : 1;
    std::vector<int> tc(nt);
    HIPCHK(hipMemcpyAsync(tc.data(), c->thick.p, nt * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    l1.slot.assign((size_t)l1.nvx * l1.nvy * l1.nvz, -1);
    auto vtx = [&](int s, int q) {
        const long cell = tc[s];
        const int i = (int)(cell % g.nx), j = (int)((cell / g.nx) % g.ny), k = (int)(cell / ((long)g.nx * g.ny));
        return ((long)(k + ((q >> 2) & 1)) * l1.nvy + j + ((q >> 1) & 1)) * l1.nvx + i + (q & 1);
    };
    for (int s = 0; s < nt; ++s)
        for (int q = 0; q < nch; ++q) l1.slot[vtx(s, q)] = 0;
    for (long v = 0; v < (long)l1.slot.size(); ++v)
        if (l1.slot[v] == 0) {
            l1.slot[v] = (int)l1.pos.size();
            l1.pos.push_back(v);
        }
    const int n1 = (int)l1.pos.size();
    std::vector<int> vnodes((size_t)n1 * nch, -1), nodev((size_t)nt * nn);
    for (int s = 0; s < nt; ++s)
        for (int q = 0; q < nch; ++q) {
            const int w = l1.slot[vtx(s, q)];
            vnodes[(size_t)w * nch + q] = s * nn + q;
            nodev[(size_t)s * nn + q] = w;
        }
    DevBuf<long> vpos;
    DevBuf<double> coef1;
    if ((rc = vpos.ensure(n1)) || (rc = coef1.ensure((size_t)n1 * ns)) || (rc = c->mg_vnodes.ensure(vnodes.size())) ||
        (rc = c->mg_nodev.ensure(nodev.size())) || (rc = c->cz0.ensure((size_t)nt * nn)) ||
        (rc = c->cres.ensure((size_t)nt * nn)))
        return rc;
    HIPCHK(hipMemcpy(vpos.p, l1.pos.data(), n1 * sizeof(long), hipMemcpyHostToDevice));
    {
        std::vector<int> vt(vnodes.size());   // offset-major on the device
        for (int w = 0; w < n1; ++w)
            for (int q = 0; q < nch; ++q) vt[(size_t)q * n1 + w] = vnodes[(size_t)w * nch + q];
        HIPCHK(hipMemcpy(c->mg_vnodes.p, vt.data(), vt.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(c->mg_nodev.p, nodev.data(), nodev.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(coef1.p, 0, (size_t)n1 * ns * sizeof(double)));
    MgDev& m = c->mg;
    m = MgDev{};
    m.dim = dim;
    m.ns = ns;
    m.n[1] = n1;
    m.vnodes = c->mg_vnodes.p;
    m.nodev = c->mg_nodev.p;
    HIPCHK(launch_vmg_probe(g, c->thick.p, c->slot.p, c->sigt.p, c->sigs.p, m, l1.nvx, l1.nvy, vpos.p, c->cz0.p,
                            c->cres.p, coef1.p, c->stream));
    l1.coef.resize((size_t)n1 * ns);
    HIPCHK(hipMemcpyAsync(l1.coef.data(), coef1.p, l1.coef.size() * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    mg_coarsen(lv, dim, 256, MG_MAXL);
    const int L = (int)lv.size() - 1;
    // dense inverse of the coarsest operator
    const int nL = (int)lv[L].pos.size();
    std::vector<double> A((size_t)nL * nL, 0.0), Ainv;
    for (int i = 0; i < nL; ++i)
        for (int o = 0; o < ns; ++o) {
            const int j = lv[L].nbr[(size_t)i * ns + o];
            if (j >= 0) A[(size_t)i * nL + j] += lv[L].coef[(size_t)i * ns + o];
        }
    if (!spd_inverse(nL, A, Ainv)) return fail(SN_ERR_CG_BREAKDOWN, "coarsest multigrid operator is not SPD");
    // flatten
    m.L = L;
    long nv = 0, np = 0;
    for (int l = 1; l <= L; ++l) {
        m.n[l] = (int)lv[l].pos.size();
        m.vo[l] = nv;
        m.so[l] = nv * ns;
        m.po[l] = np;
        nv += m.n[l];
        if (l < L) np += (long)m.n[l] * nch;
    }
    std::vector<double> coef((size_t)nv * ns), pw(std::max<long>(np, 1), 0.0);
    std::vector<int> nbr((size_t)nv * ns), chl((size_t)nv * ns, -1), par(std::max<long>(np, 1), -1);
    // device tables are offset-major within each level
    for (int l = 1; l <= L; ++l) {
        const long n = m.n[l];
        for (long f = 0; f < n; ++f) {
            for (int o = 0; o < ns; ++o) {
                coef[m.so[l] + o * n + f] = lv[l].coef[(size_t)f * ns + o];
                nbr[m.so[l] + o * n + f] = lv[l].nbr[(size_t)f * ns + o];
                if (l >= 2) chl[m.so[l] + o * n + f] = lv[l].chl[(size_t)f * ns + o];
            }
            if (l < L)
                for (int q = 0; q < nch; ++q) {
                    par[m.po[l] + q * n + f] = lv[l].par[(size_t)f * nch + q];
                    pw[m.po[l] + q * n + f] = lv[l].pw[(size_t)f * nch + q];
                }
        }
    }
    if ((rc = c->mg_coef.ensure(coef.size())) || (rc = c->mg_nbr.ensure(nbr.size())) ||
        (rc = c->mg_chl.ensure(chl.size())) || (rc = c->mg_par.ensure(par.size())) ||
        (rc = c->mg_pw.ensure(pw.size())) || (rc = c->mg_b.ensure(nv)) || (rc = c->mg_x.ensure(nv)) ||
        (rc = c->mg_y.ensure(nv)) || (rc = c->mg_r.ensure(nv)) || (rc = c->mg_ainv.ensure(Ainv.size())))
        return rc;
    HIPCHK(hipMemcpy(c->mg_coef.p, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->mg_nbr.p, nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->mg_chl.p, chl.data(), chl.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->mg_par.p, par.data(), par.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->mg_pw.p, pw.data(), pw.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->mg_ainv.p, Ainv.data(), Ainv.size() * sizeof(double), hipMemcpyHostToDevice));
    m.coef = c->mg_coef.p;
    m.nbr = c->mg_nbr.p;
    m.chl = c->mg_chl.p;
    m.par = c->mg_par.p;
    m.pw = c->mg_pw.p;
    m.b = c->mg_b.p;
    m.x = c->mg_x.p;
    m.y = c->mg_y.p;
    m.r = c->mg_r.p;
    m.ainv = c->mg_ainv.p;
    m.omega = env_double("SN_MG_OMEGA", 0.7);
    c->mg_omega0 = env_double("SN_MG_OMEGA0", 0.8);
    // the smallest levels (at most SN_MG_COARSE unknowns, default 2048) run
    // in the single-workgroup kernel, the others as grid-wide kernels
    const int small = (int)env_double("SN_MG_COARSE", 2048);
    int lc = L;
    while (lc > 1 && m.n[lc - 1] <= small) --lc;
    c->mg_lc = lc;
    c->mg_levels = L;
    c->mg_ready = true;
    return 0;
}

bool bad_dsa_opts(const sn_dsa_opts& o) {
    return !(o.cg_rtol >= 0) || o.cg_maxit < 1 || (o.mass_kind != 0 && o.mass_kind != 1) ||
           (o.precond != SN_PRECOND_BLOCK_JACOBI && o.precond != SN_PRECOND_MG &&
            o.precond != SN_PRECOND_DIRECT) ||
           (o.diffusion != SN_DIFFUSION_SIP && o.diffusion != SN_DIFFUSION_NIP &&
            o.diffusion != SN_DIFFUSION_MNIP);
}

// The thick solve D_ff x = b of a nonsymmetric form (NIP, mNIP) by
// GMRES(SN_DSA_GMRES_RESTART) right-preconditioned by M: D M^{-1} u = b from
// u = 0, x = M^{-1} u into ctx->cx.  M^{-1} is the inverse of the form's own
// diagonal blocks (block Jacobi, fused into the operator kernel), or one
// V-cycle of the SIP multigrid (a fixed linear map, so the basis of u need
// not be kept preconditioned).  Classical
// Gram-Schmidt twice, each pass one reduction that also yields the squared
// norm of the vector it orthogonalises (the new vector is formed in its basis
// slot, V_{j+1}); the norm after the second pass is ||w||^2 - |h2|^2, the
// second pass's coefficients being tiny.  Each restart starts from the true
// residual b - D B^{-1} u, the stop test of the last restart.
// The full inverse diagonal blocks of a nonsymmetric form, built once per
// form; also the check that mNIP is defined (sigma_t > 0 at every thick cell
// and its face neighbours).
int form_blocks(sn_context* ctx, int op) {
    const DsaGeom& g = ctx->dg;
    int rc;
    if ((rc = ctx->binvf.ensure((size_t)ctx->nthick * ctx->nn * ctx->nn)) || (rc = ctx->gbad.ensure(1))) return rc;
    if (ctx->binvf_op != op) {
        HIPCHK(hipMemsetAsync(ctx->gbad.p, 0, sizeof(int), ctx->stream));
        HIPCHK(launch_block_inverse_full(g, op, ctx->thick.p, ctx->nbr.p, ctx->sigt.p, ctx->sigs.p, ctx->binvf.p,
                                         ctx->gbad.p, ctx->stream));
        int bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, ctx->gbad.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (bad) {
            ctx->binvf_op = -1;
            return fail(SN_ERR_INVALID, op == SN_DIFFUSION_MNIP
                                            ? "mNIP diffusion: sigma_t <= 0 at a thick cell or its neighbour, or a "
                                              "singular diagonal block"
                                            : "NIP diffusion: singular diagonal block");
        }
        ctx->binvf_op = op;
    }
    return 0;
}

// The exact thick solve of any form for small systems: the band LU factors,
// built on the device once per form (SN_ERR_UNSUPPORTED beyond the solve
// kernel's limits: nthick nn <= 8192 unknowns, kl + ku < 1024), then
// x = D^{-1} b into ctx->cx.
int dsa_direct(sn_context* ctx, const double* phi_old, const double* phi_si, const sn_dsa_opts* o) {
    const DsaGeom& g = ctx->dg;
    const long nf = (long)ctx->nthick * ctx->nn;
    const int op = o->diffusion;
    int rc;
    if (op != SN_DIFFUSION_SIP && (rc = form_blocks(ctx, op))) return rc;
    if (ctx->band_op != op) {
        if (nf > kBandSolveMaxN)
            return fail(SN_ERR_UNSUPPORTED, "direct thick solve: %ld unknowns exceed %ld", nf, kBandSolveMaxN);
        if ((rc = ctx->gbad.ensure(1))) return rc;
        HIPCHK(hipMemsetAsync(ctx->gbad.p, 0, sizeof(int), ctx->stream));
        HIPCHK(launch_band_width(g, ctx->nbr.p, ctx->gbad.p, ctx->stream));
        int wc = 0;
        HIPCHK(hipMemcpyAsync(&wc, ctx->gbad.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        const int kl = (wc + 1) * ctx->nn - 1, ku = kl;
        if (kl + ku > kBandMaxWidth)
            return fail(SN_ERR_UNSUPPORTED, "direct thick solve: band half width %d too large", kl);
        const int ldb = 2 * kl + ku + 1;
        if ((rc = ctx->band.ensure((size_t)nf * ldb)) || (rc = ctx->bpiv.ensure(nf)) || (rc = ctx->gb.ensure(nf)))
            return rc;
        ctx->band_op = -1;
        HIPCHK(hipMemsetAsync(ctx->band.p, 0, (size_t)nf * ldb * sizeof(double), ctx->stream));
        HIPCHK(launch_band_assemble(g, op, ctx->thick.p, ctx->nbr.p, ctx->sigt.p, ctx->sigs.p, kl, ldb, ctx->band.p,
                                    ctx->stream));
        HIPCHK(hipMemsetAsync(ctx->gbad.p, 0, sizeof(int), ctx->stream));
        HIPCHK(launch_band_factor(nf, kl, ku, ldb, ctx->band.p, ctx->bpiv.p, ctx->gbad.p, ctx->stream));
        int bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, ctx->gbad.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (bad) return fail(SN_ERR_INVALID, "direct thick solve: the diffusion matrix is singular");
        ctx->band_op = op;
        ctx->band_kl = kl;
        ctx->band_ku = ku;
        ctx->band_ldb = ldb;
    }
    HIPCHK(launch_dsa_rhs_vec(g, ctx->thick.p, ctx->sigt.p, ctx->sigs.p, o->mass_kind, phi_old, phi_si, ctx->gb.p,
                              ctx->stream));
    HIPCHK(launch_band_solve(nf, ctx->band_kl, ctx->band_ku, ctx->band_ldb, ctx->band.p, ctx->bpiv.p, ctx->gb.p,
                             ctx->cx.p, ctx->stream));
    return 0;
}

// GMRES(SN_DSA_GMRES_RESTART) on the thick vector (nf values): D M^{-1} u = b
// from u = 0, b in ctx->gb, u in ctx->gu.  apply(v, bb, w) writes
// w = D M^{-1} v, or bb - D M^{-1} v when bb is given; finish(u) forms
// x = M^{-1} u in ctx->cx.  Stops on the true residual of a restart.
template <typename Apply, typename Finish>
int gmres_core(sn_context* ctx, long nf, const sn_dsa_opts* o, Apply apply, Finish finish, int* iters,
               double* relres) {
    const int m = SN_DSA_GMRES_RESTART;
    int rc;
    if ((rc = ctx->gv.ensure((size_t)(m + 1) * nf)) || (rc = ctx->gdot.ensure(m + 2)) ||
        (rc = ctx->gpart.ensure((size_t)(m + 2) * krylov_blocks(nf))))
        return rc;
    if (!ctx->gdot_host)
        HIPCHK(hipHostMalloc((void**)&ctx->gdot_host, (m + 2) * sizeof(double), hipHostMallocDefault));
    double* V = ctx->gv.p;
    double* b = ctx->gb.p;
    double* u = ctx->gu.p;
    auto dotk = [&](int k, const double* Vb, const double* w, double* out) -> int {
        HIPCHK(launch_multi_dot(nf, k, Vb, w, ctx->gpart.p, ctx->gdot.p, ctx->gdot_host, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        for (int i = 0; i < k; ++i) out[i] = ctx->gdot_host[i];
        return 0;
    };
    HIPCHK(hipMemsetAsync(u, 0, nf * sizeof(double), ctx->stream));
    double bb;
    if ((rc = dotk(1, b, b, &bb))) return rc;
    const double bnorm = std::sqrt(bb);
    if (!std::isfinite(bnorm)) return fail(SN_ERR_DIVERGED, "diffusion right-hand side is not finite");
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gg(m + 1), y(m), h(m + 2), h2(m + 2);
    int it = 0;
    double beta = bnorm;
    bool first = true;
    while (bnorm > 0.0) {
        if (first) {
            HIPCHK(hipMemcpyAsync(V, b, nf * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        } else {
            if ((rc = apply(u, b, V))) return rc;
            double rr;
            if ((rc = dotk(1, V, V, &rr))) return rc;
            beta = std::sqrt(rr);
        }
        first = false;
        if (!std::isfinite(beta)) return fail(SN_ERR_DIVERGED, "diffusion GMRES residual is not finite");
        if (beta <= o->cg_rtol * bnorm || it >= o->cg_maxit) break;
        HIPCHK(launch_scale(nf, 1.0 / beta, V, V, ctx->stream));
        std::fill(gg.begin(), gg.end(), 0.0);
        gg[0] = beta;
        int j = 0;
        for (; j < m && it < o->cg_maxit; ++j) {
            double* vn = V + (size_t)(j + 1) * nf;
            if ((rc = apply(V + (size_t)j * nf, nullptr, vn))) return rc;
            if ((rc = dotk(j + 2, V, vn, h.data()))) return rc;
            HIPCHK(launch_multi_axpy(nf, j + 1, V, ctx->gdot.p, -1.0, vn, ctx->stream));
            if ((rc = dotk(j + 2, V, vn, h2.data()))) return rc;
            HIPCHK(launch_multi_axpy(nf, j + 1, V, ctx->gdot.p, -1.0, vn, ctx->stream));
            double hh2 = 0.0;
            for (int i = 0; i <= j; ++i) hh2 += h2[i] * h2[i];
            const double hn = std::sqrt(std::max(0.0, h2[j + 1] - hh2));
            if (!std::isfinite(hn) || !std::isfinite(h[j + 1]))
                return fail(SN_ERR_DIVERGED, "diffusion GMRES residual is not finite");
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i] + h2[i];
            H[(size_t)(j + 1) * m + j] = hn;
            if (hn > 0.0) HIPCHK(launch_scale(nf, 1.0 / hn, vn, vn, ctx->stream));
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], c2 = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * c2;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c2;
            }
            const double a = H[(size_t)j * m + j], c2 = H[(size_t)(j + 1) * m + j];
            const double den = std::sqrt(a * a + c2 * c2);
            cs[j] = den > 0.0 ? a / den : 1.0;
            sn[j] = den > 0.0 ? c2 / den : 0.0;
            H[(size_t)j * m + j] = den;
            gg[j + 1] = -sn[j] * gg[j];
            gg[j] = cs[j] * gg[j];
            ++it;
            if (std::fabs(gg[j + 1]) <= o->cg_rtol * bnorm || hn == 0.0) {
                ++j;
                break;
            }
        }
        // u += V y, H(0:j, 0:j) y = g(0:j)
        for (int i = j - 1; i >= 0; --i) {
            double sum = gg[i];
            for (int k = i + 1; k < j; ++k) sum -= H[(size_t)i * m + k] * y[k];
            y[i] = sum / H[(size_t)i * m + i];
        }
        if (j > 0) {
            for (int i = 0; i < j; ++i) ctx->gdot_host[i] = y[i];
            HIPCHK(hipMemcpyAsync(ctx->gdot.p, ctx->gdot_host, j * sizeof(double), hipMemcpyHostToDevice,
                                  ctx->stream));
            HIPCHK(launch_multi_axpy(nf, j, V, ctx->gdot.p, 1.0, u, ctx->stream));
            // the pinned coefficients must not be overwritten before the copy ran
            HIPCHK(hipStreamSynchronize(ctx->stream));
        }
    }
    if ((rc = finish(u))) return rc;
    *iters = it;
    *relres = bnorm > 0.0 ? beta / bnorm : 0.0;
    return 0;
}

int dsa_gmres(sn_context* ctx, const double* phi_old, const double* phi_si, const sn_dsa_opts* o, int* iters,
              double* relres) {
    const DsaGeom& g = ctx->dg;
    const long nf = (long)ctx->nthick * ctx->nn;
    const int op = o->diffusion;
    int rc;
    const bool mg = o->precond == SN_PRECOND_MG;
    if ((rc = form_blocks(ctx, op))) return rc;
    if ((rc = ctx->gb.ensure(nf)) || (rc = ctx->gu.ensure(nf)) || (mg && (rc = ctx->gz.ensure(nf)))) return rc;
    if (mg && !ctx->mg_ready && (rc = mg_setup(ctx))) return rc;
    // the V-cycle kernels stop early once the CG status says done
    if (mg) HIPCHK(hipMemsetAsync(ctx->scal.p, 0, sizeof(CgScalars), ctx->stream));
    // out = M^{-1} v (multigrid only)
    auto vcycle = [&](const double* v, double* out) -> int {
        HIPCHK(launch_mg_vcycle(g, ctx->thick.p, ctx->nbr.p, ctx->sigt.p, ctx->sigs.p, ctx->binv.p, v, ctx->cz0.p,
                                ctx->cres.p, out, ctx->mg, ctx->mg_lc, ctx->mg_omega0, ctx->partb.p, ctx->nparts,
                                ctx->scal.p, ctx->stream));
        return 0;
    };
    auto apply = [&](const double* v, const double* bb_, double* w) -> int {
        int e;
        if (mg) {
            if ((e = vcycle(v, ctx->gz.p))) return e;
            HIPCHK(launch_nip_apply(g, op, ctx->thick.p, ctx->nbr.p, ctx->sigt.p, ctx->sigs.p, nullptr, ctx->gz.p,
                                    bb_, w, ctx->stream));
        } else {
            HIPCHK(launch_nip_apply(g, op, ctx->thick.p, ctx->nbr.p, ctx->sigt.p, ctx->sigs.p, ctx->binvf.p, v, bb_,
                                    w, ctx->stream));
        }
        return 0;
    };
    auto finish = [&](const double* u) -> int {
        if (mg) return vcycle(u, ctx->cx.p);
        HIPCHK(launch_full_block_apply(g, ctx->binvf.p, u, ctx->cx.p, ctx->stream));
        return 0;
    };
    HIPCHK(launch_dsa_rhs_vec(g, ctx->thick.p, ctx->sigt.p, ctx->sigs.p, o->mass_kind, phi_old, phi_si, ctx->gb.p,
                              ctx->stream));
    return gmres_core(ctx, nf, o, apply, finish, iters, relres);
}

// The thick correction at order p >= 2 (2D): the block rows of the form,
// assembled once per form (with the full inverse diagonal blocks), then
// GMRES right-preconditioned by those inverses or the exact band LU
// (SN_PRECOND_DIRECT, same limits as at order 1); x into ctx->cx, then the
// scatter phi_out = phi_si + P x.
int dsa_hp(sn_context* ctx, const double* phi_old, const double* phi_si, double* phi_out, const sn_dsa_opts* o,
           sn_dsa_stats* stats) {
    const long n = ctx->nc * ctx->nn;
    const int nn = ctx->nn, nt = ctx->nthick, op = o->diffusion;
    const long nf = (long)nt * nn;
    int its = 0;
    double rel = 0.0;
    int rc;
    if (o->precond == SN_PRECOND_MG)
        return fail(SN_ERR_UNSUPPORTED, "the multigrid preconditioner is built for order 1 only");
    if (nt == 0) {
        if (phi_out != phi_si)
            HIPCHK(hipMemcpyAsync(phi_out, phi_si, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    } else {
        if (ctx->hblk_op != op) {
            if ((rc = ctx->hblk.ensure((size_t)nt * 5 * nn * nn)) || (rc = ctx->hcol.ensure((size_t)nt * 5)) ||
                (rc = ctx->binvf.ensure((size_t)nt * nn * nn)) || (rc = ctx->gbad.ensure(1)))
                return rc;
            ctx->hblk_op = -1;
            ctx->band_op = -1;
            HIPCHK(hipMemsetAsync(ctx->gbad.p, 0, sizeof(int), ctx->stream));
            HIPCHK(launch_hp_assemble(ctx->hp, ctx->dg, op, ctx->thick.p, ctx->nbr.p, ctx->sigt.p, ctx->sigs.p,
                                      ctx->hblk.p, ctx->hcol.p, ctx->gbad.p, ctx->stream));
            HIPCHK(launch_hp_block_inverse(nn, nt, ctx->hblk.p, ctx->binvf.p, ctx->gbad.p, ctx->stream));
            int bad = 0;
            HIPCHK(hipMemcpyAsync(&bad, ctx->gbad.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
            if (bad)
                return fail(SN_ERR_INVALID, "order-%d diffusion: sigma_t <= 0 next to a thick cell (mNIP) or a "
                            "singular diagonal block", ctx->hp.p);
            ctx->hblk_op = op;
        }
        if ((rc = ctx->gb.ensure(nf)) || (rc = ctx->gu.ensure(nf)) || (rc = ctx->gz.ensure(nf))) return rc;
        HIPCHK(launch_hp_rhs(ctx->hp, nt, ctx->dg.h[0], ctx->dg.h[1], ctx->thick.p, ctx->sigt.p, ctx->sigs.p,
                             o->mass_kind, phi_old, phi_si, ctx->gb.p, ctx->stream));
        if (o->precond == SN_PRECOND_DIRECT) {
            if (ctx->band_op != op) {
                if (nf > kBandSolveMaxN)
                    return fail(SN_ERR_UNSUPPORTED, "direct thick solve: %ld unknowns exceed %ld", nf, kBandSolveMaxN);
                HIPCHK(hipMemsetAsync(ctx->gbad.p, 0, sizeof(int), ctx->stream));
                HIPCHK(launch_band_width(ctx->dg4, ctx->nbr.p, ctx->gbad.p, ctx->stream));
                int wc = 0;
                HIPCHK(hipMemcpyAsync(&wc, ctx->gbad.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
                HIPCHK(hipStreamSynchronize(ctx->stream));
                const int kl = (wc + 1) * nn - 1, ku = kl;
                if (kl + ku > kBandMaxWidth)
                    return fail(SN_ERR_UNSUPPORTED, "direct thick solve: band half width %d too large", kl);
                const int ldb = 2 * kl + ku + 1;
                if ((rc = ctx->band.ensure((size_t)nf * ldb)) || (rc = ctx->bpiv.ensure(nf))) return rc;
                HIPCHK(hipMemsetAsync(ctx->band.p, 0, (size_t)nf * ldb * sizeof(double), ctx->stream));
                HIPCHK(launch_hp_band(nn, nt, ctx->hblk.p, ctx->hcol.p, kl, ldb, ctx->band.p, ctx->stream));
                HIPCHK(hipMemsetAsync(ctx->gbad.p, 0, sizeof(int), ctx->stream));
                HIPCHK(launch_band_factor(nf, kl, ku, ldb, ctx->band.p, ctx->bpiv.p, ctx->gbad.p, ctx->stream));
                int bad = 0;
                HIPCHK(hipMemcpyAsync(&bad, ctx->gbad.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
                HIPCHK(hipStreamSynchronize(ctx->stream));
                if (bad) return fail(SN_ERR_INVALID, "direct thick solve: the diffusion matrix is singular");
                ctx->band_op = op;
                ctx->band_kl = kl;
                ctx->band_ku = ku;
                ctx->band_ldb = ldb;
            }
            HIPCHK(launch_band_solve(nf, ctx->band_kl, ctx->band_ku, ctx->band_ldb, ctx->band.p, ctx->bpiv.p,
                                     ctx->gb.p, ctx->cx.p, ctx->stream));
        } else {
            auto apply = [&](const double* v, const double* bb_, double* w) -> int {
                HIPCHK(launch_hp_block_apply(nn, nt, ctx->binvf.p, v, ctx->gz.p, ctx->stream));
                HIPCHK(launch_hp_spmv(nn, nt, ctx->hblk.p, ctx->hcol.p, ctx->gz.p, bb_, w, ctx->stream));
                return 0;
            };
            auto finish = [&](const double* u) -> int {
                HIPCHK(launch_hp_block_apply(nn, nt, ctx->binvf.p, u, ctx->cx.p, ctx->stream));
                return 0;
            };
            if ((rc = gmres_core(ctx, nf, o, apply, finish, &its, &rel))) return rc;
        }
        HIPCHK(launch_dsa_scatter(ctx->nc, nn, ctx->slot.p, phi_si, ctx->cx.p, phi_out, ctx->stream));
    }
    if (stats) {
        stats->cg_iters = its;
        stats->cg_relres = rel;
        stats->n_thick_cells = nt;
    }
    return 0;
}

int residual3(sn_context* ctx, const double* a, const double* b, double out[3]);

// Source iteration at order p >= 2 (eq. DSA_fp; FP64, forward, diagonal
// DSA): phi_SI = moment of the sweep of (sigma_s phi + q)/4pi, the stop test
// ||phi_SI - phi|| / ||b|| before the DSA step (b: the moment of the sweep of
// q from phi = 0), then phi = phi_SI + P_T D_ff^{-1} Sigma_f R_T (phi_SI - phi).
int si_hp(sn_context* ctx, const double* q, const double* inflow, double* phi, const sn_iter_opts* o,
          sn_iter_stats* stats, std::chrono::steady_clock::time_point t0) {
    if (o->prec != SN_FP64 || o->transpose || o->dsa_form != SN_DSA_DIAGONAL || o->phi_ckpt)
        return fail(SN_ERR_UNSUPPORTED, "order %d: FP64 forward source iteration with the diagonal DSA and no "
                    "checkpoints only", ctx->order);
    const long n = ctx->nc * ctx->nn;
    int rc;
    if ((rc = ctx->phisi.ensure(n)) || (rc = ctx->psi64.ensure((size_t)n * ctx->ndirs))) return rc;
    ctx->sweeps = 0;
    auto sweep_moment = [&](const double* ph, double* out) -> int {
        HIPCHK(launch_sweep_hp(ctx->hp, ctx->mesh.nx, ctx->mesh.ny, ctx->ndirs, ctx->nbf, ctx->dirs.p, ctx->sigt.p,
                               ctx->sigs.p, ph, q, inflow, ctx->psi64.p, ctx->stream));
        HIPCHK(launch_moment_hp(ctx->nc, ctx->ndirs, ctx->nn, ctx->w.p, ctx->psi64.p, out, ctx->stream));
        ++ctx->sweeps;
        return 0;
    };
    double r3[3];
    if ((rc = sweep_moment(nullptr, ctx->phisi.p)) || (rc = residual3(ctx, ctx->phisi.p, ctx->phisi.p, r3)))
        return rc;
    double bnorm = std::sqrt(r3[1]);
    if (bnorm == 0.0) bnorm = 1.0;
    int it = 0, status = SN_ERR_NOT_CONVERGED;
    double first = -1.0;
    for (; it < o->max_it;) {
        if ((rc = sweep_moment(phi, ctx->phisi.p)) || (rc = residual3(ctx, ctx->phisi.p, phi, r3))) {
            status = rc;
            break;
        }
        const double res = std::sqrt(r3[0]) / bnorm;
        int gi = 0;
        if (o->use_dsa) {
            sn_dsa_stats ds{};
            if ((rc = dsa_hp(ctx, phi, ctx->phisi.p, phi, &o->dsa, &ds))) {
                status = rc;
                break;
            }
            gi = ds.cg_iters;
        } else {
            HIPCHK(hipMemcpyAsync(phi, ctx->phisi.p, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        }
        if (stats && stats->res_hist) stats->res_hist[it] = res;
        if (stats && stats->cg_hist) stats->cg_hist[it] = gi;
        ++it;
        if (first < 0) first = res;
        if (!std::isfinite(res) || res > 1e6 * first) {
            status = fail(SN_ERR_DIVERGED, "source iteration diverged at iteration %d (residual %g)", it - 1, res);
            break;
        }
        if (res <= o->tol) {
            status = SN_OK;
            break;
        }
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (status == SN_ERR_NOT_CONVERGED) fail(status, "not converged in %d iterations", o->max_it);
    if (stats) {
        stats->iters = it;
        stats->sweeps = ctx->sweeps;
        stats->fp64_checks = 0;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

// res_part / res_nparts: source-iteration residual partial sums to reduce in
// the solve's first kernel into ctx->res3 and the pinned ctx->hpin->r3 (the
// host's wait for the solve's stop flag, which a later kernel writes, then
// also covers that read-back)
// warm: start the CG from the previous call's solution (within one
// source-iteration call), projected onto the new right-hand side
// next_src (2D source iteration, FP64 form): the final update also writes the
// next sweep's source from phi_out and next_q
int do_dsa(sn_context* ctx, const double* phi_old, const double* phi_si, double* phi_out, const sn_dsa_opts* o,
           sn_dsa_stats* stats, const double* res_part = nullptr, int res_nparts = 0, bool warm = false,
           bool next_src = false, const double* next_q = nullptr) {
    const long n = ctx->nc * ctx->nn;
    if (ctx->nthick == 0) {
        if (res_part)
            HIPCHK(launch_residual_final(res_nparts, res_part, ctx->res3.p, ctx->hpin->r3, ctx->stream));
        if (phi_out != phi_si)
            HIPCHK(hipMemcpyAsync(phi_out, phi_si, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        if (res_part) HIPCHK(hipStreamSynchronize(ctx->stream));
        if (stats) {
            stats->cg_iters = 0;
            stats->cg_relres = 0.0;
            stats->n_thick_cells = 0;
        }
        return 0;
    }
    const DsaGeom& g = ctx->dg;
    size_t e0 = 0, e1 = 0;
    int rc;
    const int bj = o->precond == SN_PRECOND_MG ? 0 : 1;
    const bool fuse_src = next_src && ctx->mesh.dim == 2;
    if (fuse_src && (rc = ensure_skew(ctx, ctx->srcskew64))) return rc;
    auto scatter = [&]() -> int {
        if (fuse_src) {
            HIPCHK(launch_scatter_source_skew2d(ctx->sg.nx, ctx->sg.ny, ctx->slot.p, phi_si, ctx->cx.p,
                                                ctx->sigs.p, next_q, phi_out, ctx->srcskew64.p, ctx->stream));
            ctx->src_tok = true;
            ctx->src_tok_phi = phi_out;
            ctx->src_tok_q = next_q;
        } else {
            HIPCHK(launch_dsa_scatter(ctx->nc, ctx->nn, ctx->slot.p, phi_si, ctx->cx.p, phi_out, ctx->stream));
        }
        return 0;
    };
    if (o->diffusion != SN_DIFFUSION_SIP || o->precond == SN_PRECOND_DIRECT) {
        if (res_part) HIPCHK(launch_residual_final(res_nparts, res_part, ctx->res3.p, ctx->hpin->r3, ctx->stream));
        if (ctx->timing == 1 && (rc = record_event(ctx, &e0))) return rc;
        int its = 0;
        double rel = 0.0;
        if (o->precond == SN_PRECOND_DIRECT) {
            if ((rc = dsa_direct(ctx, phi_old, phi_si, o))) return rc;
            // the host reads the residual scalars the caller asked for
            if (res_part) HIPCHK(hipStreamSynchronize(ctx->stream));
        } else if ((rc = dsa_gmres(ctx, phi_old, phi_si, o, &its, &rel))) {
            return rc;
        }
        if ((rc = scatter())) return rc;
        if (ctx->timing == 1) {
            if ((rc = record_event(ctx, &e1))) return rc;
            ctx->dsa_ev.emplace_back(e0, e1);
        }
        if (stats) {
            stats->cg_iters = its;
            stats->cg_relres = rel;
            stats->n_thick_cells = ctx->nthick;
        }
        return 0;
    }
    if (!bj && !ctx->mg_ready && (rc = mg_setup(ctx))) return rc;
    CgScalars& hs = ctx->hpin->cs;
    auto vcycle = [&]() -> int {
        HIPCHK(launch_mg_vcycle(g, ctx->thick.p, ctx->nbr.p, ctx->sigt.p, ctx->sigs.p, ctx->binv.p, ctx->cr.p,
                                ctx->cz0.p, ctx->cres.p, ctx->cz.p, ctx->mg, ctx->mg_lc, ctx->mg_omega0,
                                ctx->partb.p, ctx->nparts, ctx->scal.p, ctx->stream));
        return 0;
    };
    auto apply = [&](int it) -> int {
        HIPCHK(launch_cg_apply(g, ctx->thick.p, ctx->nbr.p, ctx->sigt.p, ctx->sigs.p, ctx->cz.p, ctx->cp.p,
                               ctx->cp1.p, ctx->cq.p, ctx->parta.p, ctx->partb.p, ctx->nparts, ctx->scal.p, &hs,
                               o->cg_rtol, o->cg_maxit, it, ctx->stream));
        return 0;
    };
    auto update = [&](int it) -> int {
        HIPCHK(launch_cg_update(g, ctx->binv.p, ctx->cx.p, ctx->cr.p, ctx->cz.p, ctx->cp.p, ctx->cp1.p, ctx->cq.p,
                                ctx->parta.p, ctx->partb.p, ctx->nparts, ctx->scal.p, &hs, it, bj, ctx->stream));
        if (!bj) {
            // the next iteration's stop test before its V-cycle, which is then
            // skipped when the solve has converged
            HIPCHK(launch_cg_test(ctx->partb.p, ctx->nparts, ctx->scal.p, &hs, o->cg_rtol, o->cg_maxit, it + 1,
                                  ctx->stream));
            return vcycle();
        }
        return 0;
    };
    // The stop fields of the pinned copy are cleared here, before the solve
    // is enqueued: the host may get here while earlier work is still
    // running, and the previous solve wrote them for the last time when its
    // stop test passed (the host saw that write before returning).
    hs.done = 0;
    hs.breakdown = 0;
    hs.iters = 0;
    if (ctx->timing == 1 && (rc = record_event(ctx, &e0))) return rc;
    if (warm)
        HIPCHK(launch_dsa_warm(g, ctx->thick.p, ctx->nbr.p, ctx->sigt.p, ctx->sigs.p, o->mass_kind, phi_old, phi_si,
                               ctx->cx.p, ctx->cq.p, ctx->parta.p, ctx->nparts, ctx->stream));
    HIPCHK(launch_dsa_rhs(g, ctx->thick.p, ctx->sigt.p, ctx->sigs.p, o->mass_kind, phi_old, phi_si, ctx->binv.p,
                          ctx->cx.p, ctx->cr.p, ctx->cz.p, ctx->cp.p, ctx->partb.p, ctx->nparts, bj, ctx->scal.p,
                          res_part, res_nparts, ctx->res3.p, ctx->hpin->r3, warm ? ctx->cq.p : nullptr,
                          warm ? ctx->parta.p : nullptr, ctx->stream));
    if (!bj && (rc = vcycle())) return rc;
    // Batches of iterations, each ended by the stop test of the next
    // iteration (its apply kernel), then one host wait and a look
    // at the stop flags, which the kernels also write to pinned host memory.
    // The first batch is sized by the last two calls' iteration counts; when
    // a batch does not suffice, the next one starts with the update that the
    // last test left pending.
    int it = 0;  // iteration whose apply kernel runs next
    bool pending = false;
    const bool speculate = phi_out != phi_si;
    // (the larger of the last two counts, which alternate under the warm
    // start: a batch of b iterations ends with the stop test of iteration b,
    // so it covers a solve of up to b iterations; a batch that falls short
    // costs a host round trip and a trickle of late launches, surplus
    // iterations only early-exit kernels)
    int batch = std::max(0, std::min(std::max(ctx->cg_hint, ctx->cg_hint2), o->cg_maxit));
    while (true) {
        if (pending && (rc = update(it - 1))) return rc;
        const int nb = std::min(batch, o->cg_maxit - it);
        for (int b = 0; b < nb; ++b, ++it)
            if ((rc = apply(it)) || (rc = update(it))) return rc;
        if ((rc = apply(it))) return rc;
        ++it;
        pending = true;
        // Without aliasing the final update phi_out = phi_si + P x can be
        // enqueued ahead of the stop decision: the CG kernels never read
        // phi_out (phi_old is read by the right-hand side only), and if the
        // solve goes on the update is enqueued again after the next batch.
        if (speculate && (rc = scatter())) return rc;
        // wait for the stop flag in pinned memory (written as soon as the
        // test passes, ahead of the kernel's end) or for the batch to finish.
        // The event is queried on every turn of the loop: the query also
        // makes the runtime hand the enqueued kernels to the device (with
        // sparser queries the kernels were measured to start late)
        HIPCHK(hipEventRecord(ctx->cg_ev, ctx->stream));
        volatile int* flag = &hs.done;
        while (!*flag) {
            const hipError_t e = hipEventQuery(ctx->cg_ev);
            if (e == hipSuccess) break;
            if (e != hipErrorNotReady) HIPCHK(e);
        }
        if (hs.done || it > o->cg_maxit) break;
        batch = 4;
    }
    if (!speculate && (rc = scatter())) return rc;
    if (ctx->timing == 1) {
        if ((rc = record_event(ctx, &e1))) return rc;
        ctx->dsa_ev.emplace_back(e0, e1);
    }
    ctx->cg_hint2 = ctx->cg_hint;
    ctx->cg_hint = hs.iters;
    if (stats) {
        stats->cg_iters = hs.iters;
        stats->cg_relres = hs.bb > 0 ? std::sqrt(hs.rr / hs.bb) : 0.0;
        stats->n_thick_cells = ctx->nthick;
    }
    if (hs.breakdown) return fail(SN_ERR_CG_BREAKDOWN, "diffusion CG breakdown (p^T D p <= 0)");
    return 0;
}

// Alg. 1, second step, on a vector phi whose thick update started from
// phi_old (NULL: zero): phi_thin += (sum_d w_d L_d^{-1} Sigma_s bar)_thin,
// bar = (phi - phi_old) on the thick cells, zero source and vacuum inflow
int triangular_step(sn_context* ctx, const double* phi_old, double* phi, int transpose, sn_precision prec) {
    const long n = ctx->nc * ctx->nn;
    int rc;
    if ((rc = ctx->phibar.ensure(n)) || (rc = ctx->zeta.ensure(n))) return rc;
    HIPCHK(launch_thick_diff(ctx->nc, ctx->nn, ctx->slot.p, phi, phi_old, ctx->phibar.p, ctx->stream));
    if ((rc = do_sweep_flux(ctx, ctx->phibar.p, nullptr, nullptr, nullptr, transpose, prec, ctx->zeta.p, 0)))
        return rc;
    HIPCHK(launch_thin_add(ctx->nc, ctx->nn, ctx->slot.p, ctx->zeta.p, phi, ctx->stream));
    return 0;
}

// k dot products V_i . w (i < k) into ctx->kdot (device) and out (host)
int dots(sn_context* ctx, int k, const double* V, const double* w, double* out) {
    const long n = ctx->nc * ctx->nn;
    HIPCHK(launch_multi_dot(n, k, V, w, ctx->kpart.p, ctx->kdot.p, ctx->kdot_host, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < k; ++i) out[i] = ctx->kdot_host[i];
    return 0;
}

// Inflow-layout range [f0, f1) of the domain face `face` (2 axis + side)
void face_range(const sn_mesh& m, int face, long* f0, long* f1) {
    const int F = m.dim == 2 ? 2 : 4;
    const long sx = (long)m.ny * m.nz * F, sy = (long)m.nx * m.nz * F, sz = m.dim == 3 ? (long)m.nx * m.ny * F : 0;
    const int ax = face >> 1;
    const long off[4] = {0, sx, sx + sy, sx + sy + sz};
    *f0 = off[ax];
    *f1 = off[ax + 1];
}

// Omega_d . n of the outward normal of `face`
double face_dot(const sn_context* ctx, int face, int d) {
    return ((face & 1) ? 1.0 : -1.0) * ctx->omega[3 * d + (face >> 1)];
}

int residual3(sn_context* ctx, const double* a, const double* b, double out[3]) {
    const long n = ctx->nc * ctx->nn;
    HIPCHK(launch_residual(n, a, b, ctx->rpart.p, ctx->nrpart, ctx->res3.p, ctx->stream));
    HIPCHK(hipMemcpyAsync(out, ctx->res3.p, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return 0;
}

}  // namespace

extern "C" {

const char* sn_last_error(void) { return g_err.c_str(); }

long sn_inflow_size(const sn_mesh* mesh) {
    if (check_mesh(mesh)) return -1;
    return inflow_size(mesh);
}

int sn_thick_count(const sn_context* ctx) { return ctx ? ctx->nthick : -1; }

void sn_context_destroy(sn_context* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->evpool) (void)hipEventDestroy(e);
    if (ctx->res_ev) (void)hipEventDestroy(ctx->res_ev);
    if (ctx->cg_ev) (void)hipEventDestroy(ctx->cg_ev);
    for (int k = 1; k < MAX_SPLIT; ++k) {
        if (ctx->split.st[k]) {
            (void)hipStreamSynchronize(ctx->split.st[k]);
            (void)hipStreamDestroy(ctx->split.st[k]);
        }
        if (ctx->split.join[k]) (void)hipEventDestroy(ctx->split.join[k]);
    }
    if (ctx->split.fork) (void)hipEventDestroy(ctx->split.fork);
    if (ctx->hpin) (void)hipHostFree(ctx->hpin);
    ctx->fpart.release();
    ctx->evpool.clear();
    ctx->dirs.release();
    ctx->w.release();
    ctx->wn.release();
    ctx->sigt.release();
    ctx->sigs.release();
    ctx->sigt32.release();
    ctx->flags.release();
    ctx->blocksums.release();
    ctx->total.release();
    ctx->slot.release();
    ctx->thick.release();
    ctx->binv.release();
    ctx->cx.release();
    ctx->cr.release();
    ctx->cz.release();
    ctx->cp.release();
    ctx->cp1.release();
    ctx->nbr.release();
    ctx->cq.release();
    ctx->parta.release();
    ctx->partb.release();
    ctx->scal.release();
    ctx->tiles.release();
    ctx->groups.release();
    ctx->xf64.release();
    ctx->yf64.release();
    ctx->zf64.release();
    ctx->src64.release();
    ctx->sink64.release();
    ctx->sink32.release();
    ctx->xf32.release();
    ctx->yf32.release();
    ctx->zf32.release();
    ctx->src32.release();
    ctx->sigskew64.release();
    ctx->sigskew32.release();
    ctx->srcskew64.release();
    ctx->srcskew32.release();
    ctx->psi64.release();
    ctx->psi32.release();
    ctx->phisi.release();
    ctx->phitmp.release();
    ctx->phiprev.release();
    ctx->rpart.release();
    ctx->res3.release();
    ctx->phioct.release();
    ctx->mg_coef.release();
    ctx->mg_pw.release();
    ctx->mg_b.release();
    ctx->mg_x.release();
    ctx->mg_y.release();
    ctx->mg_r.release();
    ctx->mg_ainv.release();
    ctx->cz0.release();
    ctx->cres.release();
    ctx->mg_nbr.release();
    ctx->mg_chl.release();
    ctx->mg_par.release();
    ctx->mg_vnodes.release();
    ctx->mg_nodev.release();
    ctx->order2d_parts.release();
    ctx->face_out.release();
    ctx->part_w.release();
    ctx->part_wn.release();
    ctx->psi_a.release();
    ctx->psi_b.release();
    ctx->phiold.release();
    ctx->phibar.release();
    ctx->zeta.release();
    ctx->kv.release();
    ctx->kz.release();
    ctx->kw.release();
    ctx->kb.release();
    ctx->kzero.release();
    ctx->kdot.release();
    ctx->kpart.release();
    ctx->binvf.release();
    ctx->gv.release();
    ctx->gdot.release();
    ctx->gpart.release();
    ctx->gb.release();
    ctx->gu.release();
    ctx->gz.release();
    ctx->gbad.release();
    ctx->band.release();
    ctx->bpiv.release();
    ctx->hblk.release();
    ctx->hcol.release();
    if (ctx->kdot_host) (void)hipHostFree(ctx->kdot_host);
    if (ctx->gdot_host) (void)hipHostFree(ctx->gdot_host);
    delete ctx;
}

int sn_context_create(const sn_mesh* mesh, const sn_quad* quad, const double* sigma_t, const double* sigma_s,
                      double eta, void* stream, sn_context** out) {
    g_err.clear();
    if (!out) return fail(SN_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int rc = check_mesh(mesh);
    if (rc) return rc;
    if (!quad || quad->ndirs <= 0 || !quad->omega || !quad->w)
        return fail(SN_ERR_INVALID, "quadrature missing or empty");
    if (!sigma_t || !sigma_s) return fail(SN_ERR_INVALID, "sigma_t / sigma_s is NULL");
    if (std::isnan(eta)) return fail(SN_ERR_INVALID, "eta is NaN");
    const int dim = mesh->dim;
    double wsum = 0.0;
    for (int d = 0; d < quad->ndirs; ++d) {
        const double* o = quad->omega + 3 * d;
        if (!(quad->w[d] > 0) || !std::isfinite(quad->w[d])) return fail(SN_ERR_INVALID, "weight %d not positive", d);
        double nrm = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
        if (!(std::fabs(nrm - 1.0) < 1e-10)) return fail(SN_ERR_INVALID, "direction %d is not a unit vector", d);
        for (int a = 0; a < dim; ++a)
            if (o[a] == 0.0) return fail(SN_ERR_UNSUPPORTED, "direction %d has a zero component", d);
        wsum += quad->w[d];
    }
    if (std::fabs(wsum - 4.0 * kPi) > 1e-12 * 4.0 * kPi) return fail(SN_ERR_INVALID, "weights sum to %.17g, not 4 pi", wsum);

    std::unique_ptr<sn_context> c(new sn_context());
    // owned by unique_ptr until success; sn_context_destroy frees device memory
    struct Guard {
        std::unique_ptr<sn_context>& c;
        ~Guard() {
            if (c) {
                sn_context_destroy(c.release());
            }
        }
    } guard{c};
    c->mesh = *mesh;
    c->order = mesh->order >= 2 ? mesh->order : 1;
    c->nn = c->order >= 2 ? (c->order + 1) * (c->order + 1) : (dim == 2 ? 4 : 8);
    if (c->order >= 2 && !hp_tables(c->order, &c->hp))
        return fail(SN_ERR_UNSUPPORTED, "order %d: eigenbasis of the 1D upwind operator failed its check", c->order);
    c->nc = (long)mesh->nx * mesh->ny * mesh->nz;
    c->ndirs = quad->ndirs;
    c->nbf = inflow_size(mesh);
    c->eta = eta;
    c->stream = (hipStream_t)stream;
    const double h[3] = {mesh->hx, mesh->hy, dim == 3 ? mesh->hz : 1.0};
    c->hw.assign(quad->w, quad->w + quad->ndirs);
    c->omega.assign(quad->omega, quad->omega + 3 * quad->ndirs);
    c->hdirs.resize(quad->ndirs);
    for (int d = 0; d < quad->ndirs; ++d) {
        const double* o = quad->omega + 3 * d;
        DirInfo& di = c->hdirs[d];
        di.ax = std::fabs(o[0]) / h[0];
        di.ay = std::fabs(o[1]) / h[1];
        di.az = dim == 3 ? std::fabs(o[2]) / h[2] : 0.0;
        di.w = quad->w[d];
        di.rx = o[0] < 0;
        di.ry = o[1] < 0;
        di.rz = dim == 3 ? (o[2] < 0) : 0;
        di.pad = 0;
    }
    // validate cross sections on the host
    const long nc = c->nc;
    std::vector<double> st(nc), ss(nc);
    HIPCHK(hipMemcpy(st.data(), sigma_t, nc * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ss.data(), sigma_s, nc * sizeof(double), hipMemcpyDeviceToHost));
    for (long i = 0; i < nc; ++i) {
        if (!std::isfinite(st[i]) || !std::isfinite(ss[i]) || st[i] < 0 || ss[i] < 0)
            return fail(SN_ERR_INVALID, "cell %ld: cross sections must be finite and non-negative", i);
        if (ss[i] > st[i]) return fail(SN_ERR_INVALID, "cell %ld: sigma_s > sigma_t", i);
    }
    std::vector<float> st32(st.begin(), st.end());
    if ((rc = c->dirs.ensure(c->ndirs)) || (rc = c->w.ensure(c->ndirs)) || (rc = c->sigt.ensure(nc)) ||
        (rc = c->sigs.ensure(nc)) || (rc = c->sigt32.ensure(nc)))
        return rc;
    HIPCHK(hipMemcpy(c->dirs.p, c->hdirs.data(), c->ndirs * sizeof(DirInfo), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->w.p, c->hw.data(), c->ndirs * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->sigt.p, st.data(), nc * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->sigs.p, ss.data(), nc * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->sigt32.p, st32.data(), nc * sizeof(float), hipMemcpyHostToDevice));

    // sweep geometry
    SweepGeom& g = c->sg;
    g.dim = dim;
    g.nx = mesh->nx;
    g.ny = mesh->ny;
    g.nz = mesh->nz;
    g.ndirs = c->ndirs;
    g.nbf = c->nbf;
    if (dim == 2) {
        g.nchunk = (mesh->ny + ROWS2D - 1) / ROWS2D;
        g.xstride = (long)mesh->ny * 2;
        g.ystride = (long)g.nchunk * mesh->nx * 2;
        g.zstride = 0;
        g.TX = 0;
        g.nTx = g.nTy = g.nTz = 0;
        g.nplanes = 0;
        c->plane_off.assign(1, 0);
        if ((rc = c->tiles.ensure(1))) return rc;
        // Workgroup order: workgroups are dealt to the eight XCDs round robin
        // (workgroup i on XCD i % 8) and every XCD has its own L2, so the
        // directions of one quadrant, which read the same input arrays, go
        // to XCDs 2q and 2q + 1; leftovers fill the remaining positions.
        {
            std::vector<std::vector<int>> cls(4);
            for (int d = 0; d < c->ndirs; ++d) {
                const DirInfo& di = c->hdirs[d];
                cls[di.rx | (di.ry << 1)].push_back(d);
            }
            std::vector<std::vector<int>> xq(8);
            for (int q = 0; q < 4; ++q)
                for (size_t e = 0; e < cls[q].size(); ++e) xq[2 * q + (e & 1)].push_back(cls[q][e]);
            std::vector<int> order, rest;
            std::vector<size_t> pos(8, 0);
            for (int i = 0; i < c->ndirs; ++i) {
                auto& v = xq[i % 8];
                if (pos[i % 8] < v.size()) order.push_back(v[pos[i % 8]++]);
                else order.push_back(-1);
            }
            for (int x = 0; x < 8; ++x)
                for (size_t e = pos[x]; e < xq[x].size(); ++e) rest.push_back(xq[x][e]);
            size_t ri = 0;
            for (auto& o : order)
                if (o < 0) o = rest[ri++];
            if ((rc = c->groups.ensure(order.size()))) return rc;
            HIPCHK(hipMemcpy(c->groups.p, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice));
            g.groups = c->groups.p;
        }
        g.nclasses = g.groups_per_class = 0;
        // sigma_t in the diagonal-major layout of the 2D sweep
        const size_t ns = (size_t)skew2d_elems(mesh->nx, mesh->ny, 1);
        if ((rc = c->sigskew64.ensure(ns)) || (rc = c->sigskew32.ensure(ns))) return rc;
        HIPCHK(hipMemsetAsync(c->sigskew64.p, 0, ns * sizeof(double), c->stream));
        HIPCHK(hipMemsetAsync(c->sigskew32.p, 0, ns * sizeof(float), c->stream));
        HIPCHK(launch_skew2d<double>(mesh->nx, mesh->ny, 1, c->sigt.p, c->sigskew64.p, c->stream));
        HIPCHK(launch_skew2d<float>(mesh->nx, mesh->ny, 1, c->sigt32.p, c->sigskew32.p, c->stream));
    } else {
        // Tile length along x: at most 32, the length of the sweep kernels'
        // LDS tile.  32 when a tile-plane launch then holds on average at
        // least one workgroup per CU; 16 for smaller meshes, which would
        // otherwise leave most CUs idle (measured at 64^3, S8: time to 1e-8
        // FP64 0.079 -> 0.071 s, FP32 form 0.071 -> 0.055 s).  SN_SWEEP_TX in
        // the environment overrides the choice.
        int tx = 32;
        {
            bool used[8] = {};
            int ncls = 0;
            for (int d = 0; d < c->ndirs; ++d) {
                const DirInfo& di = c->hdirs[d];
                const int m = di.rx | (di.ry << 1) | (di.rz << 2);
                if (!used[m]) ++ncls;
                used[m] = true;
            }
            int dev = 0, ncu = 0;
            HIPCHK(hipGetDevice(&dev));
            HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
            const long ntx = (mesh->nx + 31) / 32, nty = (mesh->ny + 3) / 4, ntz = (mesh->nz + 3) / 4;
            const long per_plane = ncls * ntx * nty * ntz / (ntx + nty + ntz - 2);
            if (per_plane < ncu) tx = 16;
        }
        if (const char* e = std::getenv("SN_SWEEP_TX")) tx = std::max(1, std::atoi(e));
        g.TX = std::min(std::min(tx, 32), mesh->nx);
        g.nTx = (mesh->nx + g.TX - 1) / g.TX;
        g.nTy = (mesh->ny + 3) / 4;
        g.nTz = (mesh->nz + 3) / 4;
        if (g.nTx > 1023 || g.nTy > 1023 || g.nTz > 1023)
            return fail(SN_ERR_UNSUPPORTED, "more than 1023 sweep tiles along an axis");
        g.nplanes = g.nTx + g.nTy + g.nTz - 2;
        g.nchunk = 0;
        g.xstride = (long)g.nTx * mesh->nz * mesh->ny * 4;  // y and z: tile slots (yz_face_elems)
        g.ystride = g.zstride = 0;
        std::vector<int> tl;
        c->plane_off.assign(1, 0);
        for (int p = 0; p < g.nplanes; ++p) {
            for (int I = 0; I < g.nTx; ++I)
                for (int J = 0; J < g.nTy; ++J) {
                    int K = p - I - J;
                    if (K >= 0 && K < g.nTz) tl.push_back(I | (J << 10) | (K << 20));
                }
            c->plane_off.push_back((int)tl.size());
        }
        if ((rc = c->tiles.ensure(tl.size()))) return rc;
        HIPCHK(hipMemcpy(c->tiles.p, tl.data(), tl.size() * sizeof(int), hipMemcpyHostToDevice));
        // direction groups: directions with the same reflection (octant), in
        // index order, four per group
        std::vector<std::vector<int>> cls(8);
        for (int d = 0; d < c->ndirs; ++d) {
            const DirInfo& di = c->hdirs[d];
            cls[di.rx | (di.ry << 1) | (di.rz << 2)].push_back(d);
        }
        int ncls = 0, gpc = 1;
        for (auto& v : cls)
            if (!v.empty()) {
                ++ncls;
                gpc = std::max(gpc, (int)((v.size() + 3) / 4));
            }
        if (gpc > 6) return fail(SN_ERR_UNSUPPORTED, "more than 24 directions per octant");
        // per group: four direction ids (-1 = empty), the first id if the
        // valid ones are consecutive (else -1), the number of valid ids
        std::vector<int> gr((size_t)ncls * gpc * 6, -1);
        int ci = 0;
        for (auto& v : cls) {
            if (v.empty()) continue;
            for (size_t e = 0; e < v.size(); ++e) gr[((size_t)ci * gpc + e / 4) * 6 + e % 4] = v[e];
            for (int gidx = 0; gidx < gpc; ++gidx) {
                int* gg = &gr[((size_t)ci * gpc + gidx) * 6];
                int nv = 0;
                bool consec = true;
                for (int k = 0; k < 4; ++k)
                    if (gg[k] >= 0) {
                        if (gg[k] != gg[0] + k) consec = false;
                        ++nv;
                    }
                gg[5] = nv;
                gg[4] = (nv > 0 && consec) ? gg[0] : -1;
            }
            ++ci;
        }
        if ((rc = c->groups.ensure(gr.size()))) return rc;
        HIPCHK(hipMemcpy(c->groups.p, gr.data(), gr.size() * sizeof(int), hipMemcpyHostToDevice));
        g.nclasses = ncls;
        g.groups_per_class = gpc;
        g.groups = c->groups.p;
        // the psi sweep without branches around memory operations needs each
        // direction group consecutive (one psi resource per wave) and byte
        // offsets below 2^31 from a tile's lowest cell (FP64 bounds, which
        // cover FP32); SN_SWEEP_BUF=0 selects the other variant
        {
            bool consec = true;
            for (size_t e = 0; e + 5 < gr.size(); e += 6)
                if (gr[e + 5] > 0 && gr[e + 4] < 0) consec = false;
            const double lim = 2147483648.0 - 4096.0;
            const double psi_span = ((3.0 * mesh->ny + 3.0) * mesh->nx + g.TX) * c->ndirs * 64.0 + 4096.0;
            const char* e = std::getenv("SN_SWEEP_BUF");
            g.buf = consec && psi_span < lim && !(e && std::atoi(e) == 0);
        }
    }

    // direction parts: 3D the reflection classes (local index 4 group + slot),
    // 2D the quadrants (local index = position in the quadrant's list)
    {
        if (dim == 3) {
            const int gpc = g.groups_per_class;
            std::vector<int> gr((size_t)g.nclasses * gpc * 6);
            HIPCHK(hipMemcpy(gr.data(), g.groups, gr.size() * sizeof(int), hipMemcpyDeviceToHost));
            // the stride is the largest valid local index + 1 (S12: 21 of the
            // 24 slots of six groups; the empty slots of the last group are
            // never written, so they need no room)
            for (int ci = 0; ci < g.nclasses; ++ci) {
                std::vector<int> ids(4 * gpc, -1);
                for (int gi = 0; gi < gpc; ++gi)
                    for (int k = 0; k < 4; ++k) {
                        ids[4 * gi + k] = gr[((size_t)ci * gpc + gi) * 6 + k];
                        if (ids[4 * gi + k] >= 0) c->part_stride = std::max(c->part_stride, 4 * gi + k + 1);
                    }
                c->parts.push_back(SweepPart{ci, 1, 0, 1, nullptr});
                c->part_dirs.push_back(ids);
            }
            for (auto& pp : c->parts) pp.pstride = c->part_stride;
            for (auto& ids : c->part_dirs) ids.resize(c->part_stride);
        } else {
            std::vector<std::vector<int>> qd(4);
            for (int d = 0; d < c->ndirs; ++d) qd[c->hdirs[d].rx | (c->hdirs[d].ry << 1)].push_back(d);
            std::vector<int> flat;
            for (auto& v : qd) {
                c->part_stride = std::max(c->part_stride, (int)v.size());
                flat.insert(flat.end(), v.begin(), v.end());
            }
            if ((rc = c->order2d_parts.ensure(std::max<size_t>(flat.size(), 1)))) return rc;
            HIPCHK(hipMemcpy(c->order2d_parts.p, flat.data(), flat.size() * sizeof(int), hipMemcpyHostToDevice));
            size_t off = 0;
            for (auto& v : qd) {
                if (v.empty()) continue;
                c->parts.push_back(SweepPart{0, (int)v.size(), 0, 1, c->order2d_parts.p + off});
                std::vector<int> ids(v);
                c->part_dirs.push_back(ids);
                off += v.size();
            }
            for (auto& pp : c->parts) pp.pstride = c->part_stride;
            for (auto& ids : c->part_dirs) ids.resize(c->part_stride, -1);
        }
        std::vector<double> pw((size_t)c->parts.size() * c->part_stride, 0.0);
        for (size_t pi = 0; pi < c->parts.size(); ++pi)
            for (int l = 0; l < c->part_stride; ++l) {
                const int d = c->part_dirs[pi][l];
                if (d >= 0) pw[pi * c->part_stride + l] = quad->w[d];
            }
        if ((rc = c->part_w.ensure(pw.size())) || (rc = c->part_wn.ensure(pw.size())) ||
            (rc = c->face_out.ensure(c->ndirs)))
            return rc;
        HIPCHK(hipMemcpy(c->part_w.p, pw.data(), pw.size() * sizeof(double), hipMemcpyHostToDevice));
    }

    // thick set
    const int nblk = (int)((nc + 255) / 256);
    if ((rc = c->flags.ensure(nc)) || (rc = c->blocksums.ensure(nblk)) || (rc = c->total.ensure(1)) ||
        (rc = c->slot.ensure(nc)) || (rc = c->thick.ensure(nc)))
        return rc;
    HIPCHK(launch_thick_flags(nc, c->sigs.p, eta, c->flags.p, c->blocksums.p, nblk, c->stream));
    HIPCHK(launch_thick_scan(nblk, c->blocksums.p, c->total.p, c->stream));
    HIPCHK(launch_thick_scatter(nc, c->flags.p, c->blocksums.p, c->slot.p, c->thick.p, c->stream));
    int nthick = 0;
    HIPCHK(hipMemcpyAsync(&nthick, c->total.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->nthick = nthick;
    DsaGeom& dg = c->dg;
    dg.dim = dim;
    dg.nx = mesh->nx;
    dg.ny = mesh->ny;
    dg.nz = mesh->nz;
    dg.nn = c->nn;
    for (int a = 0; a < 3; ++a) {
        dg.h[a] = h[a];
        double s = 0.0;
        for (int d = 0; d < c->ndirs; ++d) s += quad->w[d] * std::fabs(quad->omega[3 * d + a]);
        dg.kappa0[a] = s / (8.0 * kPi);
    }
    dg.nthick = nthick;
    const long nf = (long)nthick * c->nn;
    c->nparts = std::max(1, std::min((nthick + 255) / 256, 1024));
    if ((rc = c->binv.ensure((size_t)std::max(nthick, 1) * bj_entries_of(c->nn))) || (rc = c->cx.ensure(nf)) ||
        (rc = c->cr.ensure(nf)) || (rc = c->cz.ensure(nf)) || (rc = c->cp.ensure(nf)) || (rc = c->cp1.ensure(nf)) ||
        (rc = c->cq.ensure(nf)) || (rc = c->nbr.ensure((size_t)std::max(nthick, 1) * 2 * dim)) ||
        (rc = c->parta.ensure(3 * c->nparts)) || (rc = c->partb.ensure(3 * c->nparts)) ||
        (rc = c->scal.ensure(1)))
        return rc;
    c->dg4 = dg;
    c->dg4.nn = dim == 2 ? 4 : 8;
    if (c->order == 1)
        HIPCHK(launch_block_jacobi(dg, c->thick.p, c->slot.p, c->sigt.p, c->sigs.p, c->binv.p, c->stream));
    HIPCHK(launch_neighbour_table(c->dg4, c->thick.p, c->slot.p, c->nbr.p, c->stream));
    c->nrpart = (int)std::max<long>(1, std::min<long>((nc * c->nn + 255) / 256, 1024));
    if ((rc = c->rpart.ensure(3 * c->nrpart)) || (rc = c->res3.ensure(3))) return rc;
    HIPCHK(hipHostMalloc((void**)&c->hpin, sizeof(sn_context::HostScalars), hipHostMallocDefault));
    // once per device (cached across contexts): the address of the fixed
    // scratch of sn_response_noalloc; a failed lookup disables only that entry
    c->noalloc_err = noalloc_scratch(&c->noalloc);
    HIPCHK(hipEventCreateWithFlags(&c->res_ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->cg_ev, hipEventDisableTiming));
    // 3D: the reflection classes of a full sweep split over up to four streams
    // of default priority (SN_SWEEP_STREAMS, 1 = the caller's stream only)
    c->split.n = 1;
    c->split.st[0] = c->stream;
    if (dim == 3 && c->sg.nclasses > 1) {
        int ns = SPLIT_DEFAULT;
        if (const char* e = std::getenv("SN_SWEEP_STREAMS")) ns = std::atoi(e);
        ns = std::max(1, std::min(std::min(ns, MAX_SPLIT), c->sg.nclasses));
        if (ns > 1) HIPCHK(hipEventCreateWithFlags(&c->split.fork, hipEventDisableTiming));
        for (int k = 1; k < ns; ++k) {
            HIPCHK(hipStreamCreateWithFlags(&c->split.st[k], hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&c->split.join[k], hipEventDisableTiming));
        }
        c->split.n = ns;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    *out = c.release();
    return SN_OK;
}

int sn_set_kernel_timing(sn_context* ctx, int enable) {
    g_err.clear();
    if (!ctx) return fail(SN_ERR_INVALID, "context is NULL");
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (enable < 0 || enable > 2) return fail(SN_ERR_INVALID, "kernel timing mode %d (0, 1 or 2)", enable);
    ctx->timing = enable;
    ctx->evused = 0;
    ctx->sweep_ev.clear();
    ctx->dsa_ev.clear();
    return 0;
}

int sn_kernel_timing(sn_context* ctx, double* sweep_ms, int* sweep_count, double* dsa_ms, int* dsa_count) {
    g_err.clear();
    if (!ctx) return fail(SN_ERR_INVALID, "context is NULL");
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double sw = 0.0, ds = 0.0;
    for (auto& pr : ctx->sweep_ev) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->evpool[pr.first], ctx->evpool[pr.second]));
        sw += ms;
    }
    for (auto& pr : ctx->dsa_ev) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->evpool[pr.first], ctx->evpool[pr.second]));
        ds += ms;
    }
    if (sweep_ms) *sweep_ms = sw;
    if (sweep_count) *sweep_count = (int)ctx->sweep_ev.size();
    if (dsa_ms) *dsa_ms = ds;
    if (dsa_count) *dsa_count = (int)ctx->dsa_ev.size();
    ctx->evused = 0;
    ctx->sweep_ev.clear();
    ctx->dsa_ev.clear();
    return 0;
}

int sn_sweep(sn_context* ctx, const double* phi, const double* q, const double* inflow, int transpose,
             sn_precision prec, void* psi) {
    g_err.clear();
    if (!ctx || !psi) return fail(SN_ERR_INVALID, "context or psi is NULL");
    if (prec != SN_FP64 && prec != SN_FP32) return fail(SN_ERR_INVALID, "unknown precision %d", (int)prec);
    if (ctx->order >= 2) {
        if (transpose || prec != SN_FP64)
            return fail(SN_ERR_UNSUPPORTED, "order %d: forward FP64 sweeps only", ctx->order);
        HIPCHK(launch_sweep_hp(ctx->hp, ctx->mesh.nx, ctx->mesh.ny, ctx->ndirs, ctx->nbf, ctx->dirs.p, ctx->sigt.p,
                               ctx->sigs.p, phi, q, inflow, (double*)psi, ctx->stream));
        ++ctx->sweeps;
        return 0;
    }
    return do_sweep(ctx, phi, nullptr, q, inflow, transpose ? 1 : 0, prec, psi);
}

int sn_scalar_flux(sn_context* ctx, const void* psi, sn_precision prec, double* phi_out) {
    g_err.clear();
    if (!ctx || !psi || !phi_out) return fail(SN_ERR_INVALID, "NULL argument");
    if (prec != SN_FP64 && prec != SN_FP32) return fail(SN_ERR_INVALID, "unknown precision %d", (int)prec);
    if (ctx->order >= 2) {
        if (prec != SN_FP64) return fail(SN_ERR_UNSUPPORTED, "order %d: FP64 psi only", ctx->order);
        HIPCHK(launch_moment_hp(ctx->nc, ctx->ndirs, ctx->nn, ctx->w.p, (const double*)psi, phi_out, ctx->stream));
        return 0;
    }
    return do_moment(ctx, psi, prec, phi_out);
}

int sn_dsa_thick_correct(sn_context* ctx, const double* phi_old, const double* phi_si, double* phi_out,
                         const sn_dsa_opts* opts, sn_dsa_stats* stats) {
    g_err.clear();
    if (!ctx || !phi_old || !phi_si || !phi_out || !opts) return fail(SN_ERR_INVALID, "NULL argument");
    if (bad_dsa_opts(*opts)) return fail(SN_ERR_INVALID, "bad DSA options");
    if (ctx->order >= 2) return dsa_hp(ctx, phi_old, phi_si, phi_out, opts, stats);
    return do_dsa(ctx, phi_old, phi_si, phi_out, opts, stats);
}

int sn_source_iterate(sn_context* ctx, const double* q, const double* inflow, double* phi, const sn_iter_opts* o,
                      sn_iter_stats* stats) {
    g_err.clear();
    auto t0 = std::chrono::steady_clock::now();
    if (!ctx || !phi || !o) return fail(SN_ERR_INVALID, "NULL argument");
    if (!(o->tol >= 0) || o->max_it < 1) return fail(SN_ERR_INVALID, "bad tolerance or iteration limit");
    if (o->phi_ckpt && o->ckpt_cap < 1) return fail(SN_ERR_INVALID, "ckpt_cap must be >= 1 with phi_ckpt");
    if (o->prec != SN_FP64 && o->prec != SN_FP32) return fail(SN_ERR_INVALID, "unknown precision");
    if (o->use_dsa && bad_dsa_opts(o->dsa)) return fail(SN_ERR_INVALID, "bad DSA options");
    if (o->fp32_refine != 0 && o->fp32_refine != 1) return fail(SN_ERR_INVALID, "fp32_refine must be 0 or 1");
    if (o->dsa_form != SN_DSA_DIAGONAL && o->dsa_form != SN_DSA_TRIANGULAR)
        return fail(SN_ERR_INVALID, "unknown DSA form %d", o->dsa_form);
    if (ctx->order >= 2) return si_hp(ctx, q, inflow, phi, o, stats, t0);
    // the inflow array is fixed for the whole call: face buffers are filled
    // once per precision (and transpose flag) and reused by later sweeps
    struct FaceReuse {
        sn_context* c;
        explicit FaceReuse(sn_context* c_) : c(c_) {
            c->fkey[0].valid = c->fkey[1].valid = false;
            c->face_reuse = true;
            c->src_tok = false;
        }
        ~FaceReuse() {
            c->face_reuse = false;
            c->src_tok = false;  // the caller may change phi before the next call
        }
    } face_reuse(ctx);
    const long n = ctx->nc * ctx->nn;
    int rc;
    if ((rc = ctx->phisi.ensure(n)) || (rc = ctx->phitmp.ensure(n)) || (rc = ctx->phiprev.ensure(n))) return rc;
    const int tr = o->transpose ? 1 : 0;
    // FP32 form.  Plain (fp32_refine = 0): every sweep is FP32 on the full
    // source; moment, residual and DSA stay FP64.  Refined (fp32_refine = 1):
    // FP32 sweeps act on the iterate increment (defect correction): after the
    // first iteration the sweep source is sigma_s (phi_i - phi_{i-1}) / 4pi
    // and its moment is added to the FP64 accumulator phi_SI, so the FP32
    // rounding error scales with the increment instead of with phi.
    const bool incr = o->prec == SN_FP32 && o->fp32_refine;
    // triangular heterogeneous DSA (Alg. 1): after the thick update, the thick
    // part of the preconditioned residual is swept once more (zero source,
    // vacuum) and the result is added to the thin DOFs
    const bool tri = o->use_dsa && o->dsa_form == SN_DSA_TRIANGULAR && ctx->nthick > 0;
    if (tri && ((rc = ctx->phiold.ensure(n)) || (rc = ctx->phibar.ensure(n)) || (rc = ctx->zeta.ensure(n))))
        return rc;
    ctx->sweeps = 0;
    if (stats) stats->fp64_checks = 0;
    double bnorm = 1.0, first = -1.0;
    int it = 0;
    int status = SN_ERR_NOT_CONVERGED;
    bool verified = false;   // FP32 form: phi_SI last recomputed by an FP64 sweep
    bool refreshed = false;  // FP32 form: the 1e-4 refresh sweep has been done
    const double refresh_at = 1e-4;
    int dsa_done = 0;  // DSA solves of this call
    for (; it < o->max_it; ++it) {
        // After the first iteration the last kernel of the sweep writes the
        // residual's partial sums, the DSA solve's first kernel reduces them
        // into pinned host memory, and the value is read after the solve,
        // which does not depend on it (one host wait per iteration).
        const bool defer = it > 0;
        int res_n = 0;
        const double* res_ref = defer ? phi : nullptr;
        if (!incr || it == 0) {
            if ((rc = do_sweep_flux(ctx, phi, nullptr, q, inflow, tr, o->prec, ctx->phisi.p, 0, res_ref, &res_n)))
                return rc;
        } else {
            if ((rc = do_sweep_flux(ctx, phi, ctx->phiprev.p, nullptr, nullptr, tr, o->prec, ctx->phisi.p, 1,
                                    res_ref, &res_n)))
                return rc;
        }
        verified = false;
        double r3[3];
        if (!defer && (rc = residual3(ctx, ctx->phisi.p, phi, r3))) return rc;
        if (it == 0) {
            if (r3[2] == 0.0) {
                bnorm = std::sqrt(r3[1]);
            } else {
                // ||b||: the transport update of q alone, from phi = 0
                if ((rc = do_sweep_flux(ctx, nullptr, nullptr, q, inflow, tr, o->prec, ctx->phitmp.p, 0))) return rc;
                double b3[3];
                if ((rc = residual3(ctx, ctx->phitmp.p, ctx->phitmp.p, b3))) return rc;
                bnorm = std::sqrt(b3[1]);
            }
            if (bnorm == 0.0) bnorm = 1.0;
        }
        // FP64 sweeps in the FP32 form: once when the residual first drops
        // below 1e-4 (this discards the FP32 rounding accumulated while the
        // increments were large) and whenever it meets tol (the form may only
        // stop on an exact residual).  phi_SI is recomputed from the iterate
        // with one FP64 sweep and the increments continue from it.
        auto wants_fp64 = [&](const double* r) {
            const double res32 = std::sqrt(r[0]) / bnorm;
            return res32 <= o->tol || (!refreshed && res32 <= refresh_at && o->tol < refresh_at);
        };
        auto refresh = [&](const double* iterate) -> int {
            refreshed = true;
            int e;
            if ((e = do_sweep_flux(ctx, iterate, nullptr, q, inflow, tr, SN_FP64, ctx->phisi.p, 0))) return e;
            if ((e = residual3(ctx, ctx->phisi.p, iterate, r3))) return e;
            verified = true;
            if (stats) stats->fp64_checks += 1;
            return 0;
        };
        if (incr) {
            if (!defer && wants_fp64(r3) && (rc = refresh(phi))) return rc;
            // the iterate, for the next increment (and for a redo below)
            HIPCHK(hipMemcpyAsync(ctx->phiprev.p, phi, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        }
        // phi <- phi_SI, corrected by the DSA solve from the iterate phi_old
        int cgi = 0;
        // (the CG warm-starts from the previous iteration's correction)
        auto update = [&](const double* phi_old, bool with_res) -> int {
            if (o->use_dsa) {
                const double* pold = phi_old;
                if (tri && phi_old == phi) {  // the thick update overwrites phi in place
                    HIPCHK(hipMemcpyAsync(ctx->phiold.p, phi, n * sizeof(double), hipMemcpyDeviceToDevice,
                                          ctx->stream));
                    pold = ctx->phiold.p;
                }
                sn_dsa_stats ds{};
                // (2D FP64 diagonal form: the final update also writes the next sweep's source)
                const int e = do_dsa(ctx, pold, ctx->phisi.p, phi, &o->dsa, &ds,
                                     with_res ? ctx->fpart.p : nullptr, res_n, dsa_done > 0,
                                     o->prec == SN_FP64 && !tri, q);
                ++dsa_done;
                cgi = ds.cg_iters;
                if (e) return e;
                return tri ? triangular_step(ctx, pold, phi, tr, o->prec) : 0;
            }
            if (with_res) {
                HIPCHK(launch_residual_final(res_n, ctx->fpart.p, ctx->res3.p, ctx->hpin->r3, ctx->stream));
                HIPCHK(hipEventRecord(ctx->res_ev, ctx->stream));
            }
            HIPCHK(hipMemcpyAsync(phi, ctx->phisi.p, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
            if (with_res) HIPCHK(hipEventSynchronize(ctx->res_ev));
            return 0;
        };
        if ((rc = update(phi, defer))) {
            status = rc;
            ++it;
            break;
        }
        if (defer) {
            for (int k = 0; k < 3; ++k) r3[k] = ctx->hpin->r3[k];
            if (incr && wants_fp64(r3)) {
                // the FP32 residual, known only now, asks for an FP64 sweep:
                // this iteration is redone from its iterate, kept in phiprev
                if ((rc = refresh(ctx->phiprev.p))) return rc;
                if ((rc = update(ctx->phiprev.p, false))) {
                    status = rc;
                    ++it;
                    break;
                }
            }
        }
        const double res = std::sqrt(r3[0]) / bnorm;
        if (stats && stats->res_hist) stats->res_hist[it] = res;
        if (first < 0) first = res;
        if (stats && stats->cg_hist) stats->cg_hist[it] = cgi;
        if (o->phi_ckpt)
            HIPCHK(hipMemcpyAsync(o->phi_ckpt + (size_t)(it % o->ckpt_cap) * n, phi, n * sizeof(double),
                                  hipMemcpyDeviceToDevice,
                                  ctx->stream));
        if (!std::isfinite(res) || res > 1e6 * first) {
            status = fail(SN_ERR_DIVERGED, "source iteration diverged at iteration %d (residual %g)", it, res);
            ++it;
            break;
        }
        if (res <= o->tol) {
            status = SN_OK;
            ++it;
            break;
        }
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (status == SN_ERR_NOT_CONVERGED) fail(status, "not converged in %d iterations", o->max_it);
    (void)verified;
    if (stats) {
        stats->iters = it;
        stats->sweeps = ctx->sweeps;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

int sn_response(sn_context* ctx, const double* r, const double* phi, int face, const void* psi, sn_precision prec,
                double* out) {
    g_err.clear();
    if (!ctx || !out) return fail(SN_ERR_INVALID, "NULL argument");
    if (ctx->order >= 2) return fail(SN_ERR_UNSUPPORTED, "built for order 1 only");
    const int dim = ctx->mesh.dim;
    if (face < -1 || face >= 2 * dim) return fail(SN_ERR_INVALID, "face must be -1 or 0..%d", 2 * dim - 1);
    if (face >= 0 && !psi) return fail(SN_ERR_INVALID, "psi is needed for a face functional");
    if ((r == nullptr) != (phi == nullptr)) return fail(SN_ERR_INVALID, "r and phi must be given together");
    if (prec != SN_FP64 && prec != SN_FP32) return fail(SN_ERR_INVALID, "unknown precision");
    int rc;
    if ((rc = ctx->wn.ensure(ctx->ndirs))) return rc;
    std::vector<double> wn(ctx->ndirs, 0.0);
    if (face >= 0) {
        const int ax = face >> 1;
        const double sgn = (face & 1) ? 1.0 : -1.0;
        for (int d = 0; d < ctx->ndirs; ++d) {
            double on = sgn * ctx->omega[3 * d + ax];
            wn[d] = on > 0 ? ctx->hw[d] * on : 0.0;
        }
    }
    HIPCHK(hipMemcpyAsync(ctx->wn.p, wn.data(), ctx->ndirs * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    const double h[3] = {ctx->mesh.hx, ctx->mesh.hy, dim == 3 ? ctx->mesh.hz : 1.0};
    double res[3];
    if (prec == SN_FP64)
        HIPCHK(launch_response<double>(ctx->nc, ctx->nn, ctx->mesh.nx, ctx->mesh.ny, ctx->mesh.nz, h, r, phi, face,
                                       ctx->ndirs, ctx->wn.p, (const double*)psi, ctx->rpart.p, ctx->nrpart,
                                       ctx->res3.p, ctx->stream));
    else
        HIPCHK(launch_response<float>(ctx->nc, ctx->nn, ctx->mesh.nx, ctx->mesh.ny, ctx->mesh.nz, h, r, phi, face,
                                      ctx->ndirs, ctx->wn.p, (const float*)psi, ctx->rpart.p, ctx->nrpart,
                                      ctx->res3.p, ctx->stream));
    HIPCHK(hipMemcpyAsync(res, ctx->res3.p, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *out = res[0] + res[1];
    return 0;
}

int sn_response_noalloc(sn_context* ctx, const double* r, const double* phi, int face, const void* psi,
                        sn_precision prec, double* out) {
    g_err.clear();
    if (!ctx || !out) return fail(SN_ERR_INVALID, "NULL argument");
    if (ctx->order >= 2) return fail(SN_ERR_UNSUPPORTED, "built for order 1 only");
    const int dim = ctx->mesh.dim;
    if (face < -1 || face >= 2 * dim) return fail(SN_ERR_INVALID, "face must be -1 or 0..%d", 2 * dim - 1);
    if (face >= 0 && !psi) return fail(SN_ERR_INVALID, "psi is needed for a face functional");
    if ((r == nullptr) != (phi == nullptr)) return fail(SN_ERR_INVALID, "r and phi must be given together");
    if (prec != SN_FP64 && prec != SN_FP32) return fail(SN_ERR_INVALID, "unknown precision");
    // scratch layout: [0, nd) face weights, then 3 * nparts partial sums, then the 3 results
    const long need = (long)ctx->ndirs + 3L * ctx->nrpart + 3;
    if (need > NOALLOC_SCRATCH_DOUBLES)
        return fail(SN_ERR_INVALID, "sn_response_noalloc: %d directions need %ld scratch doubles, more than the "
                    "fixed %ld (at most %ld directions)", ctx->ndirs, need, NOALLOC_SCRATCH_DOUBLES,
                    NOALLOC_SCRATCH_DOUBLES - 3L * 1024 - 3);
    if (!ctx->noalloc)
        return fail(SN_ERR_HIP, "device scratch address unavailable: %s", hipGetErrorString(ctx->noalloc_err));
    double* wn_d = ctx->noalloc;
    double* part = wn_d + ctx->ndirs;
    double* res_d = part + 3L * ctx->nrpart;
    std::vector<double> wn(ctx->ndirs, 0.0);
    if (face >= 0)
        for (int d = 0; d < ctx->ndirs; ++d) {
            const double on = face_dot(ctx, face, d);
            wn[d] = on > 0 ? ctx->hw[d] * on : 0.0;
        }
    HIPCHK(hipMemcpyAsync(wn_d, wn.data(), ctx->ndirs * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    const double h[3] = {ctx->mesh.hx, ctx->mesh.hy, dim == 3 ? ctx->mesh.hz : 1.0};
    if (prec == SN_FP64)
        HIPCHK(launch_response<double>(ctx->nc, ctx->nn, ctx->mesh.nx, ctx->mesh.ny, ctx->mesh.nz, h, r, phi, face,
                                       ctx->ndirs, wn_d, (const double*)psi, part, ctx->nrpart, res_d, ctx->stream));
    else
        HIPCHK(launch_response<float>(ctx->nc, ctx->nn, ctx->mesh.nx, ctx->mesh.ny, ctx->mesh.nz, h, r, phi, face,
                                      ctx->ndirs, wn_d, (const float*)psi, part, ctx->nrpart, res_d, ctx->stream));
    double res[3];
    HIPCHK(hipMemcpyAsync(res, res_d, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *out = res[0] + res[1];
    return 0;
}

int sn_gradient(sn_context* ctx, const void* psi, const void* psi_adj, sn_precision prec, const double* phi,
                const double* chi, double* g_t, double* g_s) {
    g_err.clear();
    if (!ctx || !psi || !psi_adj || !phi || !chi || !g_t || !g_s) return fail(SN_ERR_INVALID, "NULL argument");
    if (ctx->order >= 2) return fail(SN_ERR_UNSUPPORTED, "built for order 1 only");
    const double h[3] = {ctx->mesh.hx, ctx->mesh.hy, ctx->mesh.dim == 3 ? ctx->mesh.hz : 1.0};
    if (prec == SN_FP64)
        HIPCHK(launch_gradient<double>(ctx->nc, ctx->nn, ctx->ndirs, ctx->w.p, h, ctx->sigt.p, ctx->sigs.p,
                                       (const double*)psi, (const double*)psi_adj, phi, chi, g_t, g_s, ctx->stream));
    else if (prec == SN_FP32)
        HIPCHK(launch_gradient<float>(ctx->nc, ctx->nn, ctx->ndirs, ctx->w.p, h, ctx->sigt.p, ctx->sigs.p,
                                      (const float*)psi, (const float*)psi_adj, phi, chi, g_t, g_s, ctx->stream));
    else
        return fail(SN_ERR_INVALID, "unknown precision");
    return 0;
}

int sn_krylov_solve(sn_context* ctx, const double* q, const double* inflow, double* phi, const sn_krylov_opts* o,
                    sn_iter_stats* stats) {
    g_err.clear();
    auto t0 = std::chrono::steady_clock::now();
    if (!ctx || !phi || !o) return fail(SN_ERR_INVALID, "NULL argument");
    if (ctx->order >= 2 && (o->transpose || (o->use_dsa && o->dsa_form != SN_DSA_DIAGONAL)))
        return fail(SN_ERR_UNSUPPORTED, "order %d: forward sweeps with the diagonal DSA only", ctx->order);
    if (!(o->tol >= 0) || o->max_it < 1) return fail(SN_ERR_INVALID, "bad tolerance or iteration limit");
    if (o->restart < 1 || o->restart > SN_KRYLOV_MAX_RESTART)
        return fail(SN_ERR_INVALID, "restart must be in 1..%d", SN_KRYLOV_MAX_RESTART);
    if (o->use_dsa && bad_dsa_opts(o->dsa)) return fail(SN_ERR_INVALID, "bad DSA options");
    if (o->dsa_form != SN_DSA_DIAGONAL && o->dsa_form != SN_DSA_TRIANGULAR)
        return fail(SN_ERR_INVALID, "unknown DSA form %d", o->dsa_form);
    struct FaceReuse {
        sn_context* c;
        explicit FaceReuse(sn_context* c_) : c(c_) {
            c->fkey[0].valid = c->fkey[1].valid = false;
            c->face_reuse = true;
            c->src_tok = false;
        }
        ~FaceReuse() {
            c->face_reuse = false;
            c->src_tok = false;
        }
    } face_reuse(ctx);
    const long n = ctx->nc * ctx->nn;
    const int m = o->restart, tr = o->transpose ? 1 : 0;
    const bool dsa = o->use_dsa && ctx->nthick > 0;
    const bool tri = dsa && o->dsa_form == SN_DSA_TRIANGULAR;
    int rc;
    const bool fresh_zero = !ctx->kzero.p;
    if ((rc = ctx->kv.ensure((size_t)(m + 1) * n)) || (rc = ctx->kw.ensure(n)) || (rc = ctx->kb.ensure(n)) ||
        (rc = ctx->kzero.ensure(n)) || (rc = ctx->kdot.ensure(SN_KRYLOV_MAX_RESTART + 1)) ||
        (rc = ctx->kpart.ensure((size_t)(SN_KRYLOV_MAX_RESTART + 1) * krylov_blocks(n))))
        return rc;
    if (dsa && (rc = ctx->kz.ensure((size_t)m * n))) return rc;
    if (fresh_zero) HIPCHK(hipMemsetAsync(ctx->kzero.p, 0, n * sizeof(double), ctx->stream));
    if (!ctx->kdot_host)
        HIPCHK(hipHostMalloc((void**)&ctx->kdot_host, (SN_KRYLOV_MAX_RESTART + 2) * sizeof(double),
                             hipHostMallocDefault));
    ctx->sweeps = 0;
    double* V = ctx->kv.p;
    double* Z = dsa ? ctx->kz.p : ctx->kv.p;
    double* w = ctx->kw.p;
    // the moment of a full sweep from (phi, q, inflow) into out (order p >= 2:
    // through a psi workspace)
    if (ctx->order >= 2 && (rc = ctx->psi64.ensure((size_t)n * ctx->ndirs))) return rc;
    auto sweep_flux = [&](const double* ph, const double* qq, const double* in, double* out) -> int {
        if (ctx->order >= 2) {
            HIPCHK(launch_sweep_hp(ctx->hp, ctx->mesh.nx, ctx->mesh.ny, ctx->ndirs, ctx->nbf, ctx->dirs.p,
                                   ctx->sigt.p, ctx->sigs.p, ph, qq, in, ctx->psi64.p, ctx->stream));
            HIPCHK(launch_moment_hp(ctx->nc, ctx->ndirs, ctx->nn, ctx->w.p, ctx->psi64.p, out, ctx->stream));
            ++ctx->sweeps;
            return 0;
        }
        return do_sweep_flux(ctx, ph, nullptr, qq, in, tr, SN_FP64, out, 0);
    };
    // S x = x - sum_d w_d L_d^{-1} (Sigma_s x) with zero source and vacuum: into w, then w = x - w
    auto apply_S = [&](const double* x) -> int {
        int e;
        if ((e = sweep_flux(x, nullptr, nullptr, w))) return e;
        HIPCHK(launch_axpby(n, 1.0, x, -1.0, w, ctx->stream));
        return 0;
    };
    // b = sum_d w_d L_d^{-1}(q_d + inflow load)
    if ((rc = sweep_flux(nullptr, q, inflow, ctx->kb.p))) return rc;
    double bb;
    if ((rc = dots(ctx, 1, ctx->kb.p, ctx->kb.p, &bb))) return rc;
    double bnorm = std::sqrt(bb);
    if (bnorm == 0.0) bnorm = 1.0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h(m + 1), h2(m + 1);
    int it = 0, status = SN_ERR_NOT_CONVERGED;
    while (it < o->max_it && status == SN_ERR_NOT_CONVERGED) {
        // r = b - S x
        if ((rc = apply_S(phi))) return rc;
        HIPCHK(launch_axpby(n, 1.0, ctx->kb.p, -1.0, w, ctx->stream));
        double rr;
        if ((rc = dots(ctx, 1, w, w, &rr))) return rc;
        const double beta = std::sqrt(rr);
        if (!std::isfinite(beta)) {
            status = fail(SN_ERR_DIVERGED, "Krylov residual is not finite");
            break;
        }
        if (beta / bnorm <= o->tol) {
            status = SN_OK;
            break;
        }
        HIPCHK(launch_scale(n, 1.0 / beta, w, V, ctx->stream));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        bool stop = false;
        for (; j < m && it < o->max_it; ++j) {
            double* vj = V + (size_t)j * n;
            double* zj = Z + (size_t)j * n;
            int cgi = 0;
            if (dsa) {
                // the preconditioner applied to v_j as to a residual: z = v + P_T D_ff^{-1} Sigma_f R_T v
                sn_dsa_stats ds{};
                if ((rc = ctx->order >= 2 ? dsa_hp(ctx, ctx->kzero.p, vj, zj, &o->dsa, &ds)
                                          : do_dsa(ctx, ctx->kzero.p, vj, zj, &o->dsa, &ds))) {
                    status = rc;
                    break;
                }
                cgi = ds.cg_iters;
                if (tri && (rc = triangular_step(ctx, nullptr, zj, tr, SN_FP64))) return rc;
            }
            if ((rc = apply_S(zj))) return rc;
            // classical Gram-Schmidt, twice
            if ((rc = dots(ctx, j + 1, V, w, h.data()))) return rc;
            HIPCHK(launch_multi_axpy(n, j + 1, V, ctx->kdot.p, -1.0, w, ctx->stream));
            if ((rc = dots(ctx, j + 1, V, w, h2.data()))) return rc;
            HIPCHK(launch_multi_axpy(n, j + 1, V, ctx->kdot.p, -1.0, w, ctx->stream));
            double ww;
            if ((rc = dots(ctx, 1, w, w, &ww))) return rc;
            const double hn = std::sqrt(ww);
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i] + h2[i];
            H[(size_t)(j + 1) * m + j] = hn;
            if (hn > 0.0) HIPCHK(launch_scale(n, 1.0 / hn, w, V + (size_t)(j + 1) * n, ctx->stream));
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], c2 = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * c2;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c2;
            }
            {
                const double a = H[(size_t)j * m + j], c2 = H[(size_t)(j + 1) * m + j];
                const double den = std::sqrt(a * a + c2 * c2);
                cs[j] = den > 0.0 ? a / den : 1.0;
                sn[j] = den > 0.0 ? c2 / den : 0.0;
                H[(size_t)j * m + j] = den;
                H[(size_t)(j + 1) * m + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
            }
            const double res = std::fabs(g[j + 1]) / bnorm;
            if (stats && stats->res_hist) stats->res_hist[it] = res;
            if (stats && stats->cg_hist) stats->cg_hist[it] = cgi;
            ++it;
            if (!std::isfinite(res)) {
                status = fail(SN_ERR_DIVERGED, "Krylov residual is not finite");
                ++j;
                break;
            }
            if (res <= o->tol || hn == 0.0) {
                stop = true;
                ++j;
                break;
            }
        }
        if (status == SN_ERR_CG_BREAKDOWN || status == SN_ERR_HIP || status == SN_ERR_NOMEM) break;
        // x += Z y, H(0:j, 0:j) y = g(0:j)
        for (int i = j - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < j; ++k) s -= H[(size_t)i * m + k] * y[k];
            y[i] = s / H[(size_t)i * m + i];
        }
        if (j > 0) {
            for (int i = 0; i < j; ++i) ctx->kdot_host[i] = y[i];
            HIPCHK(hipMemcpyAsync(ctx->kdot.p, ctx->kdot_host, j * sizeof(double), hipMemcpyHostToDevice,
                                  ctx->stream));
            HIPCHK(launch_multi_axpy(n, j, Z, ctx->kdot.p, 1.0, phi, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
        }
        if (status != SN_ERR_NOT_CONVERGED) break;
        if (stop) status = SN_OK;
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (status == SN_ERR_NOT_CONVERGED) fail(status, "not converged in %d iterations", o->max_it);
    if (stats) {
        stats->iters = it;
        stats->sweeps = ctx->sweeps;
        stats->fp64_checks = 0;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

int sn_adjoint_source(sn_context* ctx, const double* r, int face, double* q_adj, double* inflow_adj) {
    g_err.clear();
    if (!ctx) return fail(SN_ERR_INVALID, "context is NULL");
    if (ctx->order >= 2) return fail(SN_ERR_UNSUPPORTED, "built for order 1 only");
    if (face < -1 || face >= 2 * ctx->mesh.dim) return fail(SN_ERR_INVALID, "face must be -1 or 0..%d", 2 * ctx->mesh.dim - 1);
    if ((r != nullptr) != (q_adj != nullptr)) return fail(SN_ERR_INVALID, "r and q_adj must be given together");
    if ((face >= 0) != (inflow_adj != nullptr)) return fail(SN_ERR_INVALID, "a face needs inflow_adj (and only then)");
    if (r) HIPCHK(launch_scale(ctx->nc, 4.0 * kPi, r, q_adj, ctx->stream));
    if (face >= 0) {
        std::vector<int> out(ctx->ndirs);
        for (int d = 0; d < ctx->ndirs; ++d) out[d] = face_dot(ctx, face, d) > 0.0 ? 1 : 0;
        HIPCHK(hipMemcpy(ctx->face_out.p, out.data(), ctx->ndirs * sizeof(int), hipMemcpyHostToDevice));
        long f0, f1;
        face_range(ctx->mesh, face, &f0, &f1);
        HIPCHK(launch_face_data(ctx->ndirs, ctx->nbf, f0, f1, ctx->face_out.p, inflow_adj, ctx->stream));
    }
    return 0;
}

int sn_face_response(sn_context* ctx, const double* phi, const double* q, const double* inflow, int face,
                     double* out) {
    g_err.clear();
    if (!ctx || !out) return fail(SN_ERR_INVALID, "NULL argument");
    if (ctx->order >= 2) return fail(SN_ERR_UNSUPPORTED, "built for order 1 only");
    if (face < 0 || face >= 2 * ctx->mesh.dim) return fail(SN_ERR_INVALID, "face must be 0..%d", 2 * ctx->mesh.dim - 1);
    const int S = ctx->part_stride;
    int rc;
    if ((rc = ctx->psi_a.ensure((size_t)ctx->nc * S * ctx->nn))) return rc;
    const double h[3] = {ctx->mesh.hx, ctx->mesh.hy, ctx->mesh.dim == 3 ? ctx->mesh.hz : 1.0};
    double total = 0.0;
    for (size_t pi = 0; pi < ctx->parts.size(); ++pi) {
        std::vector<double> wn(S, 0.0);
        bool any = false;
        for (int l = 0; l < S; ++l) {
            const int d = ctx->part_dirs[pi][l];
            if (d < 0) continue;
            const double on = face_dot(ctx, face, d);
            if (on > 0.0) {
                wn[l] = ctx->hw[d] * on;
                any = true;
            }
        }
        if (!any) continue;
        HIPCHK(hipMemcpy(ctx->part_wn.p + pi * S, wn.data(), S * sizeof(double), hipMemcpyHostToDevice));
        if ((rc = do_sweep(ctx, phi, nullptr, q, inflow, 0, SN_FP64, ctx->psi_a.p, &ctx->parts[pi]))) return rc;
        HIPCHK(launch_response<double>(ctx->nc, ctx->nn, ctx->mesh.nx, ctx->mesh.ny, ctx->mesh.nz, h, nullptr, nullptr,
                                       face, S, ctx->part_wn.p + pi * S, ctx->psi_a.p, ctx->rpart.p, ctx->nrpart,
                                       ctx->res3.p, ctx->stream));
        double r3[3];
        HIPCHK(hipMemcpyAsync(r3, ctx->res3.p, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        total += r3[1];
    }
    *out = total;
    return 0;
}

int sn_adjoint_gradient(sn_context* ctx, const double* phi, const double* q, const double* inflow, const double* chi,
                        const double* q_adj, const double* inflow_adj, double* g_t, double* g_s) {
    g_err.clear();
    if (!ctx || !phi || !chi || !g_t || !g_s) return fail(SN_ERR_INVALID, "NULL argument");
    if (ctx->order >= 2) return fail(SN_ERR_UNSUPPORTED, "built for order 1 only");
    const int S = ctx->part_stride;
    int rc;
    if ((rc = ctx->psi_a.ensure((size_t)ctx->nc * S * ctx->nn)) || (rc = ctx->psi_b.ensure((size_t)ctx->nc * S * ctx->nn)))
        return rc;
    const double h[3] = {ctx->mesh.hx, ctx->mesh.hy, ctx->mesh.dim == 3 ? ctx->mesh.hz : 1.0};
    for (size_t pi = 0; pi < ctx->parts.size(); ++pi) {
        const SweepPart* part = &ctx->parts[pi];
        // psi_d regenerated from the converged flux; the adjoint psi_d from chi
        if ((rc = do_sweep(ctx, phi, nullptr, q, inflow, 0, SN_FP64, ctx->psi_a.p, part))) return rc;
        if ((rc = do_sweep(ctx, chi, nullptr, q_adj, inflow_adj, 1, SN_FP64, ctx->psi_b.p, part))) return rc;
        HIPCHK(launch_gradient<double>(ctx->nc, ctx->nn, S, ctx->part_w.p + pi * S, h, ctx->sigt.p, ctx->sigs.p,
                                       ctx->psi_a.p, ctx->psi_b.p, phi, chi, g_t, pi == 0 ? g_s : nullptr, ctx->stream,
                                       pi > 0));
    }
    return 0;
}

}  // extern "C"
