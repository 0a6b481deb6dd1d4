/*
 * sn.h -- C ABI of the MI355X (gfx950) library for discrete-ordinates (S_N)
 * source iteration with heterogeneous, thick-only diffusion synthetic
 * acceleration, on uniform Cartesian grids with a Q1 upwind-DG discretisation.
 *
 * Problem (Section 1, eq. eq and eq. sntransport of the paper): steady,
 * mono-energetic transport with isotropic scattering,
 *     Omega_d . grad psi_d + sigma_t psi_d = sigma_s / (4 pi) phi + q / (4 pi),
 *     phi = sum_d w_d psi_d,  sum_d w_d = 4 pi,
 * with psi_d prescribed on the inflow boundary (vacuum when not given).
 * Discretisation (Section 3.1, eq. Tmat1 at eps = 1): Q1 Lagrange basis on the
 * cell corners, exact integrals, upwind face coupling.
 *
 * Data layout (all arrays are caller-owned; "device" means GPU memory
 * reachable from the context's device, e.g. a torch tensor's data pointer):
 *   cell c = (k*ny + j)*nx + i (x fastest); nodes per cell nn = 4 (2D) or 8
 *   (3D), node n = a + 2b + 4c with a/b/c the low (0) or high (1) corner along
 *   x/y/z.
 *   sigma_t, sigma_s, q : [ncells]            FP64, per-cell constants;
 *                          q is a total isotropic source density.
 *   phi                 : [ncells][nn]        FP64 nodal scalar flux.
 *   psi                 : [ncells][ndirs][nn] FP64 or FP32 (sn_precision).
 *   inflow              : [ndirs][nbf]        FP64, nbf = sn_inflow_size();
 *     per direction the upwind x face (x = 0 if mu > 0, else x = nx*hx), then
 *     the upwind y face, then (3D) the upwind z face; node order inside a face:
 *     x face ((k*ny + j)*F + b + 2c), y face ((k*nx + i)*F + a + 2c),
 *     z face ((j*nx + i)*4 + a + 2b), F = 2 (2D) or 4 (3D).
 *   Directions are given by the caller (host arrays); a 2D problem ignores
 *   the third component.  No direction component may be zero.
 *
 * Streams: every entry point enqueues its work on the context's HIP stream
 * and, except where stated, returns without waiting for it.  One context per
 * stream; contexts are not thread-safe.
 *
 * Errors: every int-returning entry point returns one of the SN_* codes; the
 * message of the last error on the calling thread is in sn_last_error().
 * Device buffers are never freed or resized by the library.
 */
#ifndef SN_H
#define SN_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SN_OK = 0,
    SN_ERR_INVALID = 1,        /* bad argument: null, size, non-finite, sigma < 0, sigma_s > sigma_t */
    SN_ERR_UNSUPPORTED = 2,    /* valid but not implemented (e.g. a zero direction component) */
    SN_ERR_NOMEM = 3,          /* device allocation failed */
    SN_ERR_HIP = 4,            /* a HIP runtime call failed */
    SN_ERR_NOT_CONVERGED = 5,  /* iteration limit reached; outputs hold the last iterate */
    SN_ERR_DIVERGED = 6,       /* residual non-finite or above 1e6 x the first residual */
    SN_ERR_CG_BREAKDOWN = 7    /* p^T D p <= 0 in the diffusion CG */
};

typedef enum { SN_FP64 = 0, SN_FP32 = 1 } sn_precision;

typedef struct {
    int dim;                   /* 2 or 3 */
    int nx, ny, nz;            /* cells per axis; nz = 1 in 2D */
    double hx, hy, hz;         /* cell widths; hz ignored in 2D */
    int order;                 /* DG order p (the paper runs 2 and 4 in Sec. 4): 0 or 1 for Q1 (the default,
                                  every entry point), 2, 3 or 4 for Q_p on the (p + 1)^2 Gauss-Lobatto nodes of
                                  each cell, node i + (p + 1) j, 2D only.  At p >= 2 the sweep, the moment,
                                  the DSA correction (any form; GMRES with block Jacobi, or the direct solve)
                                  and source iteration (FP64, forward, diagonal DSA, no checkpoints) are
                                  available; every other entry point returns SN_ERR_UNSUPPORTED.  The
                                  inflow data then has (p + 1) values per boundary face (sn_inflow_size). */
} sn_mesh;

typedef struct {
    int ndirs;
    const double *omega;       /* host [ndirs][3], unit vectors */
    const double *w;           /* host [ndirs], positive, sum 4 pi */
} sn_quad;

typedef struct sn_context sn_context;

/* Create a context for one mesh, quadrature and set of cross sections.
 * sigma_t, sigma_s: device [ncells] FP64 (copied; the caller may free them
 * afterwards).  eta: thick threshold, a cell is thick iff sigma_s >= eta
 * (Sections 2.3 and 3.2; the paper uses eta = 1).  Builds the thick-cell list and the
 * diffusion preconditioner on the GPU.  stream: a hipStream_t (NULL = default
 * stream).  Synchronises the stream before returning.
 * Errors: INVALID (bad sizes, sigma_s > sigma_t, negative or non-finite
 * sigma, weights not summing to 4 pi within 1e-12), UNSUPPORTED (a direction
 * with a zero component, grid above 1023 tiles per axis), NOMEM, HIP. */
int sn_context_create(const sn_mesh *mesh, const sn_quad *quad, const double *sigma_t, const double *sigma_s,
                      double eta, void *stream, sn_context **out);

/* Free the context and its device workspace (waits for its stream). */
void sn_context_destroy(sn_context *ctx);

/* Number of boundary-face nodes per direction in the inflow layout. */
long sn_inflow_size(const sn_mesh *mesh);

/* Number of thick cells of the context. */
int sn_thick_count(const sn_context *ctx);

/* Transport sweep, Section 2.2 eq. psi: for every direction d,
 *   psi_d = L_d^{-1} ( M (sigma_s phi + q) / 4pi + inflow load )   (transpose = 0)
 *   psi_d = L_d^{-T} ( same volume load + boundary load )          (transpose = 1).
 * L_d^T = L_{-d} on this discretisation, so the transposed sweep visits the
 * cells from the downwind corner; in that mode `inflow` holds the data on the
 * faces with Omega_d . n > 0, laid out as the inflow of the reversed direction.
 * phi: device [ncells][nn] or NULL (zero); q: device [ncells] or NULL (zero);
 * inflow: device [ndirs][nbf] or NULL (vacuum); psi: device output
 * [ncells][ndirs][nn], FP64 or FP32 per prec (FP32: the local solves and psi
 * are FP32; the source is formed in FP64 and rounded once). */
int sn_sweep(sn_context *ctx, const double *phi, const double *q, const double *inflow, int transpose,
             sn_precision prec, void *psi);

/* Scalar-flux moment, eq. phi: phi_out = sum_d w_d psi_d, accumulated in FP64.
 * psi: device [ncells][ndirs][nn] in prec; phi_out: device [ncells][nn]. */
int sn_scalar_flux(sn_context *ctx, const void *psi, sn_precision prec, double *phi_out);

typedef struct {
    double cg_rtol;            /* stop when ||r|| <= cg_rtol ||b|| (zero initial guess) */
    int cg_maxit;              /* iteration cap (SN_ERR_NOT_CONVERGED is not raised for it) */
    int mass_kind;             /* 0: Sigma_f = mass of sigma_s; 1: mass of sigma_t (Sec. 2.2) */
    int precond;               /* SN_PRECOND_BLOCK_JACOBI: inverse diagonal cell blocks.
                                  SN_PRECOND_DIRECT: see below.
                                  SN_PRECOND_MG: one symmetric geometric-multigrid V-cycle -- damped block
                                  Jacobi on the DG level, the continuous Q1 space on the vertices of the
                                  thick cells (Galerkin operator), vertex-grid coarsening by two with
                                  (bi/tri)linear interpolation and damped Jacobi, a dense solve on <= 256
                                  unknowns.  The hierarchy is built on the first use in a context
                                  (from the SIP operator, whatever the diffusion form). */
    int diffusion;             /* the diffusion form of Sec. 3.1 whose thick principal submatrix is solved:
                                  SN_DIFFUSION_SIP (eq. SIP, penalty max(kappa_0, 8 D / h), CG as above);
                                  SN_DIFFUSION_NIP (eq. NIP: the term -int [[u]]{D dv/dn} dropped, penalty
                                  kappa_0) or SN_DIFFUSION_MNIP (NIP with the penalty of eq. ModifiedF0:
                                  kappa_0 times the mean over the face's two cells of max(0.2 / (sigma_t h), 1),
                                  the thin neighbour's sigma_t included; on a domain face the cell's own
                                  factor).  The nonsymmetric forms are solved by GMRES(SN_DSA_GMRES_RESTART),
                                  zero initial guess, to the true residual ||b - D x|| <= cg_rtol ||b|| or
                                  cg_maxit iterations, right-preconditioned by the inverse of the form's own
                                  diagonal cell blocks (SN_PRECOND_BLOCK_JACOBI) or by one V-cycle of the SIP
                                  multigrid (SN_PRECOND_MG; effective where SIP and the form are close, as on a
                                  thick-only set, not for full DSA through thin cells).  A NaN or infinite
                                  residual returns SN_ERR_DIVERGED.  mNIP with sigma_t = 0 at a thick cell or
                                  its face neighbour returns SN_ERR_INVALID (the factor divides by sigma_t). */
} sn_dsa_opts;

#define SN_DIFFUSION_SIP 0
#define SN_DIFFUSION_NIP 1
#define SN_DIFFUSION_MNIP 2
#define SN_DSA_GMRES_RESTART 30

#define SN_PRECOND_BLOCK_JACOBI 0
#define SN_PRECOND_MG 1
#define SN_PRECOND_DIRECT 2    /* exact solve, any form: band LU with partial pivoting of the thick matrix,
                                  assembled and factored on the device on the first use of a form in a context
                                  (one workgroup; milliseconds for a few thousand unknowns), then one band
                                  solve per call.  Small systems only: nthick nn <= 8192 unknowns and
                                  kl + ku = 2 (w + 1) nn - 2 <= 1023, w the largest slot distance between
                                  face-neighbouring thick cells; SN_ERR_UNSUPPORTED beyond.  cg_rtol and
                                  cg_maxit are not used; stats report 0 iterations. */

typedef struct {
    int cg_iters;              /* CG (NIP, mNIP: GMRES) iterations of this call */
    double cg_relres;          /* final ||r|| / ||b|| */
    int n_thick_cells;
} sn_dsa_stats;

/* Heterogeneous DSA, Alg. 2 applied to the source-iteration residual:
 *   phi_out = phi_si + P_T D_ff^{-1} Sigma_f R_T (phi_si - phi_old),
 * D_ff the SIP diffusion operator (eq. SIP) on the thick DOFs only (principal
 * submatrix, Section 3.2), solved by preconditioned CG in FP64 (opts->precond).
 * Thin and void DOFs: phi_out = phi_si.  All three arrays device
 * [ncells][nn]; phi_out may alias phi_si.  The call waits until the CG stop
 * test has passed on the device (the kernels post the stop flags to pinned
 * host memory), fills stats (host, may be NULL) and returns with the final
 * update of phi_out enqueued on the stream.  Returns CG_BREAKDOWN if
 * p^T D p <= 0. */
int sn_dsa_thick_correct(sn_context *ctx, const double *phi_old, const double *phi_si, double *phi_out,
                         const sn_dsa_opts *opts, sn_dsa_stats *stats);

/* forms of the heterogeneous DSA (Section 2.3) */
#define SN_DSA_DIAGONAL 0      /* Alg. 2: thick-region update only */
#define SN_DSA_TRIANGULAR 1    /* Alg. 1: Alg. 2, then the thick part of the corrected residual is swept
                                  once (zero source, vacuum) and its moment added to the thin DOFs */

typedef struct {
    double tol;                /* stop when ||phi_SI - phi|| / ||b|| <= tol, b = sweep of q from phi = 0 */
    int max_it;
    int use_dsa;
    sn_precision prec;         /* precision of the sweep; moment, residual and DSA are FP64 (see fp32_refine) */
    sn_dsa_opts dsa;
    int transpose;             /* 1: adjoint iteration with L_d^{-T} sweeps */
    double *phi_ckpt;          /* device [ckpt_cap][ncells][nn] or NULL: phi after iteration it goes
                                  to slot it % ckpt_cap, so the last ckpt_cap iterates are kept */
    int ckpt_cap;              /* slots in phi_ckpt; must be >= 1 when phi_ckpt is not NULL */
    int fp32_refine;           /* SN_FP32 only.  0: plain FP32 form, every sweep FP32 on the full source
                                  (sigma_s phi + q)/4pi.  1: defect correction: after the first sweep the
                                  FP32 sweeps act on the increment sigma_s (phi_i - phi_{i-1}) and add their
                                  FP64 moment to phi_SI; phi_SI is recomputed by one FP64 sweep when that
                                  residual first drops below 1e-4 and whenever it meets tol, and the
                                  iteration stops only on the exact residual */
    int dsa_form;              /* SN_DSA_DIAGONAL or SN_DSA_TRIANGULAR (one extra sweep per iteration) */
} sn_iter_opts;

typedef struct {
    int iters;
    double *res_hist;          /* host [max_it] or NULL: relative residual per iteration */
    int *cg_hist;              /* host [max_it] or NULL: CG iterations per iteration */
    double seconds;            /* wall time of the call */
    int fp64_checks;           /* FP32 form with fp32_refine: number of FP64 verification sweeps */
    int sweeps;                /* transport sweeps of all directions performed by the call */
} sn_iter_stats;

/* Source iteration with optional heterogeneous DSA (eq. DSA_fp):
 *   phi_SI = sum_d w_d L_d^{-1}( M (sigma_s phi + q)/4pi + inflow load ),
 *   stop test on ||phi_SI - phi|| / ||b|| before the DSA step,
 *   phi <- phi_SI + P_T D_ff^{-1} Sigma_f R_T (phi_SI - phi)   (or phi <- phi_SI).
 * q: device [ncells] or NULL; inflow: device [ndirs][nbf] or NULL;
 * phi_inout: device [ncells][nn], initial guess in, last iterate out.
 * Waits on the host once per iteration (the residual and the CG stop flags
 * are read from pinned host memory).  With DSA, every CG solve after the
 * first of a call starts from the previous solve's correction, scaled by a
 * one-dimensional Galerkin projection onto the new right-hand side (the stop
 * test stays ||r|| <= cg_rtol ||b||).
 * Returns OK, NOT_CONVERGED, DIVERGED or CG_BREAKDOWN (phi_inout holds the
 * last iterate in all three error cases). */
int sn_source_iterate(sn_context *ctx, const double *q, const double *inflow, double *phi_inout,
                      const sn_iter_opts *opts, sn_iter_stats *stats);

/* Krylov solve of the scalar-flux Schur system (Section 2.2, eq. schur):
 *   S phi = b,  S = I - sum_d w_d L_d^{-1} Sigma_s,  b = sum_d w_d L_d^{-1}(q_d + inflow load),
 * by flexible GMRES(restart) (classical Gram-Schmidt applied twice, Givens
 * rotations on the host), right-preconditioned by the heterogeneous DSA
 * (use_dsa; dsa_form as in sn_iter_opts) applied to a Krylov vector v as to a
 * residual, z = v + P_T D_ff^{-1} Sigma_f R_T v (eq. approxD; the DSA's CG
 * tolerance may vary the preconditioner, hence the flexible form).  An
 * iteration is one application of S (one FP64 sweep of every direction).
 * Stops when the least-squares residual ||b - S phi|| / ||b|| <= tol, the
 * same quantity as the source-iteration residual.
 * phi_inout: device [ncells][nn], initial guess in, solution out.  stats:
 * res_hist[k] the residual after iteration k, cg_hist[k] the CG iterations of
 * its preconditioner.  Workspace: (2 restart + 4) FP64 vectors of ncells*nn.
 * Waits on the host a few times per iteration (dot products).
 * Returns OK, NOT_CONVERGED, DIVERGED or CG_BREAKDOWN. */
#define SN_KRYLOV_MAX_RESTART 200
typedef struct {
    double tol;
    int max_it;                /* iterations (applications of S) in total */
    int restart;               /* Krylov space size m, 1..SN_KRYLOV_MAX_RESTART (the paper uses 30) */
    int use_dsa;
    int dsa_form;
    sn_dsa_opts dsa;
    int transpose;             /* 1: the adjoint system with L_d^{-T} sweeps */
} sn_krylov_opts;
int sn_krylov_solve(sn_context *ctx, const double *q, const double *inflow, double *phi_inout,
                    const sn_krylov_opts *opts, sn_iter_stats *stats);

/* Adjoint sources of the two responses (derived from the block system,
 * eq. system): for J = sum_c r_c int_c phi the adjoint volume source is
 * q_adj = 4 pi r (device [ncells], given with r); for the partial outflow
 * current through domain face `face` (2 axis + side, -1 none) the transposed
 * sweep's boundary data is 1 on that face for every direction leaving
 * through it and 0 elsewhere (inflow_adj: device [ndirs][nbf], in the layout
 * of the reversed directions' inflow).  r/q_adj and face/inflow_adj are
 * given together or not at all. */
int sn_adjoint_source(sn_context *ctx, const double *r, int face, double *q_adj, double *inflow_adj);

/* Partial outflow current of the solution phi through domain face `face`,
 *   J = sum_{d: Omega_d.n > 0} w_d (Omega_d.n) int_face psi_d,
 * psi_d = L_d^{-1}(M (sigma_s phi + q)/4pi + inflow load) regenerated one
 * octant (3D) or quadrant (2D) at a time, so no angular flux of all
 * directions is held (workspace ncells * part * nn FP64, part = the largest
 * octant's direction count rounded up to 4).  *out (host) after a stream
 * synchronisation; the octants are summed in a fixed order. */
int sn_face_response(sn_context *ctx, const double *phi, const double *q, const double *inflow, int face,
                     double *out);

/* Adjoint gradient of a linear response (derived from the block system):
 *   g_t[c] = -sigma_t,c sum_d w_d psi_adj_d,c^T M_c psi_d,c     (d J / d log sigma_t,c)
 *   g_s[c] =  sigma_s,c chi_c^T M_c phi_c / 4pi                  (d J / d log sigma_s,c)
 * with psi_d = L_d^{-1}(M (sigma_s phi + q)/4pi + inflow load) regenerated
 * from the converged flux phi (the checkpoint of the forward solve) and
 * psi_adj_d = L_d^{-T}(M (sigma_s chi + q_adj)/4pi + inflow_adj load) from
 * the converged adjoint flux chi, both one octant (quadrant) at a time: the
 * peak workspace is two FP64 angular fluxes of one octant, never of all
 * directions.  q, inflow, q_adj, inflow_adj may be NULL (zero / vacuum).
 * g_t, g_s: device [ncells] FP64 outputs. */
int sn_adjoint_gradient(sn_context *ctx, const double *phi, const double *q, const double *inflow,
                        const double *chi, const double *q_adj, const double *inflow_adj, double *g_t,
                        double *g_s);

/* Adjoint gradient contraction (derived from the block system, eq. system):
 *   g_t[c] = -sigma_t,c sum_d w_d psi_adj_d,c^T M_c psi_d,c       (d J / d log sigma_t,c)
 *   g_s[c] =  sigma_s,c chi_c^T M_c phi_c / 4pi                    (d J / d log sigma_s,c)
 * for a response J whose adjoint angular flux psi_adj_d = L_d^{-T}(...) comes
 * from a transposed sweep at the converged adjoint flux chi.  psi, psi_adj:
 * device [ncells][ndirs][nn] in prec; phi, chi: device [ncells][nn];
 * g_t, g_s: device [ncells] FP64 outputs. */
int sn_gradient(sn_context *ctx, const void *psi, const void *psi_adj, sn_precision prec, const double *phi,
                const double *chi, double *g_t, double *g_s);

/* Linear response of a solution (the detector functionals of the adjoint):
 *   J = sum_c r_c int_c phi                                        (r != NULL)
 *     + sum_{d: Omega_d.n > 0} w_d (Omega_d.n) int_face psi_d       (face >= 0)
 * r: device [ncells] FP64 detector density or NULL (then phi must be NULL);
 * face: -1 (none) or domain face 2*axis + side (side 1 = high end of the
 * axis); psi: device [ncells][ndirs][nn] in prec (needed when face >= 0).
 * The sum is reduced in a fixed order on the device; *out (host) is written
 * after a stream synchronisation. */
int sn_response(sn_context *ctx, const double *r, const double *phi, int face, const void *psi,
                sn_precision prec, double *out);

/* sn_response for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same functional, arguments, kernels and result (bit for bit) as
 * sn_response, but it allocates nothing.  Its face weights, partial sums and
 * result live in a fixed scratch array of 16384 doubles (128 KiB) that every
 * GPU the library runs on holds from the library's load until the process
 * ends; its device address is looked up once per device when the first
 * context on that device is created.  Every call on one GPU shares that
 * array and overwrites it completely, so calls that overlap on one GPU (two
 * streams or threads at once) race; serialise them.  Needs ndirs + 3 * 1024
 * + 3 <= 16384 (at most 13309 directions): returns SN_ERR_INVALID beyond it,
 * SN_ERR_HIP if the scratch address could not be looked up.  *out (host)
 * after a stream synchronisation. */
int sn_response_noalloc(sn_context *ctx, const double *r, const double *phi, int face, const void *psi,
                        sn_precision prec, double *out);

/* Kernel timing for measurement.  enable = 1: every subsequent call records
 * HIP events on the context's stream around the sweep kernels of each sweep
 * (excluding the source and face-initialisation kernels) and around each DSA
 * solve; enable = 2: around the sweep kernels only (each recorded event holds
 * the next kernel back by a few microseconds, so fewer events perturb a timed
 * run less); enable = 0: off.  sn_kernel_timing waits for the stream, returns
 * the summed durations (ms) and counts since the last query or enable, and
 * resets them.  Enabling or disabling synchronises the stream. */
int sn_set_kernel_timing(sn_context *ctx, int enable);
int sn_kernel_timing(sn_context *ctx, double *sweep_ms, int *sweep_count, double *dsa_ms, int *dsa_count);

/* Message of the last error on the calling thread ("" if none). */
const char *sn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SN_H */
