/*
 * libdp — distance-preconditioned Wilson-clover inversion on one MI355X (gfx950).
 *
 * Method: G.M. de Divitiis, R. Petronzio, N. Tantalo, "Distance
 * preconditioning for lattice Dirac operators".  The lattice Dirac system
 * (D[U] + M) S = eta (eq. linsysunprec) is solved through the redefined
 * fields of eq. redeft and the preconditioned system of eq. linsysprec,
 * whose operator differs from D + M only in the time-direction derivatives
 * (modified nabla_0, nabla*_0 and the boundary rule eq. redeftbc), and the
 * propagator and correlator are restored afterwards (eq. backcorrection).
 *
 * Conventions of this interface
 * -----------------------------
 *  - dims = {T, L1, L2, L3}: time first; every extent even and >= 2.
 *  - Host field layouts are complex128 interleaved (re, im) with x0 slowest
 *    and x3 fastest:
 *      gauge  U  [x0][x1][x2][x3][mu][a][b]   mu = 0 (time), 1, 2, 3
 *      spinor    [x0][x1][x2][x3][spin][colour]  (12 complex per site)
 *      clover C  [x0][x1][x2][x3][12][12]     row/col 3*spin + colour
 *    Several right-hand sides are stored one after the other.
 *  - The operator is D + M with D the O(a)-improved Wilson operator
 *      D = 1/2 sum_mu {gamma_mu (nabla_mu + nabla*_mu) - nabla*_mu nabla_mu}
 *          + c_sw (i/4) sum_{mu,nu} sigma_mu_nu Fhat_mu_nu
 *    in the chiral basis (gamma5 = diag(1,1,-1,-1)), Fhat the clover-leaf
 *    field strength; fermions periodic in space, time boundary bc_t.
 *  - alpha is a table of T positive numbers used as S' = alpha(x0) S,
 *    eta' = alpha(x0) eta, so S = S'/alpha and C_PP = C'_PP / alpha^2.  This
 *    is the reciprocal of the function the paper factorises in eq. redeft.
 *  - The stopping rule (eq. stopping) is read as
 *      |eta' - (D'+M) S'|_2 <= r |eta'|_2   per right-hand side,
 *    checked on an FP64 recomputation of the residual.
 *
 * Ownership and errors
 * --------------------
 *  - Every function returns DP_OK (0) or a negative DP_ERR_* code and never
 *    throws; dp_last_error() gives a message for the last failure on a ctx.
 *  - Host buffers passed in are read (or written) before the call returns;
 *    the caller keeps ownership.  Device pointers (the *_dev variants) must be
 *    device memory of the ctx's GPU in the same host layout; the library
 *    enqueues its work on the given HIP stream (NULL: the ctx's own stream)
 *    and returns when the results are complete.
 *  - A ctx owns all device memory it allocates (gauge field, clover blocks,
 *    per-mass inverses, solver work space) until dp_destroy.
 *  - One host thread at a time per ctx.
 */
#ifndef DP_H
#define DP_H

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define DP_OK 0
#define DP_ERR_INVALID_ARG (-1)
#define DP_ERR_OOM (-2)
#define DP_ERR_DEVICE (-3)
#define DP_ERR_NOT_CONVERGED (-4)
#define DP_ERR_BREAKDOWN (-5)
#define DP_ERR_NONFINITE (-6)
#define DP_ERR_BAD_STATE (-7)
#define DP_ERR_FULL (-8) /* a batch has no free slot for the request */

/* inner precision of a solve */
#define DP_PREC_F64 0 /* FP64 throughout */
#define DP_PREC_F32 1 /* FP32 storage and arithmetic inside, FP64 outside */
#define DP_PREC_F16 2 /* FP16 storage with per-site scales, FP32 arithmetic inside */
#define DP_PREC_F32_SINGLE 3 /* one FP32 Krylov solve to r, no FP64 defect correction: the
                                single-precision solve whose residue floor the heavy-quark
                                section discusses (the FP64 residual is still recomputed
                                once, for dp_info.true_res) */

/* Krylov solver */
#define DP_SOLVER_BICGSTAB 0 /* van der Vorst 1992 */
#define DP_SOLVER_CGNR 1     /* CG on the normal equations of the Schur operator */

/* dp_apply flags */
#define DP_PRECOND 1     /* apply D' + M = alpha (D+M) alpha^-1 (else D + M) */
#define DP_DAGGER 2      /* apply the adjoint */
#define DP_HOP_ONLY 4    /* apply only the hopping term (no 4 + M, no clover) */
#define DP_APPLY_SCHUR 8 /* even-site Schur operator A_ee - H_eo A_oo^-1 H_oe on the
                            even part of the input; the odd part of the output is 0 */
#define DP_APPLY_F32 16  /* compute in the FP32 kernels (input rounded to FP32) */
#define DP_APPLY_F16 32  /* compute in the FP16-storage kernels */

typedef struct dp_ctx dp_ctx;
typedef struct dp_batch dp_batch;

typedef struct {
  double r;        /* target relative residual of the preconditioned system (> 0) */
  int solver;      /* DP_SOLVER_* */
  int precision;   /* DP_PREC_* (inner precision) */
  int max_iter;    /* cap on Krylov iterations per right-hand side (> 0) */
  double delta;    /* inner relative residual reduction per outer step (0: default
                      1e-5 for F32, 5e-3 for F16; ignored for F64) */
  int x0_src;      /* source timeslice: C_PP is indexed by t = (x0 - x0_src) mod T */
  int ncols_group; /* columns summed into one C_PP (e.g. 12 for a point source);
                      0 means every right-hand side gets its own C_PP */
} dp_params;

typedef struct {
  int status;        /* DP_OK, DP_ERR_NOT_CONVERGED, DP_ERR_NONFINITE ... */
  int iters;         /* Krylov iterations (BiCGStab steps or CG steps) */
  int outer;         /* FP64 residual recomputations (outer steps) */
  int hop_calls;     /* applications of the hop kernel (each one a parity) */
  int restarts;      /* BiCGStab breakdown restarts */
  double true_res;   /* FP64 |eta' - D'S'| / |eta'| of the returned solution */
  double seconds;    /* wall time of the solve (shared by a batch) */
  int fallback;      /* dp_solve*: 1 when the inner-precision solve of this column went
                        non-finite and the returned result is the FP64 solve's */
} dp_info;

/* Paper: eq. linsysunprec (the lattice on which D[U] + M acts) and, for the
 * time boundary, eq. redeftbc (antiperiodic fermions) and the closing remark
 * of the heavy-quark section (the Schroedinger functional's Dirichlet ends).
 * Create a context on GPU `device` for a lattice dims = {T, L1, L2, L3}
 * (all even, >= 2), time boundary bc_t = -1 (antiperiodic), +1 (periodic) or
 * 0 (Dirichlet: the fermion vanishes beyond the first and last timeslice, the
 * boundary of the Schroedinger functional with zero boundary fields; the
 * clover term is built from the given links as everywhere else).
 * The state starts with unit links, c_sw = 0, M = 0 and alpha = 1. */
int dp_create(const int dims[4], int bc_t, int device, dp_ctx** out);
void dp_destroy(dp_ctx* ctx);
const char* dp_last_error(const dp_ctx* ctx);

/* Paper: the gauge field U of D[U] in eq. linsysunprec.
 * Gauge links, host layout above (T*L1*L2*L3*4*9 complex).  Resets the clover
 * term to c_sw = 0 and drops cached per-mass inverses. */
int dp_set_gauge(dp_ctx* ctx, const double* U);
/* Same from device memory of the ctx's GPU. */
int dp_set_gauge_dev(dp_ctx* ctx, const void* U_dev, void* hip_stream);

/* Paper: the closing remark of the heavy-quark section (the Schroedinger
 * functional, where correlators decay over the whole time extent).
 * For a ctx created with bc_t = 0, whose T timeslices are the interior
 * 1 <= x0 <= T of a Schroedinger-functional lattice with boundaries at
 * x0 = 0 and x0 = T + 1: U_ext holds the links of the whole lattice, host
 * layout with T + 2 timeslices (index 0: the boundary x0 = 0, 1..T: the
 * interior, T + 1: the boundary x0 = T + 1).  The interior links become the
 * ctx's gauge field (as dp_set_gauge); the spatial links of the two
 * boundaries (the boundary gauge fields) and the time links between them
 * and the interior enter the clover term next to the boundaries, which
 * dp_set_clover builds from the whole lattice; the time links into the two
 * boundaries give the boundary sources of dp_sf_wall_sources.  ct_tilde is the coefficient
 * of the fermion boundary counterterm: (ct_tilde - 1) psi on the first and
 * last interior timeslices (1: none), in force from this call on.  The
 * fermion field vanishes on the boundaries (the hops into them drop).
 * DP_ERR_BAD_STATE on a ctx with bc_t != 0. */
int dp_set_gauge_sf(dp_ctx* ctx, const double* U_ext, double ct_tilde);

/* Paper: as dp_set_gauge_sf.
 * The boundary sources of the Schroedinger functional into eta_dev (device,
 * ncols full-lattice spinors, host layout), c = c0 + j for column j (e_c the
 * unit spin-colour vector).  side 0 (boundary x0 = 0): U_0(x0 = 0, xs)^+ P+
 * e_c on the first interior timeslice, P+ = (1 + gamma_0)/2; side 1
 * (boundary x0 = T + 1): U_0(x0 = T, xs) P- e_c on the last interior
 * timeslice, P- = (1 - gamma_0)/2; 0 elsewhere.  Each is the hop from the
 * boundary field e_c into the interior, moved to the right-hand side.
 * Needs dp_set_gauge_sf (else DP_ERR_BAD_STATE), side 0 or 1 and
 * 0 <= c0, c0 + ncols <= 12. */
int dp_sf_wall_sources(dp_ctx* ctx, int side, int c0, int ncols, void* eta_dev, void* hip_stream);

/* Paper: the O(a)-improved Wilson operator named at the start of the
 * heavy-quark section, with the coefficient c_sw of the Table 1 caption.
 * Clover term c_sw (i/4) sum sigma F from the resident links (built on the GPU;
 * with Schroedinger-functional links from the whole padded lattice, plus the
 * boundary counterterm). */
int dp_set_clover(dp_ctx* ctx, double csw);
/* A caller-supplied clover field, host layout [site][12][12]; it must be
 * Hermitian and commute with gamma5 (block diagonal in the two chiralities),
 * else DP_ERR_INVALID_ARG (and the term is set to zero).  It replaces the
 * whole term: with Schroedinger-functional links the boundary counterterm
 * is the caller's to include. */
int dp_set_clover_field(dp_ctx* ctx, const double* C);

/* Paper: the quark mass M of eq. linsysunprec (the hopping parameters of
 * Table 1 through M = 1/(2 kappa) - 4).
 * Bare mass M (operator D + M), or kappa with M = 1/(2 kappa) - 4. */
int dp_set_mass(dp_ctx* ctx, double M);
int dp_set_kappa(dp_ctx* ctx, double kappa);

/* Paper: the function of eq. redeft (heavy-quark section), e.g. the profile
 * of eq. pbcalpha; this table is its reciprocal (S' = alpha S).
 * Distance profile alpha(x0), T entries, each finite and > 0.  Read at every
 * later solve and dp_apply with DP_PRECOND; a copy is kept. */
int dp_set_alpha(dp_ctx* ctx, const double* alpha);

/* Spatial profiles of the light-quark factorisation (light-quark section,
 * eqs. redefa, betaa, redefcovs): S' = beta S, eta' = beta eta with
 * beta(y) = alpha(y0) a1(y1) a2(y2) a3(y3), alpha the time profile (the
 * ctx's, or a batch slot's own).  a1, a2, a3 hold L1, L2, L3 entries, each
 * finite and > 0; NULL means ones (all NULL: time-only, the default).  The
 * spatial hops then carry a_k(y_k)/a_k(y_k +- 1) (space stays periodic), and
 * the restoration S = S'/beta precedes the contraction of C_PP.  Applies to
 * every later solve, batch admission and dp_apply with DP_PRECOND on this ctx;
 * DP_ERR_BAD_STATE while a batch is open. */
int dp_set_alpha_space(dp_ctx* ctx, const double* a1, const double* a2, const double* a3);

/* Paper: eq. linsysunprec (D + M) and eq. linsysprec (D' + M, the modified
 * time derivatives of the heavy-quark section with the boundary rule eq.
 * redeftbc).
 * out = op(in) for one full-lattice spinor (host layout).  flags:
 * DP_PRECOND (alpha-preconditioned operator), DP_DAGGER (adjoint),
 * DP_HOP_ONLY (hopping term only) or DP_APPLY_SCHUR (even-odd Schur
 * operator), and DP_APPLY_F32 / DP_APPLY_F16 to run the inner-precision
 * kernels (for checking them; the result is returned in FP64).  The
 * operator uses the ctx's current gauge field, clover term, mass and alpha. */
int dp_apply(dp_ctx* ctx, const double* in, double* out, int flags);

/* Paper: as dp_apply (eqs. linsysunprec, linsysprec, redeftbc).
 * dp_apply on nrhs spinors in device memory (host layout, nrhs consecutive
 * full-lattice spinors, complex128): the same flags and operator, each
 * right-hand side a slot of the multi-RHS kernels (the links are read once per
 * launch for all of them).  in and out must not overlap.  Work already queued
 * on hip_stream (nullable) completes first; the call returns when out is
 * written.  The library's launch timing (dp_set_timing) covers these kernels,
 * which makes this the operator benchmark. */
int dp_apply_dev(dp_ctx* ctx, const void* in_dev, void* out_dev, int nrhs, int flags, void* hip_stream);

/* Paper: eq. linsysunprec solved through eqs. redeft and linsysprec, stopped
 * by eq. stopping (read as above), restored by eq. backcorrection (site by
 * site, then contracted to C_PP of the heavy-quark section).
 * Solve (D+M) S = eta for nrhs right-hand sides (host layout, nrhs spinors)
 * through the preconditioned system, to the residue p->r.
 *   S    : nullable; receives the nrhs restored solutions (host layout)
 *   cpp  : nullable; receives C_PP(t) = -sum_x tr[S^+ S], T doubles per group
 *          of p->ncols_group right-hand sides (or per right-hand side)
 *   info : nullable; nrhs entries
 * Returns DP_OK when every right-hand side met r, DP_ERR_NOT_CONVERGED when
 * one hit max_iter (S, cpp and info are still filled), or another error. */
int dp_solve(dp_ctx* ctx, const double* eta, int nrhs, const dp_params* p, double* S, double* cpp,
             dp_info* info);
/* Paper: as dp_solve.
 * Same with eta and S in device memory (host layout; they must not overlap,
 * else DP_ERR_INVALID_ARG); cpp and info on the host.
 * dp_solve and dp_solve_dev: a column whose FP32 / FP16 inner solve goes
 * non-finite is solved again in FP64 (info.fallback = 1); a BiCGStab
 * breakdown restarts the inner solve with a pseudo-random shadow residual,
 * and three breakdowns in a row without progress end the column with
 * DP_ERR_BREAKDOWN. */
int dp_solve_dev(dp_ctx* ctx, const void* eta_dev, int nrhs, const dp_params* p, void* S_dev, double* cpp,
                 dp_info* info, void* hip_stream);

/* Paper: the solver of the light-quark iteration counts (Table 1 and the
 * Schwarz-preconditioned GCR it cites), on the system of eqs. redefa, betaa.
 * SAP+GCR: the domain-decomposition solver of the paper's light-quark
 * iteration counts (Table 1; the Schwarz alternating procedure it cites) on
 * the preconditioned system with the ctx's mass, time profile and spatial
 * profiles.  The lattice is cut into blocks of extents block[mu], each
 * dividing its lattice extent an even number of times; one application of
 * the preconditioner runs ncy cycles over the two block colours, each block
 * solved by nmr minimal-residual steps with Dirichlet block boundaries in
 * `precision` (DP_PREC_F32 or DP_PREC_F64); flexible GCR in FP64 with restart
 * length nkv (1..64) runs until |eta' - D'S'| <= r |eta'| or max_iter
 * preconditioner applications (info.iters; info.outer = restarts). */
typedef struct {
  double r;
  int block[4];
  int ncy, nmr, nkv;
  int precision;
  int max_iter;
} dp_sap_params;
/* One right-hand side (host layout); S and cpp (T doubles) nullable. */
int dp_solve_sap(dp_ctx* ctx, const double* eta, const dp_sap_params* p, double* S, double* cpp, dp_info* info);
/* Paper: as dp_solve_sap (Table 1 and the solver it cites).
 * Same with eta and S in device memory (host layout, V x 12 complex doubles;
 * S nullable; they must not overlap, else DP_ERR_INVALID_ARG); cpp and info
 * on the host.  The library first waits for hip_stream (nullable), then works
 * on its own stream and returns when S and cpp are complete. */
int dp_solve_sap_dev(dp_ctx* ctx, const void* eta_dev, const dp_sap_params* p, void* S_dev, double* cpp,
                     dp_info* info, void* hip_stream);

/* Paper: the Schwarz preconditioner of the solver of Table 1 (the procedure
 * it cites), on the preconditioned operator D' of eqs. redefa, betaa.
 * One application psi = M r of the SAP preconditioner that dp_solve_sap uses
 * inside GCR: psi = 0, then ncy cycles over the two block colours, each
 * forming the block residual r - D' psi on the blocks of the colour and
 * running nmr minimal-residual steps of the Dirichlet block operator on it
 * (block sums in FP64).  r and psi: host layout, V x 12 complex doubles,
 * already in the preconditioned variables (no beta is applied).  Uses
 * p->block, ncy, nmr and precision (validated as for dp_solve_sap); r, nkv
 * and max_iter are ignored.  With FP32 block solves on blocks of at most
 * 1536 sites one kernel runs each colour pass (block solves in registers
 * and LDS; up to 256 sites a thread per site, above that up to three sites
 * per thread); larger blocks and FP64 launch the operator per
 * minimal-residual step.  Returns DP_ERR_INVALID_ARG / DP_ERR_BAD_STATE as
 * dp_solve_sap. */
int dp_sap_precondition(dp_ctx* ctx, const double* r, const dp_sap_params* p, double* psi);

/* Instrumentation (no passage of the paper: it reports no timings).
 * Per-kernel timing of the library's own launches.  dp_set_timing(ctx, 1)
 * clears the statistics and brackets every later kernel launch of the ctx
 * with HIP events on the stream it runs on; dp_get_timing copies up to `max`
 * entries (one per kernel variant, e.g. "hop_f32_diag") and sets *count to
 * the number available.  bytes and flops are algorithmic: each link, clover
 * block and input spinor counted once per launch, each output once. */
typedef struct {
  char name[32];
  long long launches;
  double ms;    /* summed event-to-event time */
  double bytes; /* summed algorithmic HBM bytes */
  double flops; /* summed algorithmic flops */
} dp_kernel_stat;
int dp_set_timing(dp_ctx* ctx, int enable);
int dp_get_timing(dp_ctx* ctx, dp_kernel_stat* out, int max, int* count);
/* The event-to-event duration in ms of each timed launch of the kernel variant
 * `name` (the first 65536 since dp_set_timing), in launch order: up to `max`
 * copied to ms, *count set to the number available (0 for an unknown name). */
int dp_get_timing_samples(dp_ctx* ctx, const char* name, float* ms, int max, int* count);

/* Paper: the point source of eq. linsysunprec (non-zero on one timeslice),
 * placed as in the correlator C_PP of the heavy-quark section (all 12
 * spin-colour components at one site).
 * Writes ncols unit point sources into eta_dev (device memory of the ctx's
 * GPU, ncols consecutive full-lattice spinors in host layout): column j is 1
 * in spin-colour component c0 + j (c = 3*spin + colour) at site = {x0, x1,
 * x2, x3} and 0 everywhere else.  Requires 0 <= c0, ncols >= 1, c0 + ncols
 * <= 12 and the site inside the lattice, else DP_ERR_INVALID_ARG.  Work queued
 * on hip_stream (nullable) completes first; returns when eta_dev is written.
 * The caller owns eta_dev. */
int dp_point_sources(dp_ctx* ctx, const int site[4], int c0, int ncols, void* eta_dev, void* hip_stream);

/* Paper: as dp_apply (eqs. linsysunprec, linsysprec, redeftbc), with the
 * mass of eq. linsysunprec and the profile of eq. redeft chosen per
 * right-hand side, as the slots of a batch carry them.
 * dp_apply_dev with a mass M[k] and a time profile alpha[k][0..T) for each
 * right-hand side k (each slot of the multi-RHS kernels its own A_oo^-1 and
 * hop ratios).  M NULL: the ctx's mass for every slot; alpha NULL: the ctx's
 * profile (used with DP_PRECOND only).  Every M[k] finite and every alpha
 * entry finite and > 0, else DP_ERR_INVALID_ARG.  A new mass allocates and
 * caches its inverse clover field. */
int dp_apply_dev_slots(dp_ctx* ctx, const void* in_dev, void* out_dev, int nrhs, int flags, const double* M,
                       const double* alpha, void* hip_stream);

/* For the callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * dp_apply_dev with the same arguments, flags and result, but every
 * temporary (the parity fields, their inner-precision copies, the per-slot
 * tables) lives in a static device array of DP_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends; the call
 * allocates nothing (no hipMalloc, hipFree or other allocating routine) and
 * records no launch timing.  Limits: 1 <= nrhs <= DP_NOALLOC_MAX_RHS, and the
 * temporaries must fit the array, else DP_ERR_INVALID_ARG with both sizes in
 * dp_last_error: per right-hand side 5 FP64 parity fields (V/2 * 192 bytes
 * each) for DP_APPLY_* in FP64, 4 FP64 and 5 inner-precision ones otherwise;
 * e.g. one 16^3x32 right-hand side in FP32 needs 82 MB, one 24^3x48 one
 * 414 MB (too large).  DP_APPLY_SCHUR uses the inverse clover of the ctx's
 * current mass, which an earlier dp_apply, dp_apply_dev or solve with that
 * mass must have built, else DP_ERR_BAD_STATE.  Every call on one GPU shares
 * that GPU's array and leaves its contents there: calls that overlap on one
 * GPU (several host threads, or contexts used concurrently) race and must be
 * serialised by the caller. */
#define DP_NOALLOC_SCRATCH_BYTES (128u << 20)
#define DP_NOALLOC_MAX_RHS 64
int dp_apply_dev_noalloc(dp_ctx* ctx, const void* in_dev, void* out_dev, int nrhs, int flags, void* hip_stream);

/* ------------------------------------------------------------------ batches
 * A batch is a fixed set of nslots slots on one ctx, each solving one
 * right-hand side with its own mass, alpha profile, residue and source
 * timeslice.  Requests enter (dp_batch_admit) and leave (dp_batch_harvest)
 * while others run: every dp_batch_step runs k Krylov iterations for all
 * running slots at once (the hop kernel shares the links among them), then
 * the FP64 outer step for the slots whose inner solve ended.  A slot's
 * arithmetic does not depend on the other slots, so a result is the same
 * alone and in any mix.  Several batches (one per ctx, e.g. one per resident
 * gauge field) may be driven from different host threads; their work
 * overlaps on the GPU (each ctx has its own stream).  While a batch is open
 * its ctx's links, clover and masses must not change (DP_ERR_BAD_STATE). */
typedef struct {
  long long tag;   /* the tag given at admission */
  int slot;        /* the slot that ran it */
  dp_info info;    /* info.seconds = admission to completion */
} dp_batch_result;

/* Paper: each slot solves eq. linsysprec for its own eq. redeft profile,
 * stopped by eq. stopping and restored by eq. backcorrection; the batching
 * itself is no part of the paper.  precision DP_PREC_F64, _F32, _F16 or
 * _F32_SINGLE, solver DP_SOLVER_*. */
int dp_batch_open(dp_ctx* ctx, int nslots, int precision, int solver, dp_batch** out);
void dp_batch_close(dp_batch* b);
/* Admit ncols right-hand sides (device memory, host layout, one after the
 * other), all with mass M, the T-entry profile alpha (NULL: the ctx's),
 * residue r, max_iter, inner reduction delta (0: default), source timeslice
 * x0_src and a caller tag.  S_dev (nullable, device, host layout, ncols
 * spinors) receives the restored solutions when they finish.  slots_out
 * (nullable) receives the ncols slot indices.  DP_ERR_FULL when fewer than
 * ncols slots are free.  The sources are read before the call returns. */
int dp_batch_admit(dp_batch* b, int ncols, const void* eta_dev, void* S_dev, double M, const double* alpha, double r,
                   int max_iter, double delta, int x0_src, long long tag, int* slots_out);
/* Run k inner iterations for the running slots and the outer steps that
 * follow; *ndone = results waiting to be harvested. */
int dp_batch_step(dp_batch* b, int k, int* ndone);
/* Move up to max finished results (completion order) to out, with their
 * C_PP (T doubles each, nullable) in cpp; their slots become free. */
int dp_batch_harvest(dp_batch* b, dp_batch_result* out, double* cpp, int max, int* count);
int dp_batch_status(const dp_batch* b, int* free_slots, int* running, int* done);
long long dp_batch_device_bytes(const dp_batch* b);

/* Admission gate of a server (no passage of the paper).
 * Device bytes a context would hold for the gauge field and clover of a
 * lattice, plus the solver work space for nrhs right-hand sides at the given
 * precision, plus one per-mass inverse per new mass. */
long long dp_footprint_bytes(const int dims[4], int nrhs, int precision, int new_masses);

#ifdef __cplusplus
}
#endif
#endif /* DP_H */
