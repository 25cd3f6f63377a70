/*
 * etc.h — C ABI of the MI355X (gfx950) effective-thermal-conductivity solver.
 *
 * Method (Ye, Fu and Chung, arXiv 2404.02433):
 *   - steady conduction -div(K grad p) = 0 on a voxel RVE with constant
 *     Dirichlet data p_in / p_out on the two faces normal to the load axis and
 *     zero flux on the other four (Section "Model problem");
 *   - Two-Point Flux-Approximation: one unknown per voxel, internal-face
 *     conductivity = harmonic mean of the two cells, Dirichlet faces 2 kappa
 *     (Section "Discretization scheme", eq:flux, eq:scaled bilinear forms);
 *   - preconditioned conjugate gradients (alg:pcg) with the exit test
 *     ||r||_2 / ||b||_2 <= rtol (eq:exit);
 *   - preconditioner = homogeneous reference medium (eq:refer bilinear forms)
 *     solved by DCTs along the two transverse axes and one tridiagonal solve
 *     per transverse mode along the load axis (alg:solve ref);
 *   - reference parameters from the family extrema of
 *     eq:parameters for linear programming (alg:refer parameters);
 *   - effective conductivity from the outflow-face flux
 *     (eq:effective formula dis).
 *
 * Conventions shared by every entry point:
 *   - Conductivity and solution arrays given by the caller are C-contiguous
 *     device arrays of shape n[0] x n[1] x n[2] (user layout).  `axis` names
 *     the load axis; the two other axes are the transverse ones.
 *   - Internally the plan keeps a canonical layout [k][a][b]: load axis k
 *     slowest, the two transverse axes after it in their user order, b
 *     contiguous.  Entry points marked "canonical" take vectors in that layout.
 *   - Voxel edges h_d = L[d] / n[d] (cubic voxels of edge 1 when L is all
 *     zeros); the scaled conductivity of a face normal to d is kappa / h_d^2.
 *   - Every call is enqueued on the plan's HIP stream.  Calls returning host
 *     values synchronise that stream.
 *   - A plan is not thread-safe; separate plans may run concurrently on
 *     separate streams.
 *   - Errors: every call returns an etc_status; nothing throws across the ABI.
 *     etc_last_error() gives a message for the last failure on this thread.
 */
#ifndef ETC_H
#define ETC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ETC_OK = 0,
  ETC_NOT_CONVERGED = 1,   /* warning: iteration cap reached; results stay readable */
  ETC_E_INVALID = -1,      /* bad argument or bad conductivity (<= 0, NaN, Inf)      */
  ETC_E_NOMEM = -2,        /* device allocation failed or caller workspace too small */
  ETC_E_HIP = -3,          /* a HIP runtime call failed                              */
  ETC_E_BREAKDOWN = -4,    /* w.Aw <= 0, r.z <= 0 or a non-finite scalar in PCG      */
  ETC_E_STATE = -5,        /* result requested before a successful etc_solve         */
  ETC_E_UNSUPPORTED = -6   /* a size beyond the kernels' limits                       */
} etc_status;

typedef enum { ETC_F64 = 0, ETC_F32 = 1 } etc_dtype;

/* ETC_FP64: every vector float64.  ETC_MIXED: iteration vectors and the
 * stencil/DCT arithmetic in float32, tridiagonal solves, dot products and
 * PCG scalars in float64, solution p in float64, and the residual replaced by
 * the float64 true residual b - A p every `refine_every` passes and before
 * convergence is accepted. */
typedef enum { ETC_FP64 = 0, ETC_MIXED = 1 } etc_precision;

/* Reference parameters: MID = sqrt(min * max) of each family (an optimum of
 * eq:linear programming); ONE = all 1 (the paper's "one"); USER = kref_user. */
typedef enum { ETC_KREF_MID = 0, ETC_KREF_ONE = 1, ETC_KREF_USER = 2 } etc_kref_mode;

/* Preconditioner: DCT = the reference-medium solve of alg:solve ref;
 * NONE = plain CG (z = r), for the comparison behind prop:cond. */
typedef enum { ETC_PC_DCT = 0, ETC_PC_NONE = 1 } etc_precond;

/* Dirichlet pair on the faces normal to the load axis (p_in at index 0). */
typedef struct {
  double p_in, p_out;
} etc_bc;

typedef struct {
  etc_precision precision;
  etc_kref_mode kref_mode;
  double kref_user[5];   /* order: load-axis faces, a faces, b faces, in layer, out layer */
  double rtol;           /* default 1e-6 */
  int max_iter;          /* default 1000 */
  int refine_every;      /* mixed form: true-residual period, default 20 */
  int poll_every;        /* passes enqueued between host checks, default 8 */
  void* stream;          /* hipStream_t; NULL = the null stream */
  double L[3];           /* domain length per user axis; all 0 = voxel edge 1 */
  void* workspace;       /* optional caller-owned device memory (>= etc_workspace_size) */
  size_t workspace_bytes;
  int want_grad;         /* 1: reserve the adjoint state for etc_grad (8 bytes per voxel) */
  etc_precond precond;   /* default ETC_PC_DCT */
  int autotune;          /* 1: etc_setup times the stencil's plane chunk and the
                            tridiagonal kernel's block shape and grid on the plan's
                            own buffers and keeps the fastest (cached per problem
                            shape); default 0 */
  int use_graph;         /* 1: etc_solve captures `poll_every` passes in a HIP graph on
                            first use (per solution buffer and Dirichlet pair) and
                            replays it; ignored while a kernel timer is set.  The
                            results equal those of the eager path.  Default 0. */
  int thomas_modes;      /* tridiagonal block shape: transverse modes per block and */
  int thomas_parts;      /* partitions per line, both 0 (default) for the built-in
                            choice by load-axis length; compiled shapes (float32 /
                            float64 rows): 32x8, 16x16, 32x16 and 32x32 / 16x32, plus
                            64x8 (float32).  32x8 holds load axes up to 128 (and
                            exactly 160 and 256), 16x16 and 32x16 up to 256 (32x16
                            also exactly 512), the
                            32-partition shapes up to 2048 (512 in the mixed form);
                            etc_setup returns ETC_E_UNSUPPORTED for a shape that is
                            not compiled or does not hold the load axis.  With
                            autotune the tuner keeps this shape and times its grid. */
} etc_options;

typedef struct {
  int iters;             /* PCG passes (products A w) */
  int status;            /* etc_status of the solve */
  double relres;         /* last relative residual (true residual in the mixed form) */
  double kref[5];        /* reference parameters used (order as kref_user) */
  double lambda_lo, lambda_hi; /* Lambda', Lambda'' of lem:cond for these parameters */
} etc_result;

typedef struct etc_plan etc_plan;

/* General problem data (Section "Model problem" allows K = diag(kappa^x,
 * kappa^y, kappa^z) per voxel; tab:smooth adds a volume source and Dirichlet
 * data that vary over the faces).  All pointers are device memory in the
 * user layout and are borrowed for the duration of etc_setup_ex only.
 *   kappa[0..2] : conductivity along user axes 0, 1, 2 (dtype of the call).
 *                 kappa[1] = kappa[2] = NULL means isotropic kappa[0].
 *   source      : float64 volume source f per voxel, or NULL (no source).
 *   p_in_face   : float64 Dirichlet value per face of the first load layer,
 *                 an array over the two transverse axes in user order, or
 *                 NULL (constant bc.p_in); p_out_face likewise (bc.p_out). */
typedef struct {
  const void* kappa[3];
  const double* source;
  const double* p_in_face;
  const double* p_out_face;
} etc_problem;

/* Fill `opt` with the defaults listed above. */
void etc_options_default(etc_options* opt);

/* Device bytes a plan for this size, input dtype and options needs.  Same
 * argument rules as etc_setup.  Returns ETC_E_INVALID on bad sizes. */
etc_status etc_workspace_size(const int64_t n[3], etc_dtype dt, int axis, const etc_options* opt, size_t* bytes);

/* Preparation phase (the paper separates preparation from execution, Section
 * "Performance tests of different implementations"): validates the arguments,
 * copies `kappa` (device, user layout, dtype `dt`) into the canonical layout,
 * checks every conductivity is finite and > 0, computes the family extrema and
 * the reference parameters, and builds the DCT twiddle tables.
 *   kappa : borrowed for the duration of the call only.
 *   n     : user dims; each >= 1 and <= 2^20, n[axis] >= 2.  Beyond the
 *           kernels' limits ETC_E_UNSUPPORTED: load axis n[axis] <= 2048 (the
 *           tridiagonal kernel holds a line as 32 partitions of at most 64
 *           rows; 512, partitions of at most 16 rows, in the mixed form),
 *           first transverse axis <= 65535, transverse plane < 2^31 voxels.
 *   bc    : p_in != p_out (eq:effective formula needs a drop).
 *   opt   : may be NULL (defaults).  If opt->workspace is NULL the plan
 *           allocates its device memory with hipMalloc and frees it in
 *           etc_destroy; otherwise it carves the caller's buffer (caller keeps
 *           ownership and must keep it alive until etc_destroy).
 *   plan  : receives the new plan (NULL on failure). */
etc_status etc_setup(const void* kappa, etc_dtype dt, const int64_t n[3], etc_bc bc, int axis,
                     const etc_options* opt, etc_plan** plan);

/* etc_setup for general problem data (see etc_problem); the isotropic,
 * source-free, constant-Dirichlet case is etc_setup.  With face data or a
 * source, etc_keff still reports the boundary flux sums scaled by
 * nL / (na nb (bc.p_in - bc.p_out)). */
etc_status etc_setup_ex(const etc_problem* problem, etc_dtype dt, const int64_t n[3], etc_bc bc, int axis,
                        const etc_options* opt, etc_plan** plan);

/* Workspace bytes for etc_setup_ex with this problem shape (only which
 * pointers are NULL matters). */
etc_status etc_workspace_size_ex(const etc_problem* problem, const int64_t n[3], etc_dtype dt, int axis,
                                 const etc_options* opt, size_t* bytes);

/* A batch of `nbatch` independent RVEs of one size: `kappa` holds nbatch
 * user-layout arrays back to back (nbatch x n[0] x n[1] x n[2]), isotropic,
 * one Dirichlet pair for all.  One plan stacks them along the load axis;
 * every kernel of a pass covers the whole batch in one launch, and each
 * instance keeps its own reference medium, PCG scalars, exit test and
 * convergence flag (an instance that has converged is skipped by every later
 * kernel of the solve).  etc_solve runs until every instance is done; solution
 * and gradient buffers are batch-shaped like kappa. */
etc_status etc_setup_batch(const void* kappa, etc_dtype dt, const int64_t n[3], int nbatch, etc_bc bc, int axis,
                           const etc_options* opt, etc_plan** plan);
etc_status etc_workspace_size_batch(const int64_t n[3], int nbatch, etc_dtype dt, int axis, const etc_options* opt,
                                    size_t* bytes);

/* A mixed-size ensemble: `count` independent isotropic RVEs, RVE i a
 * C-contiguous device array kappa[i] (user layout, dtype dt) of dims
 * dims[3i..3i+2], one load axis and one Dirichlet pair for all (Section
 * "Remarks on implementations": the transforms and tridiagonal systems of
 * many problems are batched).  RVEs of one shape form a group (at most 8
 * distinct shapes; load axes up to 512 voxels); every kernel of a PCG pass is
 * ONE launch for the whole ensemble, whose blocks pick their group and run
 * the kernel variant that group's size has, and every RVE keeps its own
 * reference medium, PCG scalars, exit test and convergence flag (converged
 * RVEs are skipped by every later kernel).  With opt->use_graph the passes
 * between host polls are replayed from one captured graph.
 *   kappa : count device pointers, borrowed for the duration of the call.
 *   opt   : as etc_setup; opt->workspace, when given, must hold
 *           etc_workspace_size_ensemble bytes.
 * After etc_solve (p0 must be NULL), etc_batch_results and etc_keff_batch
 * report per RVE in input order; etc_get_solution and etc_grad write the RVEs
 * back to back in input order (sum of their voxel counts, float64, user
 * layout); etc_residual_history reports RVE 0.  etc_keff, etc_apply_A,
 * etc_apply_Minv, etc_set_kernel_timer and etc_launch_info reject an
 * ensemble plan (ETC_E_INVALID). */
etc_status etc_setup_ensemble(const void* const* kappa, const int64_t* dims, int count, etc_dtype dt, etc_bc bc,
                              int axis, const etc_options* opt, etc_plan** plan);
etc_status etc_workspace_size_ensemble(const int64_t* dims, int count, etc_dtype dt, int axis, const etc_options* opt,
                                       size_t* bytes);

/* Per-instance passes, status and last relative residual of the last solve
 * (host arrays of nbatch entries; any may be NULL). */
etc_status etc_batch_results(const etc_plan* plan, int* iters, int* status, double* relres);

/* Per-instance K_out and K_in (host arrays of nbatch entries, k_in nullable). */
etc_status etc_keff_batch(etc_plan* plan, double* k_out, double* k_in);

/* Execution phase: PCG of alg:pcg from p0 (device, user layout, float64;
 * NULL = zero) until ||r|| / ||b|| <= rtol or max_iter passes.  Returns
 * ETC_OK, ETC_NOT_CONVERGED (results still readable) or an error.  `res` may
 * be NULL; for a batch it describes instance 0 and the status is the worst
 * over the batch.  Synchronises the plan's stream. */
etc_status etc_solve(etc_plan* plan, const double* p0, etc_result* res);

/* Effective conductivity along the load axis after etc_solve (host doubles):
 *   k_out    : eq:effective formula dis (outflow-face flux);
 *   k_in     : same with the inflow faces (nullable);
 *   k_energy : from the discrete dissipation (nullable; one extra pass).
 * ETC_E_STATE before a solve. */
etc_status etc_keff(etc_plan* plan, double* k_out, double* k_in, double* k_energy);

/* Gradient dK_out/dkappa for every voxel after etc_solve, by the adjoint
 * method: K_out depends on kappa directly and through p, and A p = b.  The
 * adjoint state lambda solves A lambda = dK_out/dp, which is the primal system
 * with Dirichlet pair (0, 1) scaled by nL / (na nb (p_in - p_out) fL); it is
 * solved by a second PCG with the same plan, rtol and preconditioner.  Then
 * dK/dkappa_v = dK/dkappa_v|_p - lambda . (dA/dkappa_v p - db/dkappa_v), a
 * sum over the faces of voxel v of the face-coefficient derivative times the
 * primal and adjoint jumps (harmonic-mean faces, eq:scaled bilinear forms),
 * plus the Dirichlet-face terms.
 *   dk_dkappa : device, user layout, float64, caller-owned.
 * Needs a plan made with want_grad = 1 (else ETC_E_STATE); isotropic kappa with
 * constant Dirichlet data only (else etc_setup_ex returns ETC_E_UNSUPPORTED
 * when want_grad is set).  Synchronises. */
etc_status etc_grad(etc_plan* plan, double* dk_dkappa);

/* etc_grad with the gradient written as `out_dt` (ETC_F64 or ETC_F32, e.g.
 * the dtype kappa was given in): the same float64 arithmetic, rounded once
 * on the store.  ETC_E_INVALID for another dtype. */
etc_status etc_grad_as(etc_plan* plan, void* dk_dkappa, etc_dtype out_dt);

/* Copy the solution p into `p` (device, user layout, float64, caller-owned). */
etc_status etc_get_solution(const etc_plan* plan, double* p);

/* Relative-residual history of the last solve: hist[0] = 1 (p0 = 0) up to
 * hist[iters]; copies min(cap, iters + 1) values to host memory. */
etc_status etc_residual_history(const etc_plan* plan, double* hist, int cap, int* count);

/* Canonical-layout building blocks of one PCG pass, for callers that drive
 * their own iteration.  Vectors are device arrays of V = n[0] n[1] n[2]
 * elements in the plan's storage dtype (float64 for ETC_FP64, float32 for
 * ETC_MIXED).
 *   etc_apply_A    : y = A x (eq:scaled bilinear forms); *xAx = x . y if non-NULL.
 *   etc_apply_Minv : z = A_ref^{-1} r by alg:solve ref; *rz = r . z if non-NULL.
 * Both synchronise when a dot is requested.  x/y and r/z must not alias. */
etc_status etc_apply_A(etc_plan* plan, const void* x, void* y, double* xAx);
etc_status etc_apply_Minv(etc_plan* plan, const void* r, void* z, double* rz);

/* Per-kernel timing with HIP events recorded around every launch of one hot
 * kernel on the plan's stream during etc_solve.  kernel_id: 0 off,
 * 1 operator, 2 residual update + forward row DCT, 3 forward column DCT,
 * 4 tridiagonal solve, 5 backward column DCT, 6 backward row DCT + solution
 * and direction updates.
 * etc_kernel_time returns the summed milliseconds and launch count of the
 * last solve. */
etc_status etc_set_kernel_timer(etc_plan* plan, int kernel_id);
etc_status etc_kernel_time(const etc_plan* plan, double* total_ms, int* launches);

/* Launch shapes of a plan: the stencil's plane chunk, the tridiagonal
 * kernel's persistent blocks per instance and its block shape (transverse
 * modes times partitions of each line), and whether the autotuner chose
 * them.  Any output pointer may be NULL. */
etc_status etc_launch_info(const etc_plan* plan, int* kchunk, int* thomas_blocks, int* tuned, int* thomas_modes,
                           int* thomas_parts);

/* Device-to-device copy of n doubles by a plain streaming kernel (16-byte
 * accesses): calibrates hardware byte counters and measures the streaming
 * ceiling.  src and dst must be 16-byte aligned (else ETC_E_INVALID); the
 * copy is enqueued on `stream` (hipStream_t, NULL = null stream). */
etc_status etc_copy_f64(const double* src, double* dst, int64_t n, void* stream);

void etc_destroy(etc_plan* plan);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): etc_setup,
 * etc_solve, etc_keff and (if p is non-NULL) etc_get_solution in one call,
 * for one isotropic RVE, with every device buffer of the plan carved from a
 * static device array of ETC_STATIC_SCRATCH_BYTES bytes that the library
 * holds on each GPU it runs on until the process ends (48 MiB: room for
 * 96^3 voxels in the float64 form, about 104^3 in the mixed form).  It calls
 * no hipMalloc, hipHostMalloc, hipFree or other device or pinned-memory
 * allocation; host bookkeeping uses the C++ heap.  The state mirror read
 * every few passes lives in pageable host memory.
 *   kappa, dt, n, bc, axis : as etc_setup (kappa borrowed for the call).
 *   opt   : as etc_setup, or NULL; workspace must be NULL and autotune,
 *           use_graph and want_grad 0 (else ETC_E_INVALID).
 *   p     : device, user layout, float64, caller-owned, or NULL.
 *   k_out : host, K_out of eq:effective formula dis; k_in nullable (host).
 *   res   : as etc_solve, nullable.
 * Returns ETC_E_UNSUPPORTED (and touches nothing) when etc_workspace_size for
 * these arguments exceeds ETC_STATIC_SCRATCH_BYTES; otherwise what the calls
 * it stands for return.  Every call on one GPU shares that GPU's array and
 * overwrites it (setup rebuilds every buffer it reads, so the contents a
 * previous call left do not matter): calls that overlap on one GPU, from
 * several threads or streams, race and must be serialised by the caller.
 * Synchronises the stream given in opt. */
#define ETC_STATIC_SCRATCH_BYTES (48u << 20)
etc_status etc_solve_static(const void* kappa, etc_dtype dt, const int64_t n[3], etc_bc bc, int axis,
                            const etc_options* opt, double* p, double* k_out, double* k_in, etc_result* res);

/* Message of the last failed call on the calling thread ("" if none). */
const char* etc_last_error(void);

/* Library version string. */
const char* etc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ETC_H */
