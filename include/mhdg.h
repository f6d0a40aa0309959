/*
 * mhdg.h -- C ABI of the MI355X macro-element HDG local-problem library.
 *
 * The library implements the data-parallel hot path of the macro-element
 * hybridized DG method for steady advection-diffusion in 2D
 *   div(a u + kappa q) = f,  q = -grad u  in Omega,  u = g_D on dOmega
 * (paper section 2.1, eqs. C21/C22) on triangular macro-elements K, each
 * uniformly subdivided into 4^r triangles carrying continuous piecewise-P_p
 * q and u (section 3.2), coupled only through the trace lambda on macro faces
 * with the LDG-H flux a lambda + kappa q + tau (u - lambda) n (section 3.1).
 *
 *   factor_local            assemble A_K and LU-factor it in place
 *                           (section 3.3.2, remark on the in-place LU)
 *   apply_trace_operator    S lambda = D lambda - sum_K C_K A_K^-1 B_K lambda_K,
 *                           steps 1-4 of the matrix-free algorithm, optionally
 *                           left-preconditioned by D^-1 (section 6.1)
 *   solve                   GMRES on the global problem (eq. global_problem)
 *   recover_local           A_K U_K = R_K - B_K lambda_K (eq. local_problem)
 *                           plus the transmission residual C U + D lambda
 *
 * Variants of the same operator: several trace vectors per call
 * (mhdg_apply_trace_operator_many), folded per-macro operators
 * (mhdg_fold_operator), the flux eliminated through the reference mass
 * (MHDG_QELIM), FP32/BF16 factors with FP64 refinement, coefficient
 * instances, SUPG inside the macros (mhdg_set_supg, section 3.4), the
 * adjoint (mhdg_adjoint) and the macro conservation residual
 * (mhdg_flux_balance).
 *
 * Conventions (the same written specification is implemented independently
 * by the CPU oracle used in the tests):
 *   - macro lattice node (i, j), i + j <= P = 2^r p, sits at
 *     X0 + (i/P)(X1 - X0) + (j/P)(X2 - X0), node index j(P+1) - j(j-1)/2 + i;
 *     Q = (P+1)(P+2)/2 nodes; local unknowns U_K = [q_x(Q), q_y(Q), u(Q)],
 *     N_K = 3Q;
 *   - faces are the unique macro edges sorted by (low vertex id, high vertex
 *     id); a face's level is the max of its macros' levels and it carries
 *     n_F = 2^{r_F} p + 1 trace nodes at A + t/(n_F-1) (B - A), A the
 *     lower-id vertex;
 *   - the global trace vector (length n_trace) lists interior faces in that
 *     order; boundary faces are Dirichlet and are eliminated;
 *   - f is given at the macro lattice nodes (macro-contiguous, n_nodes
 *     values): its interpolant in W(K) is the load;
 *   - g_D is given at p+2 Gauss-Legendre points on each of the 2^{r_F}
 *     segments of every boundary face (faces in sorted order, segments and
 *     points in increasing t): the Dirichlet trace is its L2 projection onto
 *     M(F) (section 2.3) by that quadrature;
 *   - local solutions U are returned macro-contiguous (n_local values);
 *   - coefficient instances (mhdg_set_instances): a handle may carry n_inst
 *     copies of the mesh that differ only in kappa and a.  Every count in
 *     mhdg_sizes is then the total over the copies, every vector argument
 *     is instance-major (instance i's block starts at i * count / n_inst),
 *     and each kernel launch covers all instances at once.
 *
 * Memory and ownership: the caller owns every pointer.  Device memory for
 * factors and scratch comes from caller workspaces sized by mhdg_query();
 * the handle keeps pointers into the factor workspace from factor_local
 * until the next factor_local or mhdg_destroy.  The handle itself owns only
 * host metadata.  Device pointers are plain device addresses (for example
 * from a torch tensor); "stream" is a hipStream_t passed as void*
 * (NULL = the null stream).  Calls are asynchronous on that stream, except
 * setup (host only), factor_local (synchronises to check kappa and the pivots) and
 * solve (synchronises each iteration to run the Arnoldi recurrences).
 *
 * Errors: every call returns an mhdg_status; nothing throws across the ABI.
 * mhdg_last_error() gives a message for the last failing call on a handle.
 * Handles are not thread-safe: one thread at a time per handle; distinct
 * handles may be driven from different threads on different streams.
 */
#ifndef MHDG_H_
#define MHDG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MHDG_OK = 0,
  MHDG_ERR_INVALID_ARG = 1,   /* NULL pointer, size out of range, bad option  */
  MHDG_ERR_MESH = 2,          /* clockwise/degenerate triangle, bad connectivity */
  MHDG_ERR_SINGULAR = 3,      /* an exactly zero pivot in some A_K            */
  MHDG_ERR_NOT_CONVERGED = 4, /* GMRES hit max_iter before rtol               */
  MHDG_ERR_WORKSPACE = 5,     /* workspace smaller than mhdg_query reports    */
  MHDG_ERR_HIP = 6,           /* a HIP runtime call failed                    */
  MHDG_ERR_STATE = 7,         /* e.g. apply before factor_local               */
  MHDG_ERR_NONFINITE = 8      /* a non-finite pivot in some A_K (an entry
                                 overflowed; macro and column in last_error)  */
} mhdg_status;

typedef enum {
  MHDG_FP64 = 0,              /* FP64 factors (the plain form)                 */
  MHDG_FP32 = 1,              /* FP32 factors on MFMA, FP64 refinement         */
  MHDG_BF16 = 2,              /* FP32 LU on MFMA rounded to BF16 for storage
                                 (a quarter of the FP64 bytes per apply; N_K
                                 <= 1024), FP64 refinement                    */
  MHDG_QELIM = 3              /* FP64 with the flux eliminated exactly: the
                                 macro mass matrix is |det J| times the
                                 reference one (section 3.2 spaces on an
                                 affine macro), so the first two block rows of
                                 A_K (section 3.3.1) give q = M^-1 (x_q + E u)
                                 and u solves the Q x Q Schur block
                                 S_u = K + kappa sum_d (E^d)^T M^-1 E^d, which
                                 is the only per-macro factor (LU with partial
                                 pivoting, Q = N_K / 3).  Same discrete
                                 operator as MHDG_FP64 up to rounding; apply,
                                 rhs, recover, local solve, solve and
                                 mhdg_fold_operator supported; no transposed
                                 solves, adjoint or autotuning; Q <= 1237     */
} mhdg_precision;

/* flags for apply_trace_operator / local_solve */
enum {
  MHDG_PRECONDITION = 1,      /* return D^-1 S lambda instead of S lambda      */
  MHDG_TRANSPOSE = 2,         /* use A_K^-T (adjoint solves)                   */
  MHDG_GRAPH = 4,             /* apply: replay a hipGraph of the launches (one
                                 per size class for all instances, then the
                                 face combine), captured on first use for this
                                 (lam, out, flags) and kept until the next
                                 factor_local or set_instances              */
  MHDG_FOLDED = 8,            /* apply: steps 1-3 with the folded operators
                                 T_K of mhdg_fold_operator (T_K^T with
                                 MHDG_TRANSPOSE)                              */
  MHDG_ASSEMBLED = 16,        /* apply: the assembled matrix S of
                                 mhdg_assemble_trace_matrix (its stored
                                 D^-1 S with PRECONDITION; no TRANSPOSE)     */
  MHDG_BOUNDARY = 32          /* apply: steps 1-3 through the boundary blocks
                                 W_K of mhdg_condense_boundary (W_K^T with
                                 MHDG_TRANSPOSE); excludes FOLDED, ASSEMBLED */
};

/* GMRES drivers (mhdg_solve_opts.driver) and stopping norms (.stop_norm) */
enum {
  MHDG_DRIVER_DEVICE = 0,     /* the Arnoldi recurrences, rotations and the
                                 least-squares solve run on the device; the
                                 host waits once per restart cycle (restart
                                 <= 2048, delayed reorthogonalisation)       */
  MHDG_DRIVER_HOST = 1        /* the host runs them and synchronises once per
                                 iteration                                   */
};
enum {
  MHDG_NORM_PRECONDITIONED = 0,  /* stop when ||D^-1 r|| <= rtol ||D^-1 f^||  */
  MHDG_NORM_TRUE = 1             /* stop when ||r|| <= rtol ||f^|| (FP64 or
                                    QELIM factors, device driver)            */
};

typedef struct mhdg_mesh mhdg_mesh;

typedef struct {
  int64_t n_macro;            /* macro-elements                               */
  int64_t n_faces;            /* all macro faces                              */
  int64_t n_interior_faces;
  int64_t n_trace;            /* global unknowns: sum of n_F, interior faces   */
  int64_t n_nodes;            /* sum over macros of Q                          */
  int64_t n_local;            /* sum over macros of N_K = 3Q                   */
  int64_t n_bnd_points;       /* Dirichlet sampling points                     */
  int32_t p;
  int32_t max_level;
  int64_t max_local;          /* max N_K                                       */
  size_t factor_ws_bytes;     /* workspace for factor_local at this precision  */
  size_t solve_ws_bytes;      /* workspace for solve at this restart length    */
  int32_t n_instances;        /* coefficient instances (mhdg_set_instances)    */
  size_t fold_ws_bytes;       /* workspace for mhdg_fold_operator              */
} mhdg_sizes;

typedef struct {
  double rtol;                /* stop when ||D^-1 r|| <= rtol ||D^-1 f^||
                                 (or ||r|| <= rtol ||f^||, see stop_norm)     */
  int32_t restart;            /* Krylov length per cycle (>= 1)                */
  int32_t max_iter;           /* total (inner) GMRES iterations                */
  int32_t zero_guess;         /* 1: start from lambda = 0; 0: use lam on entry */
  int32_t max_outer;          /* reduced-precision factors: refinement steps (0: 30) */
  double inner_rtol;          /* reduced-precision factors: inner GMRES relative
                                 tolerance per refinement step (0: 1e-5)      */
  int32_t graph;              /* device driver: 1 replays each restart cycle
                                 from hipGraphs captured on first use (per
                                 vectors, restart and flags; kept until the
                                 next factor_local); host driver: 1 replays
                                 every apply from one hipGraph (MHDG_GRAPH);
                                 0: plain launches                           */
  int32_t folded;             /* 1: GMRES applies (forward in solve, transposed
                                 in adjoint) use the folded operators
                                 (MHDG_FOLDED; needs mhdg_fold_operator)      */
  int32_t classic_gs;         /* 0: Arnoldi with delayed reorthogonalisation
                                 (one synchronisation and two passes over the
                                 basis per iteration); 1: classical
                                 Gram-Schmidt, second pass when the first
                                 keeps less than 1/sqrt(2) of the norm
                                 (host driver)                               */
  int32_t driver;             /* MHDG_DRIVER_DEVICE (default) or _HOST; the
                                 device driver falls back to the host one for
                                 classic_gs = 1 or restart > 2048             */
  int32_t stop_norm;          /* MHDG_NORM_PRECONDITIONED (default) or
                                 MHDG_NORM_TRUE                              */
  int32_t assembled;          /* 1: GMRES applies use the assembled matrix
                                 (MHDG_ASSEMBLED; needs
                                 mhdg_assemble_trace_matrix)                 */
  int32_t boundary;           /* 1: GMRES applies (solve and adjoint) use the
                                 boundary-condensed blocks (MHDG_BOUNDARY;
                                 needs mhdg_condense_boundary)               */
} mhdg_solve_opts;

typedef struct {
  int32_t iterations;         /* GMRES iterations (all inner solves)           */
  int32_t status;             /* mhdg_status of the solve                      */
  double rel_res_prec;        /* final ||D^-1 (f^ - S lam)|| / ||D^-1 f^||; with
                                 reduced-precision factors the FP64 residual of
                                 the whole system condensed onto the trace     */
  double rel_res_true;        /* final ||f^ - S lam|| / ||f^|| (FP64 factors;
                                 -1 with reduced-precision factors)            */
  double t_rhs_ms, t_gmres_ms;
  int32_t n_applies;          /* operator applies + per-macro solve passes this
                                 instance took part in                         */
  int32_t outer_iterations;   /* refinement steps (reduced-precision factors)  */
  int32_t reorth_passes;      /* second Gram-Schmidt passes taken (the second
                                 pass runs only when the first leaves less
                                 than 1/sqrt(2) of the vector's norm)        */
  int32_t cycles;             /* GMRES restart cycles run                      */
  int32_t host_waits;         /* times the host waited for the stream inside
                                 GMRES.  Device driver: once per cycle, once
                                 for the first cycle start and, with
                                 MHDG_NORM_TRUE, once for ||f^||; cycles of
                                 more than 64 columns run without graphs also
                                 wait once per 32 columns (two chunks stay
                                 queued), to skip what is left of a cycle
                                 once every instance has converged          */
} mhdg_solve_info;

/* Build the host-side macro mesh (the partition of Omega into simplicial
 * macro-elements of section 2.2, each uniformly subdivided r times as in
 * section 3.2, with the face trace spaces M(F) of section 3.2 and the finer
 * level on non-matching faces as in the local refinement of section 4.2):
 * faces, levels, orientation, numbering and the reference templates.
 * xy[n_vertices][2] (host, f64), tri[n_macro][3]
 * (host, i32, counter-clockwise), level[n_macro] (host, i32, 0..5; NULL means
 * every macro has level `uniform_level`), p in 1..4, local size
 * N_K = 3 (2^r p + 1)(2^r p + 2)/2 <= 4096.
 * Errors: INVALID_ARG (NULL, p, level or N_K out of range, vertex id out of range),
 * MESH (clockwise/degenerate triangle, an edge shared by more than 2 macros).
 * On error *out is NULL. */
mhdg_status mhdg_setup_macro_mesh(int64_t n_vertices, const double* xy, int64_t n_macro,
                                  const int32_t* tri, const int32_t* level, int32_t uniform_level,
                                  int32_t p, mhdg_mesh** out);

/* Batch n_inst coefficient instances (kappa, a) of the mesh in one handle
 * (the many-coefficient workloads of the method's parameter studies, where
 * every instance is the same discretisation with other data): the handle
 * then describes n_inst disjoint copies of the mesh, instance-major, and
 * apply/rhs/recover/solve process all of them in one launch per size class.
 * GMRES keeps one Krylov space per instance and masks converged instances
 * out of later applies.  Resets the factor state (call factor_local after).
 * n_inst >= 1 with n_inst * n_macro <= 2^28 and n_inst * n_trace < 2^31.
 * Errors: INVALID_ARG. */
mhdg_status mhdg_set_instances(mhdg_mesh* mesh, int32_t n_inst);

/* Sizes and workspace requirements for a precision and GMRES restart length. */
mhdg_status mhdg_query(const mhdg_mesh* mesh, int32_t precision, int32_t restart, mhdg_sizes* out);

/* Host copies of the sampling points: node_xy[n_nodes][2] (macro lattice
 * nodes, where f is sampled) and bnd_xy[n_bnd_points][2] (Dirichlet points).
 * Either pointer may be NULL. */
mhdg_status mhdg_sample_points(const mhdg_mesh* mesh, double* node_xy, double* bnd_xy);

/* Assemble every A_K (section 3.2 forms: blocks [[M,0,-E^x],[0,M,-E^y],
 * [kappa H^x, kappa H^y, K]]) and factor it in place with partial row
 * pivoting (ties to the smallest row), in the requested precision (BF16:
 * the FP32 factors are rounded to nearest-even BF16 for storage; the
 * refinement of solve and recover_local restores FP64 accuracy).
 * kappa: device f64[n_macro], each value finite and > 0: the values are
 * checked on the device before anything is assembled (one synchronisation)
 * and a violation returns INVALID_ARG naming the first such macro, with no
 * block assembled or factored.  a = (beta_x, beta_y) constant and finite;
 * tau finite and > 0 (both checked on the host, INVALID_ARG).  Entries that
 * still overflow (e.g. kappa or a near the largest double) make a pivot
 * non-finite: NONFINITE, with the macro and column in last_error.
 * ws: device workspace of at least factor_ws_bytes (mhdg_query with the
 * same precision); it must stay allocated while the handle uses it.
 * Synchronises (the kappa check and the pivot status).
 * Errors: INVALID_ARG, WORKSPACE, SINGULAR (an exactly zero pivot; first
 * macro and column in last_error), NONFINITE, HIP. */
mhdg_status mhdg_factor_local(mhdg_mesh* mesh, const double* kappa, double beta_x, double beta_y,
                              double tau, int32_t precision, void* ws, size_t ws_bytes,
                              void* stream);

/* factor_local with one advection vector per coefficient instance:
 * kappa device f64[n_inst * n_macro_per_instance] (instance-major), beta
 * host f64[n_inst][2].  mhdg_factor_local gives every instance the same a.
 * Errors as mhdg_factor_local. */
mhdg_status mhdg_factor_local_batched(mhdg_mesh* mesh, const double* kappa, const double* beta,
                                      double tau, int32_t precision, void* ws, size_t ws_bytes,
                                      void* stream);

/* Copy macro e's assembled (flags=0) local matrix A_e, row-major N_e x N_e,
 * into dst (device f64).  Re-assembles it from the templates; no factor
 * state is touched.  For tests of the assembly. */
mhdg_status mhdg_local_matrix(mhdg_mesh* mesh, int64_t e, double* dst, void* stream);

/* out = S lam, or D^-1 S lam with MHDG_PRECONDITION; with MHDG_TRANSPOSE the
 * transposed operator S^T lam (or D^-1 S^T lam; D is symmetric), FP64
 * factors only.  lam, out: device f64[n_trace], must not alias.  With
 * MHDG_GRAPH the launches run as one replay of a captured hipGraph; the
 * result is the same bit for bit.  (Steps 1-4 of the matrix-free method of
 * section 3.3.2: gather and lift, local solve, restriction, face sum; the
 * preconditioned step 4 is the D^-1 variant of section 6.1.)  MHDG_FOLDED,
 * MHDG_ASSEMBLED and MHDG_BOUNDARY run steps 1-3 through the stored
 * condensed operators instead of the factors.
 * Errors: STATE before factor_local, or a condensed form not yet built;
 * INVALID_ARG for MHDG_ASSEMBLED with MHDG_TRANSPOSE or with another
 * condensed form, MHDG_BOUNDARY with MHDG_FOLDED. */
mhdg_status mhdg_apply_trace_operator(mhdg_mesh* mesh, const double* lam, double* out,
                                      int32_t flags, void* stream);

/* The trace operator applied to n_rhs vectors at once: out_v = S lam_v (or
 * D^-1 S lam_v with MHDG_PRECONDITION) for v = 0 .. n_rhs-1, the same
 * operator as mhdg_apply_trace_operator (steps 1-4 of section 3.3.2) with
 * several right-hand sides per local solve: each macro's factors are read
 * once per group of vectors (8 vectors for N_K <= 512, 4 up to 1024, 2 up to
 * 2048, 1 above), not once per vector.  For callers with many vectors
 * against one factorisation (several load cases, block Krylov methods).
 * With MHDG_FOLDED the folded operators T_K (mhdg_fold_operator, from
 * MHDG_FP64 or MHDG_QELIM factors) are applied instead, each T_K read once
 * per group of 8 vectors.
 * lam, out: device f64[n_rhs][n_trace] (vector v at offset v * n_trace);
 * the two ranges must not overlap.  ws: device workspace of at least
 * mhdg_apply_many_ws_bytes(mesh, n_rhs) bytes (per-vector contribution
 * slots), owned by the caller; its contents on entry do not matter.
 * flags: MHDG_PRECONDITION and/or MHDG_FOLDED.  n_rhs = 0 is a no-op.
 * Errors: INVALID_ARG (n_rhs < 0, other flags, null or overlapping
 * vectors), STATE (before factor_local; without MHDG_FOLDED, factors other
 * than MHDG_FP64; with it, before mhdg_fold_operator), WORKSPACE (ws too
 * small). */
size_t mhdg_apply_many_ws_bytes(const mhdg_mesh* mesh, int32_t n_rhs);
mhdg_status mhdg_apply_trace_operator_many(mhdg_mesh* mesh, int32_t n_rhs, const double* lam,
                                           double* out, int32_t flags, void* ws,
                                           size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under stream or
 * graph capture, tight serving loops, hosts that forbid allocation): the
 * many-vector apply of mhdg_apply_trace_operator_many, same arguments and
 * result, without the workspace.  The contribution slots live in a fixed
 * device array of the library, MHDG_NOALLOC_SCRATCH_BYTES per GPU, held from
 * the first call on that GPU until the process ends.  The call makes no
 * device allocation and records no timing events.  Needs
 * mhdg_apply_many_ws_bytes(mesh, n_rhs) <= MHDG_NOALLOC_SCRATCH_BYTES
 * (at 8192 macros, r = 3, p = 3, up to 13 vectors per call); larger requests
 * return INVALID_ARG before anything is launched.  Every call on one GPU
 * shares that GPU's array, whose contents on entry do not matter: calls that
 * overlap on one GPU (other streams, threads or handles) race, and the caller
 * must order them.  Errors: as mhdg_apply_trace_operator_many, and HIP if the
 * array's address cannot be looked up. */
#define MHDG_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
mhdg_status mhdg_apply_trace_operator_many_noalloc(mhdg_mesh* mesh, int32_t n_rhs,
                                                   const double* lam, double* out, int32_t flags,
                                                   void* stream);

/* y_K = A_K^-1 x_K (or A_K^-T x_K with MHDG_TRANSPOSE) for every macro with
 * the stored factors (step 2).  x, y: device f64[n_local], may alias. */
mhdg_status mhdg_local_solve(mhdg_mesh* mesh, const double* x, double* y, int32_t flags,
                             void* stream);

/* Right-hand side of the global problem, f^ = -sum_K C_K A_K^-1 R_K, with
 * R_K built from f (device f64[n_nodes]) and g_D (device f64[n_bnd_points]);
 * fhat: device f64[n_trace] (D^-1 f^ with MHDG_PRECONDITION).  Keeps R_K in
 * the factor workspace for recover_local. */
mhdg_status mhdg_rhs(mhdg_mesh* mesh, const double* f_nodes, const double* g_bnd, double* fhat,
                     int32_t flags, void* stream);

/* Solve the global problem S lam = f^ (eq. global_problem of section
 * 3.3.1, with S applied matrix-free by the steps of section 3.3.2) by
 * GMRES(restart) left-preconditioned with D^-1 as in section 6.1, all
 * vector work in FP64 on the device.  Calls mhdg_rhs first.  When the
 * factors are FP32 the solve is an FP64 iterative refinement of the whole
 * hybridised system: the residual (R - A U - B lam, -(C U + D lam)) is formed
 * matrix-free in FP64 and each correction solves the condensed system with
 * the FP32 factors (inner GMRES to opts->inner_rtol), until the condensed
 * FP64 residual is below rtol relative to its initial value.  lam: device
 * f64[n_trace] (initial guess unless opts->zero_guess, then the solution).
 * ws: device workspace of at least solve_ws_bytes (mhdg_query with the same
 * restart).  info: host array of n_inst entries (one per coefficient
 * instance; iterations and residuals are per instance) or NULL.  With
 * several instances the factors must be FP64 (STATE otherwise).  The
 * stopping test (opts->stop_norm) is checked on the exact residual at the
 * start of every restart cycle; with the device driver the host waits once
 * per cycle.  Returns NOT_CONVERGED if max_iter was reached before every
 * instance converged (lam then holds the last iterates), INVALID_ARG for
 * MHDG_NORM_TRUE with reduced-precision factors or with the host driver. */
mhdg_status mhdg_solve(mhdg_mesh* mesh, const double* f_nodes, const double* g_bnd,
                       const mhdg_solve_opts* opts, double* lam, void* ws, size_t ws_bytes,
                       mhdg_solve_info* info, void* stream);

/* Macro conservation residual, per macro K: <flux^.n, 1>_dK - (f_h, 1)_K
 * with the LDG-H flux a.n lam + kappa q.n + tau (u - lam) of section 3.1
 * (eq. weak_form tested with w = 1, the statement of macro-element
 * conservation).  lam: device f64[n_trace] (the interior trace; boundary
 * faces use the Dirichlet trace of the last mhdg_rhs / mhdg_solve), qu:
 * device f64[n_local] (q_x, q_y, u per macro, as written by
 * mhdg_recover_local), f_nodes: device f64[n_nodes] (the source given to
 * rhs/solve), out: device f64[n_macro].  Zero to rounding for local fields
 * recovered from any lam; any factor precision.
 * Errors: STATE before factor_local and rhs/solve, INVALID_ARG on null
 * vectors. */
mhdg_status mhdg_flux_balance(mhdg_mesh* mesh, const double* lam, const double* qu,
                              const double* f_nodes, double* out, void* stream);

/* Local recovery U_K = A_K^-1 (R_K - B_K lam_K) into qu (device
 * f64[n_local]; with FP32 factors refined in FP64 until the local residual
 * stops decreasing) and, if flux_res is not NULL, the transmission residual
 * sum_K C_K U_K + D_F lam_F per interior trace dof (device f64[n_trace]).
 * Needs mhdg_rhs (or solve) to have run since factor_local. */
mhdg_status mhdg_recover_local(mhdg_mesh* mesh, const double* lam, double* qu, double* flux_res,
                               void* stream);

/* out_K = M_K v_K for every macro and each of the three fields (M_K the
 * macro mass matrix (phi_j, phi_i)_K); v, out: device f64[n_local], not
 * aliased.  Gives L2 inner products of local fields, e.g. for objectives. */
mhdg_status mhdg_mass_apply(mhdg_mesh* mesh, const double* v, double* out, void* stream);

/* Adjoint of a solved problem for an objective J(U) with gradient dJ_dU
 * (device f64[n_local]) at the solution (lam from solve, qu from
 * recover_local): solves K^T Psi = dJ/dX for the hybridised system by static
 * condensation with the stored FP64 LU factors (GMRES on D^-1 S^T to
 * opts->rtol, then psi_K = A_K^-T (g_K - C_K^T psi_lam)) and returns
 *   dJ_dkappa[n_macro] = dJ/dkappa_K = -Psi^T dK/dkappa_K X   (device f64)
 *   dJ_dbeta[2]        = dJ/da_d = Psi^T (dF/da_d - dK/da_d X)   (device f64)
 * plus psi_lam (device f64[n_trace]) and psi_U (device f64[n_local]).  f is
 * held fixed.  ws: the solve workspace (mhdg_query with the same restart).
 * Errors: STATE without solve, with FP32 factors or with more than one
 * coefficient instance; NOT_CONVERGED. */
mhdg_status mhdg_adjoint(mhdg_mesh* mesh, const double* lam, const double* qu, const double* dJ_dU,
                         const mhdg_solve_opts* opts, double* psi_lam, double* psi_U,
                         double* dJ_dkappa, double* dJ_dbeta, void* ws, size_t ws_bytes,
                         mhdg_solve_info* info, void* stream);

/* Kernel shapes per size class (all macros of one local size N_K).  The
 * factorisation has two forms: LU variant 1 factors 8- or 16-column panels
 * held in registers and updates the trailing matrix after each; variant 2
 * blocks 64-column panels (8-column register sub-panels, a blocked
 * triangular solve and one rank-64 MFMA update per panel), reading the
 * trailing matrix 4-8 times less often; variants 3 and 4 are variant 2 with
 * the rank-64 update's U tiles loaded once into LDS for 2 or 4 row tiles
 * per wavefront instead of streamed per row tile; variant 5 takes 128-column
 * panels, one launch per step (panel factorisation in one workgroup per
 * macro, row moves and U12 = L11^-1 A12 on MFMA, then the rank-128 trailing
 * update as a batched MFMA GEMM over 64 x 64 tiles spread across the chip,
 * all tiles of one macro on one XCD).  The per-macro triangular solves
 * (steps 1-3) run on one wavefront per macro (solve variant 1), or on four
 * or eight wavefronts per macro (variants 2, 3) that split each column, or,
 * for N_K in (512, 1024], on one wavefront per macro with the register
 * budget of 6, 5, 5 or 4 resident wavefronts per SIMD and 8, 8, 12 or 16
 * factor columns' chunks in flight per load group (variants 4 to 7). */
#define MHDG_MAX_CLASSES 8
enum { MHDG_TUNE_LU = 1, MHDG_TUNE_SOLVE = 2 };
typedef struct {
  int32_t n_classes;
  int32_t N[MHDG_MAX_CLASSES];
  int64_t count[MHDG_MAX_CLASSES];
  int32_t lu_variant[MHDG_MAX_CLASSES];     /* chosen (1 to 5)                 */
  int32_t solve_variant[MHDG_MAX_CLASSES];  /* chosen (1 to 7)                 */
  double lu_ms[MHDG_MAX_CLASSES][6];        /* [class][variant]: LU of up to 512
                                               macros of the class; 0 = not tried */
  double apply_ms[MHDG_MAX_CLASSES][8];     /* [class][variant]: one apply solve
                                               of the whole class; 0 = not tried */
} mhdg_tune_report;

/* Autotuner: times every available LU variant (flags & MHDG_TUNE_LU) on
 * the handle's own assembled matrices and every solve variant
 * (flags & MHDG_TUNE_SOLVE) on its factors, per size class, keeps the
 * fastest, refactors with the chosen LU variants (the factor state stays
 * valid) and remembers the choice for this process: later factor_local
 * calls of any handle with the same (N_K, precision, class size rounded up
 * to a power of two) start from it.  Needs factor_local first; synchronises;
 * costs about two factorisations.  out (host) may be NULL.
 * Errors: STATE, INVALID_ARG (more than MHDG_MAX_CLASSES classes), SINGULAR, HIP. */
mhdg_status mhdg_autotune(mhdg_mesh* mesh, int32_t flags, mhdg_tune_report* out, void* stream);

/* SUPG stabilisation inside the macro-elements (section 3.4): with on = 1
 * the local forms get tau_e (a.grad w, a.grad u - kappa lap u)_e on every
 * sub-triangle e and the source tau_e (a.grad w, f_h)_e, with h the
 * sub-triangle diameter, Pe = |a| h / (2 kappa) and tau = h / (2|a|)
 * (coth Pe - 1/Pe) (the classical value; zero without advection).  The
 * local blocks change, the trace system keeps its form; conservation per
 * macro is unaffected (a.grad 1 = 0).  on = 0 restores the plain forms.
 * Either way the factors are invalidated (call factor_local again).  Every
 * precision and form supports it except mhdg_adjoint (STATE: the forms are no
 * longer affine in kappa and a).  Errors: INVALID_ARG if on is not 0 or 1. */
mhdg_status mhdg_set_supg(mhdg_mesh* mesh, int32_t on);

/* Fix the variants of the size class with local size N (0 = the default
 * rule: LU variant 1 for N <= 256, else 5; solve variant 1 for N <= 512,
 * 7 for N in (512, 1024] (1 with BF16 factors), else 2).  Takes effect at the
 * next factor_local (LU) or apply (solves).
 * Errors: INVALID_ARG (no class of that size, variant not available). */
mhdg_status mhdg_set_kernel_variant(mhdg_mesh* mesh, int32_t N, int32_t lu_variant,
                                    int32_t solve_variant);

/* Fold steps 1-3 into one dense matrix per macro: T_K = C_K A_K^-1 B_K over
 * the macro's interior-face trace dofs (L_K = sum of the n_F of its interior
 * faces, at most 192), so that S lambda = D lambda - sum_K T_K lambda_K (eq.
 * global_problem) reads L_K^2 values per macro instead of the N_K^2 of the
 * factors.  The matrices are built in one launch from the stored factors as
 * a many-right-hand-side solve: every column of B_K (the lift of one trace
 * unit vector) is solved with A_K's factors, several columns per pass over
 * them, and restricted with C_K into the matching column of T_K.  With
 * MHDG_FP64 factors A_K is the full block; with MHDG_QELIM factors the
 * solve goes through the Schur block on u and the reference mass (the same
 * operator up to rounding).  ws: device workspace of at least
 * fold_ws_bytes (mhdg_query), kept by the handle until the next
 * factor_local or set_instances.  Then apply_trace_operator with
 * MHDG_FOLDED, or solve with opts->folded = 1, use them; recover_local, rhs
 * and adjoint keep using the factors.  Synchronises.
 * Errors: STATE (before factor_local, or FP32 / BF16 factors), WORKSPACE,
 * INVALID_ARG (a macro trace larger than 192). */
mhdg_status mhdg_fold_operator(mhdg_mesh* mesh, void* ws, size_t ws_bytes, void* stream);

/* The matrix-based form of section 6.1: the global trace matrix
 * S = D - sum_K C_K A_K^-1 B_K (eq. global_problem) assembled over the
 * interior trace unknowns from the folded operators T_K of
 * mhdg_fold_operator.  Storage is block-sparse: one block per pair of
 * interior faces that share a macro (rows and columns in the faces'
 * canonical trace order), S_FF' = delta_FF' D_F - sum_{K holds F, F'}
 * T_K[F, F'], each block column-major.  The left-preconditioned matrix
 * D^-1 S (block (F, F') times D_F^-1) is stored beside it in the same layout,
 * so that preconditioned products need no D_F^-1 step.  Applies with
 * MHDG_ASSEMBLED (and solves with opts->assembled) then run one block-sparse
 * product per face row, over D^-1 S with MHDG_PRECONDITION and over S
 * without.  ws: device workspace of at least mhdg_trace_matrix_ws_bytes
 * bytes, owned by the caller and used until the next factor_local or
 * fold_operator.  Layout: int32 row_ptr[n_interior_faces + 1] (the blocks of
 * face row f are row_ptr[f] .. row_ptr[f + 1] - 1); from the next 256-byte
 * boundary the block table (72 bytes per block); from the next 256-byte
 * boundary the values of S; from the next the values of D^-1 S (the same
 * size).  At 8192 macros, r = 3, p = 3: 60,292 blocks, 301 MB of values
 * each, 607 MB in all (the T_K take 369 MB).  Synchronises the stream once.
 * Errors: STATE (before mhdg_fold_operator), WORKSPACE, INVALID_ARG (face
 * traces over 129 values), HIP. */
size_t mhdg_trace_matrix_ws_bytes(const mhdg_mesh* mesh);
mhdg_status mhdg_assemble_trace_matrix(mhdg_mesh* mesh, void* ws, size_t ws_bytes, void* stream);

/* Boundary-condensed macro operators.  Steps 1-3 of section 3.3.2 apply
 * C_K A_K^-1 B_K; B_K (face integrals against the macro basis) is nonzero
 * only on boundary-node rows and C_K only on boundary-node columns, so the
 * product equals C_b W_K B_b with W_K = (A_K^-1)_bb, the block of A_K^-1 on
 * the boundary nodes of all three fields.  Where the interior block A_ii is
 * invertible, W_K is the inverse of the boundary Schur complement
 * A_bb - A_bi A_ii^-1 A_ib (the interior unknowns condensed out); W_K is
 * formed from the stored factors by 9P solves with unit right-hand sides (the
 * LU of A_K with MHDG_FP64 factors; with MHDG_QELIM the flux elimination and
 * the Schur-block LU, the same solves), which also covers a macro whose A_ii
 * is singular.
 * Layout of ws (device memory of at least mhdg_boundary_ws_bytes bytes, owned
 * by the caller and read by every later MHDG_BOUNDARY apply until the next
 * factor_local, set_instances or set_supg): int64 offsets[n_macro], then from
 * byte offset align256(8 n_macro) the blocks, W_K at element offsets[K]:
 * 9P x 9P FP64 column-major (P = 2^r_K p), rows and columns in the order
 * field (q_x, q_y, u) major, then boundary position b = kP + s, the node at
 * position s = 0 .. P-1 of local edge k (from vertex k towards vertex k+1).
 * At 8192 macros, r = 3, p = 3 the blocks take 3.06 GB (216 x 216 each).
 * Applies with MHDG_BOUNDARY (and solves or adjoints with opts->boundary)
 * then read W_K once per macro.  Synchronises the stream once.
 * Errors: STATE (before factor_local, or factors other than MHDG_FP64 and
 * MHDG_QELIM), WORKSPACE, INVALID_ARG (9P > 512), HIP. */
size_t mhdg_boundary_ws_bytes(const mhdg_mesh* mesh);
mhdg_status mhdg_condense_boundary(mhdg_mesh* mesh, void* ws, size_t ws_bytes, void* stream);

/* Per-kernel timing of the hot path, for measurement.  enable = 1 clears
 * the counters and brackets every later launch of the listed kernels with
 * HIP events recorded on the launch stream; enable = 0 stops recording,
 * waits for the recorded events and fills *out (may be NULL).  Index:
 * 0 assemble, 1 lu, 2 macro solve of apply_trace_operator (steps 1-3),
 * 3 face combine (step 4), 4 macro solve of rhs/recover/local_solve,
 * 5 condensed apply (steps 1-3 through T_K or W_K, or the assembled
 * product).  An apply replayed from a captured graph (MHDG_GRAPH) is timed
 * whole under index 2 (5 for the condensed forms). */
typedef struct {
  int32_t count[6];
  double ms[6];
} mhdg_kernel_times;
mhdg_status mhdg_profile(mhdg_mesh* mesh, int32_t enable, mhdg_kernel_times* out);

void mhdg_destroy(mhdg_mesh* mesh);
const char* mhdg_last_error(const mhdg_mesh* mesh);
const char* mhdg_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* MHDG_H_ */
