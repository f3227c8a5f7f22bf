/*
 * lyapsmw -- batched trace(E X(p)) for parametrized Lyapunov equations on MI355X.
 *
 * Problem (Section 1, equations (Ljap jdba 1) and (eq:formA)): for many
 * parameter samples p with D(p) = diag(d(p)), d(p) in R^r,
 *
 *     A(p) X + X A(p)^T = -B B^T,      A(p) = A0 - U D(p) V^T,
 *
 * evaluate f(X(p)) = trace(E X(p)).
 *
 * Method (Section 2.1): the seed A0 is factored once (A0 = Q0 Lambda0 Q0^-1,
 * offline stage of Table 1); every p is handled by a Sherman-Morrison-Woodbury
 * correction whose capacitance system (eq:SMW_linearsystem) is solved by a
 * preconditioned, restarted Krylov method (the preconditioner is eq:prec with
 * its exact block-diagonal part), and every Krylov matrix-vector product is a
 * seed Lyapunov solve with a low-rank right-hand side, i.e. a Cauchy-matrix
 * contraction in the eigenbasis (eq:Z(v), eq:N2M1).  The capacitance system is
 * solved in its n*r reduced form, unknown Y = D V^T X(p) (r x n), which carries
 * the same unknowns as the paper's 2nk vector w(v) (w1 = w2^T).  The seed option
 * tsvd_rank adds the low-rank part of eq:prec.
 *
 * Also here: full solutions X(p) for other functionals (seed_full_X), and the
 * projection framework of Section 2.2 (ek_*), whose projected equations are
 * solved by the same engine.
 *
 * Conventions shared by every entry point:
 *  - Host matrices are row-major (C order), float64.
 *  - Device buffers are float64 unless stated, and belong to the caller.
 *  - Calls are ordered on the HIP stream given as `void* hip_stream`
 *    (NULL = the default stream).  seed_factor, smw_solve_batch, seed_full_X
 *    and the ek_* calls also synchronise that stream before they return (they
 *    drive the iteration from the host).  lyap_seed_apply and trace_EX only
 *    enqueue work.
 *  - Argument errors return synchronously, before any launch, with
 *    LYAP_E_INVAL.  No call aborts, throws or exits.
 *  - Per-parameter numerical failures are reported in lyap_result.status;
 *    the call itself then returns LYAP_OK.
 *  - A seed is read-only after seed_factor and may be used from several
 *    streams at once, except that lyap_seed_apply and trace_EX share a
 *    per-seed scratch area: calls of those two on one seed must not overlap.
 */
#ifndef LYAPSMW_H
#define LYAPSMW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lyap_seed_s* lyap_seed;
typedef struct lyap_engine_s* lyap_engine;
typedef struct lyap_ek_s* lyap_ek;

typedef enum {
  LYAP_OK = 0,
  LYAP_E_INVAL = 1,        /* bad argument (size, pointer, non-finite host input, workspace) */
  LYAP_E_NOMEM = 2,        /* device or host allocation failed */
  LYAP_E_UNSTABLE = 3,     /* seed has lambda_i + lambda_j ~ 0: no unique Lyapunov solution */
  LYAP_E_NOCONV = 4,       /* per-parameter: iteration limit reached before the tolerance */
  LYAP_E_BREAKDOWN = 5,    /* per-parameter: Krylov breakdown without convergence */
  LYAP_E_DEVICE = 6,       /* a HIP runtime call failed */
  LYAP_E_UNSUPPORTED = 7,  /* requested option not available (e.g. no host LAPACK found) */
  LYAP_E_NONFINITE = 8     /* per-parameter: NaN/Inf in d(p) or in the iteration */
} lyap_status;

typedef enum {
  LYAP_BASIS_AUTO = 0,   /* eigenbasis unless its condition estimate exceeds max_eig_cond */
  LYAP_BASIS_EIG = 1,    /* complex eigenbasis of A0 (Section 2.1), stored in real form */
  LYAP_BASIS_SCHUR = 2   /* real Schur basis with a triangular Bartels-Stewart seed solve */
} lyap_basis;

typedef enum {
  LYAP_PREC_FP64 = 0,     /* every matrix-vector product in FP64 (MFMA f64) */
  LYAP_PREC_FP32_IR = 1,  /* inner Krylov products in FP32 MFMA, FP64 residuals and refinement */
  LYAP_PREC_BF16_IR = 2,  /* inner products as three BF16 MFMA products (split operands), FP32
                             accumulation, FP64 residuals and refinement */
  LYAP_PREC_FP32 = 3      /* FP32 MFMA products, no FP64 refinement (tolerance ~1e-6) */
} lyap_prec;

typedef struct {
  int32_t basis;          /* lyap_basis */
  int32_t E_is_diag;      /* 1: E is an n-vector (diagonal); 0: E is dense n x n (symmetrised) */
  double max_eig_cond;    /* AUTO switches to the Schur basis when the eigenbasis condition
                             estimate ||S||_1 ||S^-1||_1 exceeds this (default 1e5 if <= 0;
                             the refined eigenbasis route kept trace errors below 1e-12 up to
                             1.3e5 and first exceeded 1e-10 at 5e5 on nearly defective seeds) */
  int32_t tsvd_rank;      /* rank pbar of the truncated SVD of the dense coupling block that
                             completes the preconditioner of eq:prec (Section 2.1); 0 (default)
                             keeps only its exact block-diagonal part; at most 64; eigenbasis
                             seeds only (ignored in the Schur basis) */
  int32_t schur_dense;    /* Schur basis only: 0 (default) assembles the capacitance operator
                             as a dense (r ld)^2 matrix when n <= 2048 and r ld <= 8192 (one
                             GEMM per Krylov step; assembly: r n quasi-triangular solves of
                             size n); -1 keeps the per-slot quasi-triangular solve in every
                             step (no (r ld)^2 memory) */
  int32_t seed_refine;    /* eigen basis only: steps of fixed-precision iterative refinement
                             of the seed quantities every parameter shares -- t0, c0 and the
                             trace weights are formed from the explicit seed solution X0 and
                             adjoint solution G, each refined with its FP64 residual in
                             physical coordinates (a few n x n GEMMs per step, once per seed).
                             0 (default) = 1 step, -1 = none (quantities straight from the
                             eigenbasis), 1..4 = that many steps */
} lyap_seed_opts;

typedef struct {
  int32_t prec;           /* lyap_prec */
  int32_t max_iter;       /* total matrix-vector products per parameter (default 600) */
  int32_t restart;        /* Krylov dimension per cycle m (0: default, 64 for restarted
                             GMRES and 40 with recycle_k > 0; at most 64) */
  int32_t use_precond;    /* right preconditioner of eq:prec: 1 (default) = its exact
                             block-diagonal part plus the seed's coupling TSVD if it holds one
                             (lyap_seed_opts.tsvd_rank), 2 = block-diagonal part only,
                             0 = none; the eigenbasis path with r <= 8 only */
  int32_t recycle_k;      /* GCRO-DR recycle space dimension s (Section 2.1, Parks et al.):
                             0 = restarted GMRES (default); at most 16, restart + recycle_k
                             <= 64.  Each cycle end replaces the space by the harmonic Ritz
                             vectors of smallest magnitude; a slot that takes a new parameter
                             rebuilds C = A P^-1 U with recycle_k extra products */
  int32_t max_refine;     /* FP64 refinement steps for the *_IR modes (default 30) */
  double tol;             /* FP64 relative residual target ||b - A y|| / ||b|| (default 1e-12) */
  double inner_tol;       /* relative reduction per inner cycle in *_IR modes (default 1e-4) */
} lyap_solve_opts;

typedef struct {
  int32_t status;         /* lyap_status of this parameter */
  int32_t iters;          /* matrix-vector products (all precisions) */
  int32_t cycles;         /* restart cycles (= FP64 residual evaluations) */
  int32_t refinements;    /* FP64 refinement steps that were followed by an inner solve */
  double rel_residual;    /* final FP64 relative residual of the capacitance system */
  double trace;           /* trace(E X(p)) from the eigen-coordinate solution */
  double err_est;         /* estimated relative error of trace, twice the first-order
                             estimate 2 (eps_seed (max(1, |t0| / |trace|) + kappa (1 + g))
                             + kappa rel_residual), g = ||y - D c0|| / ||D c0|| the
                             strength of the low-rank correction (y the capacitance solution),
                             eps_seed = the seed's measured eigenbasis error (relative
                             change of t0 under the seed refinement), kappa = a condition
                             estimate of the preconditioned capacitance system from the
                             last Krylov cycle; NaN for an unrefined seed (seed_refine =
                             -1), a Schur-basis seed, or the shifted-family solve */
} lyap_result;

typedef struct {
  int64_t n, r, s;
  int64_t npairs;         /* complex-conjugate eigenvalue pairs (h); real eigenvalues = n - 2h */
  int64_t ld;             /* padded leading dimension of every n-vector on the device */
  int32_t basis;          /* basis actually used */
  int32_t tsvd_rank;      /* rank of the coupling TSVD held by the seed (0: none) */
  double cond_est;        /* ||S||_1 ||S^-1||_1 of the real eigenbasis (unit-norm eigenvectors) */
  double min_lam_sum;     /* min |lambda_i + lambda_j| / max |lambda_i + lambda_j| */
  double max_re_lambda;   /* largest real part of the seed spectrum */
  double t0;              /* trace(E X0) of the seed equation (eq:seedLE) */
  double t0_unrefined;    /* t0 straight from the eigenbasis, before seed_refine */
  double eps_seed;        /* |t0_unrefined - t0| / |t0| (NaN if not refined) */
  int32_t seed_refine;    /* refinement steps applied (0: none) */
  double factor_seconds;  /* host wall time of seed_factor */
  size_t device_bytes;
} lyap_seed_info;

/* ------------------------------------------------------------------------ */
/* Offline stage (Table 1, left column).                                     */
/* ------------------------------------------------------------------------ */

/* Factor the seed A0 and precompute everything that does not depend on p.
 *   n, r, s  : sizes, 1 <= r <= n, 1 <= s, n <= 16384.
 *   A0       : host n x n.     U, V : host n x r (A(p) = A0 - U diag(d) V^T).
 *   B        : host n x s (right-hand side -B B^T).
 *   E        : host n (opts->E_is_diag) or n x n.
 *   opts     : may be NULL (AUTO basis, diagonal E).
 * The host eigendecomposition uses LAPACK dgeev resolved at run time from the
 * process (e.g. the copy inside libtorch_cpu) or from the library named by the
 * environment variable LYAP_LAPACK_LIB; LYAP_E_UNSUPPORTED if none is found.
 * Returns LYAP_E_UNSTABLE if some Re(lambda) >= 0 or lambda_i + lambda_j ~ 0.
 * On success *out owns all device memory of the seed until seed_release. */
lyap_status seed_factor(int64_t n, int64_t r, int64_t s, const double* A0, const double* U,
                        const double* V, const double* B, const double* E,
                        const lyap_seed_opts* opts, void* hip_stream, lyap_seed* out);

lyap_status seed_info(lyap_seed seed, lyap_seed_info* out);
lyap_status seed_release(lyap_seed seed);
size_t seed_device_bytes(lyap_seed seed);

/* ------------------------------------------------------------------------ */
/* The seed Lyapunov solve with a low-rank right-hand side (eq:Z(v)): for each */
/* b < batch, with Y_b = Y_dev + b*r*n (r x n row-major),                      */
/*     G_b = V^T X_b,   A0 X_b + X_b A0^T = U Y_b + Y_b^T U^T,                */
/* written to G_dev + b*r*n.  Transform into the eigenbasis, Cauchy           */
/* contraction (the division by lambda_i + lambda_j), transform back.          */
/* prec: LYAP_PREC_FP64 (other values return LYAP_E_UNSUPPORTED; the engine's   */
/* mixed-precision modes run inside smw_solve_batch).                         */
/* ------------------------------------------------------------------------ */
lyap_status lyap_seed_apply(lyap_seed seed, int64_t batch, const double* Y_dev, double* G_dev,
                            int32_t prec, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as lyap_seed_apply, which grows a work area on the
 * seed when a batch needs more; this variant allocates nothing.  Its work
 * area is a fixed array of 32 MiB per GPU, held from the first call on that
 * GPU until the process ends.  The work area takes (3 r + 2 r^2) ld 8 bytes
 * per batch entry for an eigenbasis seed and (3 r + ld) ld 8 bytes for a
 * Schur-basis seed (ld = n rounded up to a multiple of 128); a batch that
 * needs more returns LYAP_E_INVAL before any launch.  The seed's device must
 * be the current device (LYAP_E_INVAL otherwise).  Every call on one GPU
 * uses the same area: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  Only enqueues work;
 * the area is cleared by a kernel at the start of each call. */
lyap_status lyap_seed_apply_noalloc(lyap_seed seed, int64_t batch, const double* Y_dev,
                                    double* G_dev, int32_t prec, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Online stage (Table 1, right column).                                     */
/* ------------------------------------------------------------------------ */

/* Device workspace smw_solve_batch needs for P parameters: every buffer of the
 * batched Krylov engine (basis, iterates, preconditioner blocks, GEMM operands,
 * device queue) plus the solution store, exactly what the call uses; 0 if the
 * seed or the options are not supported by the engine (lyap_last_error says
 * why).  The Krylov kernel holds one capacitance vector per workgroup:
 * r * ld <= 16384, ld = n rounded up to a multiple of 128. */
size_t smw_workspace_bytes(lyap_seed seed, int64_t P, const lyap_solve_opts* opts);

/* Solve the capacitance system for P parameters.
 *   d_dev     : device P x r, row p = diag of D(p).  Entries must be finite;
 *               zero is allowed (the system is used in the form (I - D K) Y = D c0).
 *   Y_dev     : device P x r x n output, Y(p) = D(p) V^T X(p) (physical coordinates).
 *   res_host  : host array of P results (status, iterations, residual, trace).
 *   workspace : device buffer of at least smw_workspace_bytes(seed, P, opts) bytes,
 *               256-byte aligned, or NULL.  Given a workspace, the call carves every
 *               engine buffer from it and allocates no device memory of its own; the
 *               seed keeps the engine's captured step graphs for the next call with
 *               the same P, options and workspace, which then only resets the
 *               engine's state (no allocation, no capture).  The workspace must stay
 *               allocated while the seed may reuse it (until a call with another
 *               workspace, P or options, or seed_release).  With NULL, the seed
 *               allocates and owns the engine and the solution store
 *               (seed_device_bytes counts them).
 * All P parameters are batched: slots of the Krylov engine are filled with
 * parameters in order and refilled as parameters converge.  The call
 * synchronises the stream (the host polls the engine's progress). */
lyap_status smw_solve_batch(lyap_seed seed, int64_t P, const double* d_dev,
                            const lyap_solve_opts* opts, double* Y_dev, lyap_result* res_host,
                            void* workspace_dev, size_t workspace_bytes, void* hip_stream);

/* Shifted-family solve for one-column parameters (r = 1 only; not in the
 * paper).  For d != 0 the capacitance system (I - d K) y = d c0 equals
 * (sigma I - K) y = c0 with sigma = 1/d, so one Arnoldi process on K started
 * from c0 serves every parameter (GMRES for each shift, no preconditioner).
 * Cost: the Arnoldi steps the hardest parameter needs, nearly independent of P.
 *   d_host : host P doubles (finite; 0 gives y = 0).
 *   opts   : tol (relative residual, default 1e-12) and max_iter (Arnoldi
 *            steps, default 600, at most 2048); other fields are ignored.
 *   Y_dev  : device P x n output or NULL.   res_host: host P results (trace;
 *            iters = Arnoldi steps shared by all parameters).
 * LYAP_E_UNSUPPORTED if r != 1; LYAP_E_BREAKDOWN if the Krylov space becomes
 * invariant before every parameter has converged. */
lyap_status smw_solve_shifted(lyap_seed seed, int64_t P, const double* d_host,
                              const lyap_solve_opts* opts, double* Y_dev, lyap_result* res_host,
                              void* hip_stream);

/* trace(E X(p)) = t0 + 2 <Gamma, Y(p)> with Gamma = G U, A0^T G + G A0 = E
 * (the additive split of f in Section 2.1, collapsed to O(r n) per p).
 * Y_dev: device P x r x n from smw_solve_batch; trace_dev: device P doubles. */
lyap_status trace_EX(lyap_seed seed, int64_t P, const double* Y_dev, double* trace_dev,
                     void* hip_stream);

/* Full solutions for functionals other than the trace (eq:Xsmalllastline in
 * explicit form, O(n^3) per parameter): for each b < P,
 *     X_b = X0 + L^-1(U Y_b + Y_b^T U^T),  i.e.  A0 X_b + X_b A0^T = -B B^T + U Y_b + Y_b^T U^T,
 * with Y_b = Y_dev + b*r*n from smw_solve_batch (so X_b = X(p_b)).  Y_dev = NULL
 * with P = 1 returns X0.  X_dev: device P x n x n row-major (symmetric).
 * Eigen basis: block-diagonal real Lyapunov solve in the eigenbasis, then two
 * MFMA GEMMs; Schur basis: batched quasi-triangular solve, then the same GEMMs.
 * Work buffers of up to 3 GiB are allocated per call.  LYAP_E_UNSUPPORTED for
 * projected seeds (they hold no B). */
lyap_status seed_full_X(lyap_seed seed, int64_t P, const double* Y_dev, double* X_dev,
                        void* hip_stream);

/* Stability filter of a parameter sweep (the multi-agent importance example
 * of Section 4 discards every sample whose A(p) = A0 - U diag(d_p) V^T has an
 * eigenvalue with Re >= 0).  For each p < P, count_dev[p] = the number of
 * eigenvalues of A(p) in the open right half-plane, from the argument
 * principle applied to f(s) = det(I + D_p V^T (s I - A0)^-1 U) along the
 * imaginary axis (A0 is stable, so those eigenvalues are the zeros of f
 * there); V^T (i w - A0)^-1 U comes from the seed's eigenbasis on a frequency
 * grid shared by all p, and phase steps above pi/2 (an eigenvalue of A(p) near
 * the axis) are refined by direct evaluations in a second pass over the
 * samples concerned.  flag_dev[p] != 0 when the count is still not certain
 * (bit 1: a refined phase step still above pi/2, i.e. an eigenvalue of A(p)
 * extremely close to the axis; bit 2: f not near 1 at the last frequency;
 * bit 4: the phase total is not close to a multiple of pi, or not finite; bit 8: f = 0 at a
 * grid frequency); such samples are to be treated as not known to be stable.
 * d_dev: device P x r (P < 2^31); count_dev, flag_dev: device P int32.  Work buffers are
 * allocated per call; the call synchronises the stream.  LYAP_E_UNSUPPORTED
 * for a Schur-basis or projected seed, or r > 8. */
lyap_status seed_unstable_count(lyap_seed seed, int64_t P, const double* d_dev, int32_t* count_dev,
                                int32_t* flag_dev, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Continuous-batching engine (one seed, a fixed number of slots).            */
/* smw_solve_batch runs on an engine; a serving loop drives engines directly. */
/* ------------------------------------------------------------------------ */

/* Create an engine with `slots` concurrent parameters.  It allocates its own
 * device state (engine_device_bytes) and captures one Krylov step as a HIP
 * graph on `hip_stream`, which it keeps using. */
lyap_status engine_create(lyap_seed seed, int64_t slots, const lyap_solve_opts* opts,
                          void* hip_stream, lyap_engine* out);
size_t engine_device_bytes(lyap_seed seed, int64_t slots, const lyap_solve_opts* opts);
lyap_status engine_destroy(lyap_engine eng);

/* Queue `count` parameters (host count x r) with caller tags (host, may be NULL:
 * tags are then consecutive from the engine's running counter). */
lyap_status engine_submit(lyap_engine eng, int64_t count, const double* d_host,
                          const int64_t* tags);

/* Run up to `max_steps` Krylov steps (one matrix-vector product for every busy
 * slot per step), refilling slots from the queue every `poll_every` steps.
 * Returns when the engine is idle or max_steps is reached; *busy receives the
 * number of parameters still queued or in flight. */
lyap_status engine_run(lyap_engine eng, int64_t max_steps, int32_t poll_every, int64_t* busy);

/* Non-blocking variant for overlapping several engines: enqueue `steps`
 * Krylov steps on the engine's stream and return at once. */
lyap_status engine_launch(lyap_engine eng, int64_t steps);

/* Parameters submitted so far and finished so far (synchronises the engine's
 * stream to read the device counter). */
lyap_status engine_status(lyap_engine eng, int64_t* submitted, int64_t* done);

/* Move up to `max_out` finished results to the caller (tags, results). */
lyap_status engine_harvest(lyap_engine eng, int64_t max_out, int64_t* tags_out,
                           lyap_result* res_out, int64_t* n_out);

/* ------------------------------------------------------------------------ */
/* Projection framework (Section 2.2, eq:EK_def, eq:param_projected,          */
/* Proposition on the backward error, Algorithm EKSM_opt).                    */
/*                                                                            */
/* One extended Krylov space EK_m(A0, P), P = [X0 V, U], serves every         */
/* parameter.  The projected equation of a parameter is the SMW capacitance   */
/* system of a small projected seed (T_m = Q_m^T A0 Q_m, U_m, V_m, E_m), solved */
/* by the same batched Krylov engine; the backward error of each projected    */
/* solution is computed on the device from the p-independent tables of the    */
/* Proposition.  The basis is built on the host with LU solves of A0 (host    */
/* LAPACK dgetrf/dgetrs) and kept in host memory; each level's projected seed */
/* lives on the device.                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t status;         /* LYAP_OK: accepted (delta <= eps, or the space became invariant);
                             LYAP_E_NOCONV: not accepted up to m_max; else the failure
                             status of the projected solve at the last level tried (a
                             parameter whose projected solve fails is retried at the
                             next level) */
  int32_t level;          /* level m of the last projected solve (blocks in the basis) */
  int32_t dim;            /* projected dimension at that level */
  int32_t iters;          /* Krylov products over all levels tried */
  double delta;           /* backward error at that level */
  double trace;           /* trace(E X(p)) = t0 + trace(E_m Y_m(p)) at that level */
} lyap_ek_result;

typedef struct {
  int64_t n, r;
  int64_t level, dim;     /* current level and its projected dimension */
  int64_t blocks;         /* blocks built (the current level uses the first `level`) */
  int64_t basis_cols;     /* columns of the basis built so far */
  int32_t exhausted;      /* 1: the last block deflated to nothing (invariant space) */
  int32_t proj_basis;     /* basis of the projected seed (LYAP_BASIS_*), -1 before a level */
  double proj_cond;       /* eigenbasis condition estimate of the projected seed */
  double basis_seconds;   /* host time spent building basis blocks */
  double level_seconds;   /* host time spent forming projected seeds */
  double solve_seconds;   /* wall time of the batched projected solves */
  double delta_seconds;   /* wall time of the backward-error computations */
  int64_t batches;        /* batched projected solves run so far */
} lyap_ek_info;

/* V^T X0 of a factored seed, returned as X0 V (host n x r row-major): the
 * first half of P for ek_create when the seed solution comes from seed_factor. */
lyap_status seed_x0v(lyap_seed seed, double* X0V_host);

/* Build the first basis block span[P, A0^-1 P] (eq:EK_def).
 *   A0 : host n x n row-major (must be nonsingular; LU-factored here).
 *   U, V : host n x r (A(p) = A0 - U diag(d) V^T; the paper's B_l = U, B_r = V).
 *   X0V  : host n x r, X0 V with X0 the seed solution (A0 X0 + X0 A0^T = -B B^T).
 *   t0   : trace(E X0).      E : host n (E_is_diag) or n x n.
 * 2 <= n, 1 <= r <= 16, 4 r <= n.  The handle keeps host copies of its
 * inputs; ek_release frees everything. */
lyap_status ek_create(int64_t n, int64_t r, const double* A0, const double* U, const double* V,
                      const double* X0V, double t0, const double* E, int32_t E_is_diag,
                      void* hip_stream, lyap_ek* out);

/* Make level m current: extend the basis to m + 1 blocks (block m + 1 gives the
 * backward error of level m), project, factor the projected seed (proj_opts:
 * basis, max_eig_cond, tsvd_rank; E_is_diag is ignored) and upload the
 * backward-error data.  If the space becomes invariant first, the level stops
 * at the last nonempty block (ek_info reports the level actually used). */
lyap_status ek_set_level(lyap_ek ek, int32_t m, const lyap_seed_opts* proj_opts);

/* Solve the projected equations of P parameters at the current level.
 *   d_dev     : device P x r.      W_dev : device P x r x dim output (the
 *               capacitance solution of the projected seed, physical coordinates).
 *   delta_dev : device P output, backward error of each projected solution.
 *   norms_dev : device 2P output (||Y_m||_F, ||L Y_m||_F per parameter) or NULL.
 *   res_host  : host P results of the projected solves (trace = EK trace).
 * Synchronises the handle's stream before returning. */
lyap_status ek_solve(lyap_ek ek, int64_t P, const double* d_dev, const lyap_solve_opts* opts,
                     double* W_dev, double* delta_dev, double* norms_dev, lyap_result* res_host);

/* Algorithm EKSM_opt for P parameters (host d, P x r), levels m_start,
 * m_start + check_every, ... up to m_max (the algorithm starts at m_start = 1;
 * a later sweep on the same space may continue from the level an earlier one
 * reached, as in the algorithm's use inside optimisation loops).  Parameters are tested in order; the first whose backward
 * error exceeds eps (or whose projected solve fails) moves it and all after it
 * to the next level.  The queue head is solved in batches of 1, 4, 16, ...
 * parameters, keeping the accepted prefix of each batch, which reproduces the
 * sequential loop's decisions.  Levels (projected seeds, engines) are kept in
 * the handle and reused by later sweeps.  out: host P results. */
lyap_status ek_sweep(lyap_ek ek, int64_t P, const double* d_host, const lyap_solve_opts* opts,
                     const lyap_seed_opts* proj_opts, double eps, int32_t m_start,
                     int32_t m_max, int32_t check_every, lyap_ek_result* out);

lyap_status ek_info(lyap_ek ek, lyap_ek_info* out);
lyap_status ek_release(lyap_ek ek);

/* ------------------------------------------------------------------------ */
/* Measurement helpers (not part of the method).                             */
/* ------------------------------------------------------------------------ */

/* Per-kernel timings of engine steps, accumulated process-wide while
 * profiling is enabled.  Level 1: one step in 4 is timed (the others replay
 * the production graph); a timed step replays captured segments
 * before, between and after the Cauchy products and launches each product
 * between two HIP events on the engine stream, per-step active counts being
 * recorded by a small kernel.  Level 2: every step launched directly with
 * events also around the Krylov kernel.  *_flops are algorithmic: 2 r^2 n^2
 * per active parameter per product (the real-compressed Cauchy contraction),
 * not the padded tile work.  krylov_* stay zero at level 1. */
typedef struct {
  double gemm64_ms, gemm64_flops;
  double gemmlo_ms, gemmlo_flops;
  double krylov_ms;
  int64_t gemm64_launches, gemmlo_launches, krylov_launches;
  int64_t steps, slot_steps;
  int64_t graph_steps;    /* steps timed inside the captured profiling graph (the rest: direct launches) */
  int64_t tuned_bk, tuned_grid_min, tuned_xcd_off;  /* FP64 Cauchy GEMM launch chosen by the
                                                       autotuner for the last engine created */
} lyap_profile;

void lyap_profile_enable(int32_t level); /* 0 off, 1 GEMMs, 2 GEMMs + Krylov; resets counters */
lyap_status lyap_profile_read(lyap_profile* out);

/* Host-only real Schur decomposition used by the Schur-basis seed solve:
 * A = Z T Z^T, Z orthogonal, T upper quasi-triangular with 2x2 blocks only for
 * complex-conjugate pairs (Householder Hessenberg reduction + implicit
 * double-shift QR).  A, T, Z: host n x n row-major.  No GPU is touched.
 * Returns LYAP_E_UNSTABLE if the iteration does not converge. */
lyap_status lyap_real_schur(int64_t n, const double* A, double* T, double* Z);

/* Plain device copy of `bytes` bytes with a simple vector-load kernel; used to
 * calibrate hardware byte counters against a known traffic. */
lyap_status lyap_calib_copy(const void* src_dev, void* dst_dev, size_t bytes, void* hip_stream);

const char* lyap_status_string(lyap_status s);

/* Text of the most recent error raised by any entry point (process-wide). */
const char* lyap_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LYAPSMW_H */
