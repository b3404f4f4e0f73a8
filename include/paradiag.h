/*
 * paradiag.h -- C ABI of the MI355X (gfx950) ParaDiag solver.
 *
 * Solves the all-at-once backward-Euler system of a linear evolution problem
 * (Gander & Palitta, "A new ParaDiag time-parallel time integration method",
 * Section 1, all-at-once equation; generalised with a mass matrix M):
 *
 *     (M + tau K) U - M U Sigma_1^T = M [u0 + tau f_1, tau f_2, ..., tau f_ell]
 *
 * with the method of Section 2 (Algorithm 1): a DFT along time diagonalises
 * the circulant part C_1 of Sigma_1 = C_1 - e_1 e_ell^T, the shifted blocks
 * P_j = (1 - pi_j) M + tau K are solved independently, and the rank-one
 * correction is applied through the Sherman-Morrison-Woodbury formula with
 * the capacitance system J_ell x = b (eq. SMW_linearsystemII), solved here
 * by GMRES.  alpha < 1 selects the alpha-circulant variant (Section 4,
 * Algorithm 3, with the full correction always applied).
 *
 * Conventions (all entry points)
 *   - Every array argument named u0, F, U, v, x, b, Jv, Hhat, Uhat is a
 *     DEVICE pointer (e.g. torch.Tensor.data_ptr() of a contiguous tensor on
 *     the plan's GPU).  M and K are HOST pointers, copied at plan creation.
 *   - Space-time arrays are time-major float64: F[j*nbar + i] is f(x_i, t_{j+1})
 *     and U[j*nbar + i] is u_{j+1}(x_i), j = 0..ell-1 (row j = the paper's
 *     column j+1).  u0 has nbar entries.
 *   - 1D: nbar = n.  2D (opt.dims = 2): n is the grid side, nbar = n*n,
 *     node (y, x) at index y*n + x, K is the 1D factor T of
 *     K_2D = I (x) T + T (x) I and must be symmetric Toeplitz, M must be NULL
 *     (identity).
 *   - Spectra ("Hhat", "Uhat") are the half spectrum j = 0..ell/2 of the
 *     time-DFT, frequency-major [ell/2+1][nbar], interleaved complex:
 *     complex128 for PD_FP64 plans, complex64 for PD_MIXED / PD_FP32 plans.
 *   - Work is enqueued on opt.stream (NULL = the null stream).  Entry points
 *     that return a scalar to the host (solve, residual, capacitance_solve)
 *     synchronise that stream before returning; the others are asynchronous.
 *   - Errors are returned as pd_status codes; no exception or abort crosses
 *     the ABI.  paradiag_last_error() gives a thread-local message.  On an
 *     error other than PD_ENOTCONV the output arrays are unspecified.
 *   - Calls on one plan must not overlap (the plan owns one workspace).
 */
#ifndef PARADIAG_H
#define PARADIAG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pd_plan_s *pd_plan;

typedef enum {
  PD_OK = 0,
  PD_EINVAL = 1,      /* invalid argument (sizes, tau, alpha, NULL pointer)  */
  PD_ENOMEM = 2,      /* device or host allocation failed                    */
  PD_EHIP = 3,        /* a HIP runtime call failed                           */
  PD_ENOTCONV = 4,    /* tolerance not reached within maxit / max_sweeps;    */
                      /* U holds the last iterate                            */
  PD_ESINGULAR = 5,   /* P_0 = tau K (alpha = 1) is singular, or a zero pivot */
  PD_ENONFINITE = 6,  /* a NaN or Inf appeared in a norm                     */
  PD_EBUDGET = 7,     /* request exceeds a device-memory budget              */
  PD_ENOTSUP = 8      /* valid but unsupported size or structure             */
} pd_status;

typedef enum {
  PD_KRYLOV_GMRES = 0,       /* GMRES on J_ell (Arnoldi on J_ell itself)         */
  PD_KRYLOV_FOM = 1          /* Algorithm 2: Galerkin projection onto            */
                             /* K_m(tau M^{-1} K, b) (= K_m(K, b) for M = I),   */
                             /* residual every fom_q steps; 1D float64 plans    */
                             /* with constant-diagonal M, K; at most 32 steps   */
} pd_krylov;

typedef enum {
  PD_SHIFTED_PARTITION = 0,  /* tridiagonal partition solves + parallel cyclic   */
                             /* reduction, capacitance system by GMRES (any M, K) */
  PD_SHIFTED_SINE = 1        /* 1D, float64, symmetric Toeplitz M and K (uniform */
                             /* grid, zero Dirichlet ends), n + 1 a power of two */
                             /* >= 16 or n <= 4095 (chirp-z DST): every shifted  */
                             /* matrix and J_ell diagonal in the DST-I basis;    */
                             /* capacitance solved exactly                       */
} pd_shifted_solver;

typedef enum {
  PD_FP64 = 0,        /* everything in float64 / complex128                  */
  PD_MIXED = 1,       /* complex64 transforms and shifted solves, float64    */
                      /* capacitance Arnoldi, residual and refinement        */
  PD_FP32 = 2         /* one complex64 sweep, no refinement                  */
} pd_precision;

/* A tridiagonal matrix: lower[i] multiplies x[i-1] in row i, upper[i]
 * multiplies x[i+1]; lower[0] and upper[n-1] are ignored.  Host pointers,
 * each of length n. */
typedef struct {
  const double *lower;
  const double *diag;
  const double *upper;
} pd_tridiag;

typedef struct {
  int dims;            /* 1 or 2                                            */
  int precision;       /* pd_precision                                      */
  double alpha;        /* alpha-circulant parameter in (0, 1]; 1 = Alg. 1   */
  int maxit;           /* capacitance GMRES iteration cap (1..64)           */
  int max_sweeps;      /* refinement sweeps cap for PD_MIXED (1..64)        */
  int check_residual;  /* PD_FP64/PD_FP32: also compute the float64 true    */
                       /* all-at-once residual after the solve              */
  void *stream;        /* hipStream_t                                       */
  int autotune;        /* 1D: time the candidate time-transform tile widths */
                       /* and shifted-solve rows per thread at plan creation */
                       /* and keep the fastest (cached per n, ell,          */
                       /* precision); 0 = built-in choice                   */
  int early_exit;      /* Algorithm 3's test: first form U_1 (the alpha-    */
                       /* circulant solve, x = 0) and return it when        */
                       /* ||G - A(U_1)||_F <= tol * ||M U_1||_F (M = I: the */
                       /* paper's ||U_1||_F), skipping the capacitance      */
                       /* solve; 0 = always correct                         */
  int shifted_solver;  /* pd_shifted_solver                                 */
  int krylov;          /* pd_krylov (ignored by PD_SHIFTED_SINE plans, whose */
                       /* capacitance system is solved exactly); BDF plans: */
                       /* PD_KRYLOV_FOM selects the block Galerkin method   */
                       /* of Section 5 (basis dimension s m <= 32)          */
  int fom_q;           /* PD_KRYLOV_FOM: residual check every fom_q steps   */
  int bdf_order;       /* s = 1..6: BDF of order s in time (Section 5,      */
                       /* table of BDF coefficients); 1 = backward Euler.   */
                       /* s > 1: PD_FP64, alpha 1, partition solves (1D or */
                       /* 2D; block Galerkin: 1D), no early_exit, ell >= 2s; */
                       /* u0 holds the                                      */
                       /* s starting values u_{1-s}..u_0 as [s][nbar] and   */
                       /* capacitance vectors are [s][nbar]                 */
} pd_options;

typedef struct {
  int gmres_iters;            /* capacitance GMRES iterations, all sweeps  */
  int sweeps;                 /* refinement sweeps done                    */
  int pint_loops;             /* batches of ell shifted solves (#PinT)     */
  double rel_residual;        /* ||G - A(U)||_F / ||G||_F, or -1           */
  double gmres_rel_residual;  /* last capacitance residual / ||b||         */
  int early_exit;             /* 1: U = U_1 was returned (early_exit test)  */
  double est_rel_error;       /* bound on ||M^1/2 (U* - U)||_F / ||M^1/2 U||_F
                                 from the computed residual R (U* the exact
                                 solution): sqrt(ell (ell+1) / 2)
                                 sqrt(lmax(M) / lmin(M)) ||R||_F / ||M U||_F,
                                 valid when M is symmetric positive definite
                                 and K symmetric positive semi-definite (both
                                 checked by Gershgorin's theorem at plan
                                 creation; backward Euler only).  Filled
                                 whenever the solve computes the float64
                                 residual (check_residual, or PD_MIXED's last
                                 check); otherwise -1. */
} pd_info;

/* Fill *opt with defaults: dims 1, PD_FP64, alpha 1, maxit 64,
 * max_sweeps 16, check_residual 0, stream NULL, autotune 0, early_exit 0,
 * shifted_solver PD_SHIFTED_PARTITION, krylov PD_KRYLOV_GMRES, fom_q 1,
 * bdf_order 1. */
void paradiag_default_options(pd_options *opt);

/* Every check paradiag_plan_create makes that needs no device, with the same
 * status codes: sizes, options, finite M and K, and -- with alpha = 1 -- a
 * nonsingular zero-frequency block P_0 = tau K (Section 2: the shift
 * 1 - pi_0 vanishes; a pure-Neumann K is rejected with PD_ESINGULAR).  Runs
 * on the host only (no GPU is touched); M, K are host pointers as for
 * paradiag_plan_create, opt may be NULL (defaults). */
pd_status paradiag_plan_check(int n, int ell, double tau, const pd_tridiag *M,
                              const pd_tridiag *K, const pd_options *opt);

/* Create a plan for an n x ell problem with time step tau (Section 1).
 * Computes pi_j, gamma_j (Section 2; Appendix), the shifted-matrix
 * coefficients and twiddle tables in float64 on the host, allocates the
 * device workspace and uploads the constants.
 * Sizes: ell a power of two, 2 <= ell <= 4096.  1D: 2 <= n <= 8192 for
 * PD_FP64, n <= 16384 otherwise.  2D: 2 <= n <= 1024 (the DST-I along x is
 * one FFT of length 2(n+1) per pair of rows when n + 1 is a power of two,
 * else the chirp-z form with FFTs of length L >= 2n - 1).
 * M == NULL means M = I.  Errors: PD_EINVAL, PD_ENOTSUP, PD_ENOMEM, PD_EHIP. */
pd_status paradiag_plan_create(pd_plan *out, int n, int ell, double tau,
                               const pd_tridiag *M, const pd_tridiag *K,
                               const pd_options *opt);

/* Algorithm 1 end to end: U = solution of the all-at-once system for
 * initial value u0 [nbar] and nodal source F [ell][nbar] (device float64),
 * written to U [ell][nbar] (device float64, must not alias u0 or F).
 * tol: the capacitance GMRES stops at residual <= tol/100 * ||b|| (with
 * float32 shifted solves, PD_MIXED and PD_FP32, at no less than 1e-7 * ||b||,
 * the resolution of float32 capacitance products); PD_MIXED refines until
 * the float64 relative all-at-once residual is <= tol, or until a sweep
 * fails to lower it: then that sweep's correction is taken back and the best
 * iterate is returned with PD_ENOTCONV (info->rel_residual is its residual).
 * BDF plans (bdf_order s > 1, Section 5): the system is
 * (M + tau beta K) U - M U Sigma_s^T = G with G_t = M (sum_{j>t} alpha_j
 * u_{t+1-j} + tau beta f_{t+1}); u0 is [s][nbar] (u_{1-s} first), and the
 * capacitance GMRES runs on the s x s block system J^(s) x = b^(s).
 * info may be NULL.  Synchronises the plan's stream. */
pd_status paradiag_solve(pd_plan plan, const double *u0, const double *F,
                         double *U, double tol, pd_info *info);

/* Solve `count` independent problems, each with its own plan.  Plans that
 * batch together -- 1D, uniform grid, float64 or float32 (not PD_MIXED),
 * backward Euler with the GMRES capacitance solver, the same precision and
 * maxit, no repeats -- form groups, and every stage of a group is one launch
 * for all of its problems (lockstep GMRES, each problem stopping on its own
 * convergence flag; a group's results equal the problems' results solved
 * alone, bit for bit).  Every other problem (2D, PD_MIXED, non-uniform
 * grids, BDF, the sine basis, Algorithm 2) and any group of one is solved
 * with paradiag_solve, one after another.  Arrays as in paradiag_solve, one
 * per problem.  infos may be NULL.  Synchronises each group's first plan's
 * stream. */
pd_status paradiag_solve_batch(const pd_plan *plans, int count,
                               const double *const *u0,
                               const double *const *F, double *const *U,
                               double tol, pd_info *infos);

pd_status paradiag_plan_destroy(pd_plan plan);

/* The launch configuration a plan uses: point pairs per time-transform
 * tile (*fft_C) and rows per thread of the shifted solves (*rows_per_thread;
 * 1D).  Either pointer may be NULL.  Errors: PD_EINVAL. */
pd_status paradiag_plan_config(pd_plan plan, int *fft_C, int *rows_per_thread);

/* Thread-local message describing the last failure ("" if none). */
const char *paradiag_last_error(void);

/* ---- components: one stage of Algorithm 1 each (for tests and tools) ---- */

/* Size in bytes of one half-spectrum array [ell/2+1][nbar] of this plan. */
size_t paradiag_spectrum_bytes(pd_plan plan);

/* First stage of Algorithm 1 (the right-hand side times D_alpha F^T,
 * Sections 2 and 4) WITHOUT the mass matrix:
 * Hhat_k = sum_t alpha^(t/ell) h_t exp(-2 pi i t k / ell), k = 0..ell/2,
 * with h_0 = u0 + tau f_1 and h_t = tau f_{t+1}.  (M commutes with the
 * time transform and is applied inside the shifted solves.)  BDF plans:
 * h_t = sum_{j=t+1}^{s} alpha_j u_{t+1-j} + tau beta f_{t+1}, u0 [s][nbar]. */
pd_status paradiag_forward_transform(pd_plan plan, const double *u0,
                                     const double *F, void *Hhat);

/* The parfor of shifted solves (Algorithm 1, first and second parfor):
 * for k = 0..ell/2,  Y_k = P_k^{-1} M (Hhat_k - w x),  w = alpha^(1/ell),
 * P_k = (1 - pi_k) M + tau K.  x may be NULL (= 0).
 * If Uhat != NULL, Y is written there (Uhat may equal Hhat).
 * If b != NULL, b = sum over the full spectrum k = 0..ell-1 of
 * gamma_k P_k^{-1} M Hhat_k (real, float64; x does not enter b), the
 * conjugate half being implied (Section 2, b = L F^{-T} e_ell).  At least one
 * of Uhat, b must be non-NULL.  BDF plans: P_k = (1 - pi_k) M + tau beta K
 * with pi_k the eigenvalues of C_s; only Uhat with x = NULL (PD_ENOTSUP
 * otherwise). */
pd_status paradiag_shifted_solve(pd_plan plan, const void *Hhat,
                                 const double *x, void *Uhat, double *b);

/* PD_SHIFTED_SINE plans: orthonormal DST-I along space of each of the ell
 * rows of a [ell][n] float64 array, out[t][k-1] = sqrt(2/(n+1)) sum_j
 * in[t][j-1] sin(pi j k/(n+1)), j, k = 1..n (the basis that diagonalises M
 * and K; Section 6.1 uses it along x in 2D).  out may equal in.
 * Errors: PD_EINVAL, PD_ENOTSUP (plan without the sine basis). */
pd_status paradiag_sine_transform(pd_plan plan, const double *in, double *out);

/* One capacitance product Jv = v + w sum_k gamma_k P_k^{-1} M v
 * (eq. SMW_linearsystemII; eq. innersystem_alpha), v and Jv float64 [nbar].
 * BDF plans: the block product J^(s) v (eq. linearsystem_s), block k =
 * v_k + sum_h sum_i gamma_i^(k) theta_i^(h) P_i^{-1} M v_h with
 * P_i = (1 - pi_i) M + tau beta K, v and Jv float64 [s][nbar]. */
pd_status paradiag_capacitance_apply(pd_plan plan, const double *v,
                                     double *Jv);

/* GMRES on J_ell x = b (BDF plans: J^(s), b and x [s][nbar]) from x = 0
 * until residual <= rtol * ||b|| or the plan's maxit.  iters and relres (may be NULL) receive the iteration count
 * and final residual / ||b||.  Returns PD_ENOTCONV if rtol was not met.
 * Synchronises the plan's stream. */
pd_status paradiag_capacitance_solve(pd_plan plan, const double *b,
                                     double *x, double rtol, int *iters,
                                     double *relres);

/* Last stage: U_t = alpha^(-t/ell) (1/ell) sum_{k=0}^{ell-1} Uhat_k
 * exp(+2 pi i t k / ell) with the conjugate half implied (U = Uhat F^{-T}
 * D_alpha^{-1}); the imaginary parts of Uhat_0 and Uhat_{ell/2} are taken as
 * zero.  U float64 [ell][nbar]. */
pd_status paradiag_inverse_transform(pd_plan plan, const void *Uhat,
                                     double *U);

/* Relative float64 residual ||G - A(U)||_F / ||G||_F of the all-at-once
 * system (Algorithm 3, residual test; BDF plans: eq. discrete_probBDF with
 * u0 [s][nbar]), written to *rel (host).
 * Synchronises the plan's stream. */
pd_status paradiag_residual(pd_plan plan, const double *u0, const double *F,
                            const double *U, double *rel);

/* For callers that cannot allocate device memory during the call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * paradiag_residual with no allocation at all.  The per-block partial norms
 * and their totals live in a file-scope device array of the library (at most
 * 8192 partial-norm blocks, 196,640 bytes, held on every GPU the library runs
 * on until the process ends; the plan's own reduction buffer is not used),
 * the totals are summed on the device in a fixed order, and three doubles
 * come back to the host.  Backward-Euler plans only (PD_ENOTSUP for
 * bdf_order > 1); PD_ENOTSUP with a message if a plan ever needed more blocks
 * than the array holds.  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (other streams, other threads) race.  Synchronises
 * the plan's stream. */
pd_status paradiag_residual_noalloc(pd_plan plan, const double *u0, const double *F,
                                    const double *U, double *rel);

/* ---- serving: continuous batching of independent solves ---------------- */

typedef struct pd_server_s *pd_server;

/* One request: the problem (as for paradiag_plan_create) and its device
 * arrays (as for paradiag_solve).  M may be NULL.  The arrays must stay
 * alive and untouched until the request completes. */
typedef struct {
  int n, ell;
  double tau;
  const pd_tridiag *M;
  const pd_tridiag *K;
  pd_options opt;              /* opt.stream is ignored (the server owns streams) */
  const double *u0;
  const double *F;
  double *U;
  double tol;
} pd_request;

/* Create a server with `workers` host threads, each owning one HIP stream on
 * the current device, that admits requests while the device memory it
 * accounts for (plan workspace of running and cached plans plus the requests'
 * u0, F and U) stays within budget_bytes.  Plans are cached by problem
 * (n, ell, tau, M, K, options) and keep their constants and Krylov workspace
 * on the device between requests; idle cached plans are evicted when the
 * budget needs room.  Work of different workers runs concurrently on the GPU.
 * Errors: PD_EINVAL, PD_ENOMEM, PD_EHIP. */
pd_status pd_server_create(pd_server *out, int workers, size_t budget_bytes);

/* Queue a request; returns at once with a ticket (>= 0).  PD_EBUDGET if the
 * request alone can never fit the budget.  The server copies *req (but not
 * the arrays). */
pd_status pd_server_submit(pd_server s, const pd_request *req, long *ticket);

/* Wait for ticket to finish (timeout_ms < 0: forever; 0: poll).  Returns
 * PD_OK with *done = 1 and the request's status/info when finished, *done = 0
 * on timeout.  info and status may be NULL. */
pd_status pd_server_wait(pd_server s, long ticket, int timeout_ms, int *done,
                         pd_status *status, pd_info *info);

/* Statistics: requests completed, peak accounted bytes, plan-cache hits and
 * misses, current accounted bytes.  Any pointer may be NULL. */
pd_status pd_server_stats(pd_server s, long *completed, size_t *peak_bytes,
                          long *cache_hits, long *cache_misses,
                          size_t *current_bytes);

/* Finish all queued work, free every plan and stream. */
pd_status pd_server_destroy(pd_server s);

/* ---- the serving admission policy, replayed on the host ---------------- */

/* One scripted event: op 0 = request `id` arrives and joins the FIFO queue
 * (with its problem identity `key` -- requests with equal keys can share a
 * cached plan -- its array bytes and its plan's workspace bytes); op 1 =
 * request `id`, which must be running, finishes (create_fails = 1: its plan
 * could not be created, so no plan joins the cache). */
typedef struct {
  int op;
  int id;
  int key;
  int create_fails;
  size_t io_bytes;
  size_t plan_bytes;
} pd_admission_event;

/* What happened to one request: admitted_after = index of the event after
 * which it was admitted (-1 never, -2 rejected at arrival because its arrays
 * and plan alone exceed the budget, PD_EBUDGET in the server); cache_hit = 1
 * if an idle cached plan was reused; evicted = idle plans evicted to admit it
 * (least recently used first) and first_victim_key the key of the first;
 * used_after = accounted bytes right after its admission. */
typedef struct {
  int admitted_after;
  int cache_hit;
  int evicted;
  int first_victim_key;
  size_t used_after;
} pd_admission_outcome;

/* Replay the admission and eviction policy of pd_server (the same policy
 * code, no device work) on nevents events with at most `workers` requests
 * running at once and a budget of budget_bytes.  outcomes has nreq entries,
 * indexed by request id; *peak_bytes (may be NULL) receives the largest
 * accounted total.  For tests and capacity planning.  Errors: PD_EINVAL
 * (bad arguments, an id out of range, a request arriving twice or
 * finishing while not running). */
pd_status pd_admission_replay(size_t budget_bytes, int workers, const pd_admission_event *events,
                              int nevents, pd_admission_outcome *outcomes, int nreq,
                              size_t *peak_bytes);

/* Device bytes a plan for this problem would allocate (workspace and
 * constants), without creating it. */
size_t paradiag_plan_bytes(int n, int ell, const pd_options *opt);

#ifdef __cplusplus
}
#endif

#endif /* PARADIAG_H */
