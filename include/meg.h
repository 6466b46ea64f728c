/*
 * meg.h - C ABI of the MI355X low-rank Matrix Exponentiated Gradient library.
 *
 * Method: D. Garber, A. Kaplan, "On the Efficient Implementation of the Matrix
 * Exponentiated Gradient Algorithm for Low-Rank Matrix Optimization"
 * (arXiv 2012.10469).  The library minimises a convex f over the spectrahedron
 * S_n = {X symmetric, X >= 0, tr X = 1} (Section 1, problem (1)) with the
 * low-rank MEG method (Section 3, Definition 1 and Algorithm 2): the iterate is
 * kept in the factored form X_t = alpha I + V diag(d) V^T of Section 3, each
 * step forms M_t = log X_t - eta grad f(X_t) implicitly, finds its top r + 1
 * eigenpairs by warm-started block subspace iteration with Rayleigh-Ritz
 * (Section 3, the subspace-iteration discussion), exponentiates and normalises
 * the top r, and evaluates the cheap convergence certificate with b_{r+1}
 * (Section 3.1.1 and Section 7).
 *
 * Conventions for every entry point:
 *  - Every call returns meg_status; no C++ exception crosses the ABI.
 *  - Pointers documented as DEVICE are HIP device pointers (e.g. a tensor's
 *    data_ptr()); they are BORROWED: the caller keeps them alive and unchanged
 *    until meg_destroy.  Pointers documented as HOST are read (or written)
 *    during the call only.
 *  - All device work is enqueued on the stream given to meg_init (a
 *    hipStream_t passed as void*; NULL = the default stream).  Calls that
 *    return host data synchronise that stream.
 *  - One host thread at a time per context.  After MEG_ERR_DEVICE the context
 *    is sticky-failed and further calls return MEG_ERR_STATE.
 *  - A certificate that does not hold is data, not an error (Section 7.4 shows
 *    it is expected without strict complementarity).
 */
#ifndef MEG_H
#define MEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct meg_ctx_s* meg_ctx;

typedef enum {
  MEG_OK = 0,
  MEG_ERR_INVALID_ARG = 1,   /* bad size, pointer, parameter or kind         */
  MEG_ERR_OUT_OF_MEMORY = 2, /* device allocation failed                     */
  MEG_ERR_DEVICE = 3,        /* a HIP call failed; the context is now failed */
  MEG_ERR_NUMERIC = 4,       /* a Ritz value or gradient became non-finite   */
  MEG_ERR_NOT_CONVERGED = 5, /* strict mode: inner solver hit max_inner      */
  MEG_ERR_STATE = 6,         /* context previously failed, or bad state blob */
  MEG_ERR_UNSUPPORTED = 7    /* valid but not implemented combination        */
} meg_status;

/* Arithmetic of the operator apply.  Small k x k solves (Gram matrices,
 * Rayleigh-Ritz, Cholesky, exponentiation, certificate) are always FP64. */
typedef enum {
  MEG_PREC_F64 = 0,       /* state and data in double                         */
  MEG_PREC_F32 = 1,       /* state and data in float                          */
  MEG_PREC_F32_BF16X3 = 2 /* float state; dense data given as two bf16 planes
                             hi + lo, applied with three bf16 MFMA products
                             (hi*hi + hi*lo + lo*hi) accumulated in FP32      */
} meg_precision;

/* Objective, i.e. how grad f(X_t) is represented (Section 3: the cost of a
 * step is dominated by multiplying the gradient with an n x k block; the
 * paper notes sparse and low-rank gradients make this cheaper). */
typedef enum {
  MEG_GRAD_LINEAR_DENSE = 0,  /* f = <C, X>;            C dense n x n          */
  MEG_GRAD_DENOISE_DENSE = 1, /* f = 1/2 ||X - M||_F^2; M dense n x n          */
  MEG_GRAD_LINEAR_CSR = 2,    /* f = <C, X>;            C sparse symmetric CSR */
  MEG_GRAD_MASKED_CSR = 3,    /* f = 1/2 sum_{(i,j) in Omega} (X_ij - M_ij)^2,
                                 Omega symmetric, both (i,j) and (j,i) stored;
                                 grad f = P_Omega(X - M)                       */
  MEG_GRAD_QUADMEAS = 4,      /* f = 1/(2m) sum_i (a_i^T X a_i - b_i)^2; each
                                 step uses the minibatch estimate
                                 (1/L) sum_{i in B_t} (a_i^T X a_i - b_i) a_i a_i^T
                                 (Section 6, stochastic oracle)                */
  MEG_GRAD_EXTERNAL = 5,      /* the caller supplies the gradient (or an
                                 unbiased estimate of it, Section 6) at X_t
                                 for every step: meg_step_external         */
  MEG_GRAD_BILINEAR = 6       /* f = 1/2 sum_i (tr(A_i^T X B_i) - y_i)^2, the
                                 recovery problem of Section 7 (A_i = a_i,
                                 B_i = b_i for rank-1 measurements), with its
                                 full gradient (symmetric part, Section 1)
                                 1/2 sum_i r_i (A_i B_i^T + B_i A_i^T),
                                 r_i = tr(A_i^T X B_i) - y_i                   */
} meg_grad_kind;

#define MEG_FLAG_STRICT 1u   /* inner non-convergence -> MEG_ERR_NOT_CONVERGED */
#define MEG_FLAG_NO_EXTRAPOLATE 4u /* F32 forms: end every step on a tested
                                      Rayleigh-Ritz sweep (by default a step
                                      may end on the block one power step past
                                      its last sweep when that sweep's
                                      residuals, contracted by the gap ratio
                                      theta_k / theta_i <= 0.05, predict the
                                      tolerance with a factor 2 to spare)   */
#define MEG_FLAG_NO_CHEBYSHEV 8u /* plain power steps.  By default every
                                    subspace sweep applies the Chebyshev
                                    polynomial of degree 1 for the interval
                                    [0, theta_k] (theta_k: the smallest Ritz
                                    value of the block, the last sweep's, or
                                    the last step's mu_k shifted as the new
                                    operator), i.e. (Yhat - theta_k/2) scaled:
                                    the unwanted part of the spectrum of the
                                    positive semidefinite Yhat maps into
                                    [-1, 1], halving the convergence exponent
                                    of pairs near the edge of that part       */
#define MEG_FLAG_DUAL_AVERAGE 16u /* the dual-averaging reading of the step
                                     (the accumulate-forever form): the
                                     log-domain matrix is kept dense and
                                     accumulated, Y_1 = log X_1, Y_{t+1} =
                                     Y_t - eta grad f(X_t), and X_{t+1} is
                                     formed from the top-r eigenpairs of
                                     Y_{t+1} as Definition 1 forms it from
                                     those of M_t = log X_t - eta grad f(X_t)
                                     (which rebuilds log X_t from the
                                     factored iterate).  The two agree for
                                     linear f with a start on eigenvectors of
                                     C and differ otherwise.  Dense linear or
                                     denoising objectives, F64 or F32 (n x n
                                     of the state's type for Y, allocated by
                                     meg_init); each step first updates Y
                                     (one pass, with Gershgorin bounds for
                                     the shift), then decomposes Y + sigma' I
                                     with the dense apply.  meg_set_iterate
                                     restarts Y at log X; meg_set_state,
                                     meg_profile_step, meg_trace_exp,
                                     meg_certificate_bound and
                                     meg_solve_to_gap return
                                     MEG_ERR_UNSUPPORTED, as meg_init does for
                                     other objectives                        */
#define MEG_FLAG_NO_LDS_CACHE 2u /* CSR kinds: read the sparse data from global
                                    memory in every sweep instead of keeping each
                                    workgroup's rows in LDS (the cache is used
                                    only when it fits; results are the same)  */

typedef struct {
  int64_t n;          /* dimension, n >= k (see meg_block_size)               */
  int32_t r;          /* rank parameter, 1 <= r <= n - 1 (Algorithm 2)        */
  int32_t oversample; /* p >= 0; block size k = roundup16(r + 1 + p) <= 32    */
  int32_t prec;       /* meg_precision                                        */
  int32_t min_inner;  /* subspace sweeps per step: at least (>= 1) ...        */
  int32_t max_inner;  /* ... and at most (>= min_inner, <= 64)               */
  uint32_t flags;     /* MEG_FLAG_*                                           */
  double eta;         /* step size eta_t = eta > 0 (Algorithm 2 input)        */
  double eps_scale;   /* eps_t = eps_scale / (t + eps_c + 1)^eps_pow, t >= 0; */
  double eps_c;       /* Section 7 uses 0.8, 10, 2.  eps_0 must lie in        */
  double eps_pow;     /* (0, 3/4] (the approximation-error lemma's range).    */
  double inner_tol;   /* residual tolerance of the top-r Ritz pairs relative
                         to the largest Ritz value; 0 selects 1e-10 (F64) or
                         1e-6 (F32 forms).  Residuals are estimated from FP64
                         Gram matrices, which resolve them down to about
                         3e-8 of the scale.  Below that, an F64 state also
                         tests the explicit residuals ||Y q_i - theta_i q_i||
                         of the previous sweep's pairs (formed by the next
                         apply from its rows, down to ~1e-14 of the scale);
                         the F32 forms run two more sweeps instead once the
                         estimate reaches its floor.                           */
  uint64_t seed;      /* seeds the solver's extra start columns               */
  double cert_tol;    /* the (r+1)-th Ritz pair, whose value mu_{r+1} enters the
                         certificate (Section 3.1.1).  Its Ritz value is a lower
                         bound of mu_{r+1} (interlacing) and cert_L does not
                         decrease with mu_{r+1}, so cert_L from the Ritz
                         values is a lower bound of the exact L: enough to rule
                         a certificate out.  The pair counts as resolved when
                         its residual rho_{r+1} meets the tolerance (cert_tol
                         > 0, else the top pairs') and is at most a quarter of
                         the gap to the next Ritz value; cert_L + rho_{r+1} is
                         then an upper bound, and cert_holds and the stopping
                         rules act on it, never on an unresolved pair.
                         cert_tol > 0: each step iterates until the pair is
                         resolved (or max_inner).  cert_tol <= 0: no sweeps
                         are spent on it, except by meg_solve (and a server)
                         while the lower bound could meet their tol.        */
} meg_params;

typedef struct {
  int32_t kind;  /* meg_grad_kind */
  int32_t batch; /* QUADMEAS: minibatch size L (>= 1); BILINEAR: columns p of
                    each measurement matrix (0 or 1: rank-1 measurements)     */
  /* dense kinds: DEVICE, n x n symmetric, row-major with leading dimension
   * ld >= n; element type double (F64) or float (F32).  F32_BF16X3: `dense`
   * is the bf16 hi plane and `dense_lo` the bf16 lo plane (hi + lo ~ M). */
  const void* dense;
  const void* dense_lo;
  int64_t ld;
  /* CSR kinds: DEVICE, symmetric pattern, int32 row_ptr[n+1], col[nnz]
   * (sorted within each row), values val[nnz] in the state's type. */
  const int32_t* row_ptr;
  const int32_t* col;
  const void* val;
  int64_t nnz;
  /* QUADMEAS: DEVICE pool A (m rows of length lda >= n: row i is a_i, in
   * the state's type; A 16-byte aligned and lda * sizeof(type) a multiple of
   * 16), b[m], and the minibatch indices batch_idx[batch_steps * batch]
   * (int32 in [0, m), checked by meg_init; 1 <= batch <= 1024); step t uses
   * row (t - 1) mod batch_steps.  The indices are an input so that a run is
   * reproducible.  F64 and F32 only (the bf16-plane form is dense-only).
   * Each step also forms the batch x batch Gram matrix of its minibatch to
   * bound the spectrum of the gradient estimate (the solver's shift). */
  /* BILINEAR: measurements tr(A_i^T X B_i) with A_i, B_i n x p (p = `batch`,
   * 0 or 1 for a_i^T X b_i; at most 4096).  DEVICE A holds 2mp rows of length
   * lda >= n in the state's type (F64 or F32): row i p + q is column q of A_i,
   * row m p + i p + q column q of B_i; b holds y[m].  Every step forms
   * the residuals and the dense symmetric gradient (n x n, owned by the
   * context) on the device, then takes the step as meg_step_external would
   * with it.  The trace bound of Section 7 is 1: for tr X = tau pass y / tau
   * and eta * tau (the iterates are then X / tau). */
  const void* A;
  int64_t lda;
  const void* b;
  int64_t m;
  const int32_t* batch_idx;
  int64_t batch_steps;
} meg_objective;

typedef struct {
  int32_t q;              /* number of start columns, 1 <= q <= r              */
  int32_t reserved;
  const double* V0;       /* HOST, n x q column-major, orthonormal columns     */
  const double* lambda0;  /* HOST, q weights >= 0 summing to 1: X_0 = V0 diag(lambda0) V0^T */
} meg_start;

typedef struct {
  int64_t t;          /* iteration index t of the step just taken (gradient at X_t) */
  double f;           /* f(X_t) when requested, else NaN                      */
  double eps_t;       /* approximation parameter used to form X_{t+1}         */
  double cert_L;      /* log((n-r) lambda_{r+1}(Y_t) / (eps_t b^{r+1}_t)) from
                         the Ritz values: a lower bound of the exact value,
                         and within resid_r1 of it when cert_resolved        */
  double cert_bound;  /* max(2 eps_t, cert_L): bound of the error lemma       */
  int32_t cert_holds; /* cert_L_up <= 2 eps_t: the exact certificate holds   */
  int32_t inner_iters;/* subspace sweeps used                                 */
  double ritz_gap;    /* mu_r - mu_{r+1} (eigenvalues of M_t)                 */
  double resid_max;   /* max Ritz residual over the top r pairs               */
  double mu_r1;       /* mu_{r+1}                                             */
  double sigma;       /* spectral shift used by the solver                    */
  int32_t converged;  /* inner solver met its tolerance                       */
  int32_t cert_resolved; /* the (r+1)-th Ritz pair is resolved (cert_tol)   */
  double resid_r1;    /* residual bound of the (r+1)-th Ritz pair; resolved:
                         the exact L lies in [cert_L, cert_L + resid_r1]     */
  double cert_L_up;   /* upper bound of the exact L on which cert_holds and
                         the stopping rules act: cert_L + resid_r1 for a
                         resolved pair, or the bound armed by
                         meg_certificate_bound for this step (the smaller);
                         +inf without either                                 */
  double mu_r1_up;    /* the upper bound of mu_{r+1} behind cert_L_up         */
} meg_step_info;

/* Block size k used for (r, oversample); returns 0 when k would exceed 32. */
int32_t meg_block_size(int32_t r, int32_t oversample);

/* Create a context: validate, allocate device state, build the first iterate
 * X_1 = (1 - eps_0) X_0 + (eps_0/n) I (Algorithm 2, initialisation).  The
 * objective's device arrays are borrowed.  *out is NULL on failure. */
meg_status meg_init(meg_ctx* out, const meg_params* params, const meg_objective* obj,
                    const meg_start* start, void* stream);

/* One iteration t of Algorithm 2: X_t -> X_{t+1}.  info == NULL: enqueue only
 * (asynchronous; f is not evaluated).  info != NULL: also evaluate f(X_t),
 * synchronise and fill *info. */
meg_status meg_step(meg_ctx ctx, meg_step_info* info);

/* One iteration t of Algorithm 2 with a caller-supplied gradient G_t at the
 * current iterate X_t (read it with meg_get_iterate), for a context created
 * with kind MEG_GRAD_EXTERNAL: M_t = log X_t - eta G_t.  `grad` describes
 * G_t as a symmetric operator: kind MEG_GRAD_LINEAR_DENSE (dense, ld) or
 * MEG_GRAD_LINEAR_CSR (row_ptr, col, val, nnz), in the state's type (F64 or
 * F32; the bf16-plane form is not offered here).  Its DEVICE arrays are
 * read during the call only: the call synchronises the stream before it
 * returns.  The solver's shift bounds lambda_max(G_t) by Gershgorin's
 * theorem (one pass over G_t).  info (optional) as meg_step, with f = NaN.
 * Errors: MEG_ERR_INVALID_ARG for a context of another kind, a NULL or
 * malformed grad (ld < n, CSR structure or column out of range; checked
 * before any kernel reads through it), MEG_ERR_UNSUPPORTED for another grad
 * kind.  meg_step, meg_solve and meg_profile_step return MEG_ERR_INVALID_ARG
 * on an external context, meg_objective_value MEG_ERR_UNSUPPORTED (f is the
 * caller's). */
meg_status meg_step_external(meg_ctx ctx, const meg_objective* grad, meg_step_info* info);

/* Up to max_iters iterations; stops early after the first step whose
 * certificate bound max(2 eps_t, cert_L) is <= tol (tol <= 0: never).
 * *last (optional) receives the last step's info (f = NaN). */
meg_status meg_solve(meg_ctx ctx, int64_t max_iters, double tol, meg_step_info* last);

/* Info of the most recent step (certificate, eps_t, gap ...); no kernel runs. */
meg_status meg_certificate(meg_ctx ctx, meg_step_info* out);

/* f at the current iterate X_t (one pass over the data). */
meg_status meg_objective_value(meg_ctx ctx, double* f);

/* Current iterate X_t = alpha I + V diag(d) V^T.  HOST outputs: V n x r
 * column-major, d[r]; any output may be NULL. */
meg_status meg_get_iterate(meg_ctx ctx, double* V, double* d, double* alpha, int64_t* t);

/* Replace the iterate by X = alpha I + V diag(d) V^T with q <= r HOST columns
 * (orthonormal), 0 < alpha, alpha + d_i > 0, and set the iteration index to t
 * (so the next step uses eps_t).  Used for teacher-forced comparisons. */
meg_status meg_set_iterate(meg_ctx ctx, const double* V, int32_t q, const double* d, double alpha,
                           int64_t t);

/* Serialise / restore the full solver state (iterate, warm-start basis and
 * counters) for bitwise resume.  meg_get_state with buf == NULL sets *bytes. */
meg_status meg_get_state(meg_ctx ctx, void* buf, size_t* bytes);
meg_status meg_set_state(meg_ctx ctx, const void* buf, size_t bytes);

/* Timing of one step (measurement entry point).  Runs one full iteration
 * t -> t+1 exactly as meg_step does (one launch of the persistent step
 * kernel) with a HIP event pair around the launch on the context's stream,
 * and with the kernel stamping the device wall clock at each of its grid
 * barriers; synchronises.  HOST output; times in milliseconds. */
typedef struct {
  double kernel_ms;      /* the step kernel, HIP events around the launch    */
  double prep_ms;        /* work before the first sweep (0: the step scalars
                            are set at the end of the previous step and the
                            masked gradient is formed within sweep 1)        */
  double apply_ms[64];   /* sweep s: operator apply + Gram partials; sweep 1
                            of the masked objective also forms the gradient  */
  double small_ms[64];   /* sweep s: partial reduction + Rayleigh-Ritz/QR    */
  double finalize_ms;    /* next basis + its orthonormalising transform      */
  int32_t sweeps_active; /* sweeps the step used                             */
  int32_t workgroups;    /* persistent grid size                             */
  /* sweeps 1 and 2 (zero when not run), per workgroup: */
  double wg_apply_ms[2][3]; /* time from the workgroup's start of the sweep to
                               its arrival at the sweep's barrier: min, mean, max */
  double wg_skew_ms[2];     /* spread of the workgroups' start times          */
  double reduce_ms[2];      /* last arrival -> start of the small solve (the
                               partial sums reduced along the barrier tree)  */
  /* first Rayleigh-Ritz sweep of the step: */
  double rr_ms[3];          /* before the eigensolver (loads, T = W^T C), the
                               Jacobi eigensolver, sort + residuals + test   */
  double rr_tail_ms;        /* the rest: next transform, or the step's end  */
  int32_t jacobi_sweeps;    /* Jacobi sweeps it took                          */
  int32_t reserved;
} meg_kernel_times;

meg_status meg_profile_step(meg_ctx ctx, meg_kernel_times* out);

/* Work and time counters of the step kernel (measurement entry point),
 * accumulated over every launch made by meg_step, meg_solve and
 * meg_profile_step since meg_init or the last reset.  Each launch is
 * bracketed by a HIP event pair on the context's stream; kernel_ms is the sum
 * of those elapsed times.  Synchronises the stream.  HOST output.
 * reset != 0: the counters restart from zero after being read.  The work
 * counters travel with the context, not with a state blob (meg_set_state
 * keeps them). */
typedef struct {
  int64_t launches;    /* step-kernel launches                                */
  int64_t iterations;  /* iterations t -> t+1 they performed                  */
  int64_t applies;     /* operator applies (subspace sweeps) they performed   */
  int32_t workgroups;  /* persistent grid size                                */
  int32_t jacobi_sweeps; /* Jacobi sweeps of their Rayleigh-Ritz solves
                            (saturates at INT32_MAX)                          */
  double kernel_ms;    /* GPU time of those launches, milliseconds            */
  int64_t extrapolated; /* iterations that ended on the extrapolated block     */
  int64_t unconverged;  /* iterations whose top pairs missed the tolerance at
                           max_inner                                        */
} meg_counters;

meg_status meg_get_counters(meg_ctx ctx, meg_counters* out, int32_t reset);

/* Dual gap at the current iterate X_t (Section 7, the near-optimality measure
 * of the experiments): with G = grad f(X_t) and trace bound 1,
 *   gap = max_{Z >= 0, tr Z = 1} <X_t - Z, G> = <X_t, G> - lambda_min(G),
 * which bounds f(X_t) - f* from above for convex f.  <X_t, G> is accumulated
 * in FP64 over the matrix (dense) or the pattern (CSR); lambda_min(G) is the
 * smallest Ritz value of a Lanczos run with full reorthogonalisation on G
 * (FP64 basis, recurrence and products on the device; the host solves the
 * small tridiagonal problem), started from the previous call's lambda_min
 * Ritz vector plus 1e-3 of a seeded Gaussian vector (the Gaussian vector
 * alone on the first call), stopped once its Ritz residual
 * is <= tol * max |Ritz value| (checked every 8 steps) or after max_steps
 * steps.  Allocates its Lanczos basis ((max_steps + 1) x n doubles) for the
 * call.  Objectives: linear (G = C), denoising
 * (G = X_t - M, also with M as bf16 planes) and masked (G = P_Omega(X_t - M);
 * the call overwrites the context's stored gradient values, which the next
 * step recomputes).  MEG_ERR_UNSUPPORTED for the minibatch and external
 * kinds; MEG_ERR_INVALID_ARG for max_steps < 1, tol < 0 or out == NULL.
 * Synchronises; HOST output. */
typedef struct {
  double gap;         /* <X_t, G> - lambda_min                                  */
  double x_dot_g;     /* <X_t, G>                                                */
  double lambda_min;  /* smallest Ritz value of G                                */
  double resid;       /* its Ritz residual ||G s - theta s|| (|beta_m s_m|)      */
  int64_t t;          /* index of the iterate                                    */
  int32_t steps;      /* Lanczos steps taken                                     */
  int32_t converged;  /* resid <= tol * max |Ritz value|                         */
} meg_dual_gap_info;

meg_status meg_dual_gap(meg_ctx ctx, int32_t max_steps, double tol, meg_dual_gap_info* out);

/* meg_dual_gap for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, with the Lanczos workspace in a fixed device array
 * of the library (32 MiB per GPU, held until the process ends) instead of
 * the context's workspace, and a fresh seeded start vector (no warm start
 * from an earlier call), so calls are independent of each other.  Needs
 * (min(n, max_steps) + 1) n + 3 n + 3 min(n, max_steps) + 33 doubles <=
 * 4 Mi (4194304); MEG_ERR_INVALID_ARG beyond that (and as meg_dual_gap).
 * Allocates nothing on the device.  Every call on one GPU uses that GPU's
 * one array: calls that overlap on a GPU (from several host threads or
 * streams) race, and must be serialised by the caller.  Synchronises. */
meg_status meg_dual_gap_static(meg_ctx ctx, int32_t max_steps, double tol, meg_dual_gap_info* out);

/* An upper bound of mu_{r+1}, the (r+1)-th eigenvalue of M_t = log X_t -
 * eta grad f(X_t) at the CURRENT iterate (the matrix the next meg_step
 * decomposes), for the certificate of Section 3.1.1.  log X_t = log(alpha) I
 * + V diag(c) V^T vanishes on the orthogonal complement of V beyond the
 * identity, so by the Courant-Fischer theorem
 *   mu_{r+1} <= log alpha - eta lambda_min(G restricted to V's complement);
 * that lambda_min comes from a Lanczos run on the complement (the run of
 * meg_dual_gap with every vector also orthogonalised against V), lowered by
 * its Ritz residual.  The bound is armed for the next step: its cert_L_up
 * (hence cert_holds and meg_solve's stop) may use it.  It is sharp when V
 * spans the top-r eigenvectors of M_t, i.e. once the iterates settle.
 * Objectives as meg_dual_gap; MEG_ERR_INVALID_ARG for max_steps < 1, tol < 0
 * or out == NULL.  Uses the context's Lanczos workspace.  Synchronises. */
typedef struct {
  double mu_up;           /* the bound                                          */
  double lambda_min_defl; /* smallest Ritz value of G on V's complement          */
  double resid;           /* its Ritz residual                                   */
  int64_t t;              /* the iteration whose step it is armed for            */
  int32_t steps;          /* Lanczos steps taken                                 */
  int32_t converged;      /* resid <= tol * max |Ritz value|                     */
} meg_cert_bound_info;

meg_status meg_certificate_bound(meg_ctx ctx, int32_t max_steps, double tol, meg_cert_bound_info* out);

/* Iterate until the dual gap of the current iterate is <= tol (the stopping
 * rule of Section 7's measure) or max_iters iterations are done: the gap is
 * evaluated first, then after every check_every iterations (1..64, launched
 * together) as meg_dual_gap(ctx, 256, 1e-8, .) does.  *last (optional) as
 * meg_solve's; *gap (optional) the last evaluation.  Objectives as
 * meg_dual_gap (MEG_ERR_UNSUPPORTED otherwise); MEG_ERR_INVALID_ARG for
 * max_iters < 0, tol <= 0 or check_every outside 1..64.  Synchronises. */
meg_status meg_solve_to_gap(meg_ctx ctx, int64_t max_iters, double tol, int32_t check_every, meg_step_info* last,
                            meg_dual_gap_info* gap);

/* The sum b_n = tr exp(M_t) of all eigenvalues of Y_t = exp(M_t), for the
 * all-eigenvalue form of the certificate (Section 3.1.1: the approximation-
 * error lemma's condition uses b_n; the cheap certificate of meg_step uses
 * b^{r+1} <= b_n instead), following the randomised route the section
 * mentions: quadratic forms u^T exp(M_t) u from Lanczos runs, averaged over
 * probe vectors.  M_t = log X_t - eta grad f(X_t) at the CURRENT iterate X_t,
 * i.e. the matrix the next meg_step decomposes.
 *
 * The estimate splits the trace by the context's k-column solver block Q
 * (orthonormalised in FP64): with P = I - Q Q^T,
 *   b_n = tr(Q^T exp(M_t) Q) + tr(P exp(M_t) P)    (exact for any orthonormal Q);
 * the first term is computed, the second estimated as
 *   weight * sum_j (P u_j)^T exp(M_t) (P u_j)
 * over the caller's probes u_j (the deflation of Hutch++, Meyer et al.,
 * 2021).  weight = 1/p with Gaussian or Rademacher probes gives an unbiased
 * estimate; the n canonical basis vectors with weight = 1 give b_n itself.
 * Each quadratic form v^T exp(M_t) v is ||v||^2 e_1^T exp(T) e_1 for the
 * tridiagonal T of a Lanczos run from v (Gauss quadrature, with the plain
 * three-term recurrence: Lanczos for matrix functions is stable without
 * reorthogonalisation, Musco, Musco and Sidford, 2018): the runs
 * advance 64 vectors at a time in lockstep on the device (FP64 vectors, the
 * operator's data in the state's type), and stop when every estimate has
 * changed by at most tol (relative) over the last 8 steps, or after
 * max_steps steps; the host evaluates e_1^T exp(T) e_1 from T's eigenvalues
 * and first eigenvector components.
 *
 * probes: DEVICE, n x p column-major FP64 (probe j at probes + j * n), read
 * during the call only; p >= 0 (p = 0: the deflated term alone, a lower
 * bound of b_n).  weight > 0.  Objectives as meg_dual_gap (linear,
 * denoising, also with bf16 planes, and masked; the call overwrites the
 * masked kind's stored gradient values, which the next step recomputes);
 * MEG_ERR_UNSUPPORTED for the minibatch and external kinds;
 * MEG_ERR_INVALID_ARG for p < 0, p > 0 with probes == NULL, weight <= 0,
 * max_steps < 1, tol < 0 or out == NULL.  Its device workspace (five blocks
 * of 64 x n doubles, 2 x 64 x max_steps and small buffers) belongs to the
 * context: allocated by the first call, grown when a later call needs more,
 * freed by meg_destroy (MEG_ERR_OUT_OF_MEMORY when it cannot be allocated).
 * Synchronises; HOST output. */
typedef struct {
  double log_b;           /* log of the estimate of b_n = tr exp(M_t)          */
  double log_b_defl;      /* log tr(Q^T exp(M_t) Q)                             */
  double log_b_tail;      /* log of the probe estimate of tr(P exp(M_t) P);
                             -inf for p = 0 or when every P u_j is zero        */
  double tail_rel_stderr; /* standard error of the probe estimate (weight *
                             sqrt(p) * sample std of the p terms) divided by
                             the estimate of b_n; NaN for p < 2                */
  int64_t t;              /* index of the iterate                               */
  int32_t kd;             /* deflation columns kept (rank of the block)         */
  int32_t steps;          /* Lanczos steps of the longest run                   */
  int32_t converged;      /* every quadrature met tol                           */
  int32_t batches;        /* lockstep batches of up to 64 vectors               */
} meg_trace_info;

meg_status meg_trace_exp(meg_ctx ctx, const double* probes, int32_t p, double weight, int32_t max_steps, double tol,
                         meg_trace_info* out);

/* The certificate with an estimate of b_n in place of b^{r+1} (Section 3.1.1):
 *   L_full = log((n - r) lambda_{r+1}(Y_t) / (eps_t b_n))
 *          = log(n - r) + mu_{r+1} - log eps_t - log_b,
 * from the most recent step's mu_{r+1} (its Ritz value, a lower bound) and
 * eps_t and tr->log_b, which must be the estimate for that step's M_t
 * (meg_trace_exp called at the iterate the step started from: tr->t equals
 * the step's t).  *holds = 1 when L_full with the step's upper bound of
 * mu_{r+1} (meg_step_info.mu_r1_up) is <= 2 eps_t; never without one.
 * MEG_ERR_INVALID_ARG when no step has run since, when tr->t differs, or for
 * NULL pointers.  No kernel runs. */
meg_status meg_certificate_full(meg_ctx ctx, const meg_trace_info* tr, double* cert_L_full, int32_t* holds);

void meg_destroy(meg_ctx ctx);
const char* meg_status_str(meg_status s);

/* ---------------------------------------------------------------------------
 * Exact MEG (Algorithm 1, the mirror step of Section 2.2), the baseline the
 * experiments compare the low-rank method with (Section 7): dense n x n FP64
 * iterates W_{t+1} = exp(log W_t - eta grad f(W_t)) / tr(...).  With a
 * constant step size log W_t accumulates the gradients up to multiples of
 * I, so the library keeps Y_t (Y_1 = log W_1, Y_{t+1} = Y_t - eta grad
 * f(W_t)) and forms W_{t+1} = exp(Y_{t+1}) / tr exp(Y_{t+1}) by scaling and
 * squaring (Gershgorin bounds of Y for the shift and scaling, a degree-12
 * Taylor polynomial, GEMMs).  W_1 = (1 - eps_0) X_0 + (eps_0/n) I, the
 * low-rank method's first iterate for the same params and start.
 * Objectives: MEG_GRAD_LINEAR_DENSE and MEG_GRAD_DENOISE_DENSE with the
 * DEVICE FP64 matrix C or M (borrowed until meg_exact_destroy); params:
 * n (2..8192), prec MEG_PREC_F64, eta, the eps schedule (eps_0 only).
 * Allocates five n x n FP64 matrices.  All work on `stream`; calls
 * synchronise.  One host thread at a time per handle.
 * ------------------------------------------------------------------------- */
typedef struct meg_exact_s* meg_exact;

typedef struct {
  int64_t t;  /* iteration t of the step just taken (gradient at W_t) */
  double f;   /* f(W_t)                                                */
} meg_exact_info;

meg_status meg_exact_create(meg_exact* out, const meg_params* params, const meg_objective* obj,
                            const meg_start* start, void* stream);
/* One iteration t of Algorithm 1: W_t -> W_{t+1}. */
meg_status meg_exact_step(meg_exact h, meg_exact_info* info);
/* HOST W n x n row-major (optional) and the index t of the current W_t. */
meg_status meg_exact_get(meg_exact h, double* W, int64_t* t);
/* The Bregman distance of Section 2.2, B(W_t, X) = tr(W_t log W_t - W_t log X),
 * between the current exact iterate and a factored X = alpha I + V diag(d) V^T
 * (HOST V n x r column-major with orthonormal columns, d[r], alpha > 0, as
 * meg_get_iterate returns it): the experiments' distance between the exact
 * and the low-rank iterates.  log X from its closed form, tr(W log W) from
 * Y, so no eigendecomposition runs. */
meg_status meg_exact_bregman(meg_exact h, const double* V, int32_t r, const double* d, double alpha, double* out);
void meg_exact_destroy(meg_exact h);

/* ---------------------------------------------------------------------------
 * Batched serving: many independent instances of the dense denoising or
 * linear objective (Section 1, problem (1); Algorithm 2 for each) advanced
 * together by one persistent, cooperatively launched kernel.  Each launch
 * runs every resident instance for up to `launch_steps` iterations on its
 * own team of workgroups, with its own barrier words and partial sums, so
 * an instance's arithmetic does not depend on what else is resident: its
 * result is bitwise the same alone and in a mix.  Between launches the
 * server retires finished instances (results copied to the host, device
 * memory returned) and admits queued requests in arrival order as soon as
 * a free team of workgroups and room in its device arena allow (admission
 * by memory footprint: the bf16 planes of M, three n x k blocks, the
 * control block and the reduction buffers).  The operator apply is the
 * BF16x3 matrix-core form (FP32 state); M is split into its bf16 planes
 * once, at admission.  The team size per n is chosen by a built-in
 * autotuner that times the step kernel on a synthetic instance of that n
 * with each candidate size: the latency choice is the smallest team within
 * 15 % of the fastest, the throughput choice the team with the least
 * workgroup time per iteration; a request is admitted with the throughput
 * choice while others wait in the queue behind it, else with the latency
 * choice.  (Results depend on the team size only through the order of the
 * partial sums, i.e. within rounding.)
 * The solver's shift uses Gershgorin bounds of the planes' matrix (one pass
 * at admission) instead of the single-instance path's Lanczos estimate.
 * One host thread at a time per server; all work runs on its stream.
 * ------------------------------------------------------------------------- */
typedef struct meg_server_s* meg_server;

#define MEG_SERVER_FLAG_GRAPH 1u /* each scheduling round replays one captured
                                    hipGraph: the slot and team tables and the
                                    launch parameters copied from pinned host
                                    memory, the batched kernel over the whole
                                    workgroup capacity (workgroups without a
                                    team exit), the summary and its read-back;
                                    results are those of direct launches.
                                    Needs a stream other than NULL           */

typedef struct {
  int64_t budget_bytes;  /* device arena for resident instances; 0: 4 GiB   */
  int32_t launch_steps;  /* iterations per launch of the fastest resident
                            instance, 1..1024; slower ones run fewer (>= 1)
                            so that all teams finish a launch together (by
                            the autotuner's time per step); the launch is
                            the admission granularity                      */
  int32_t max_resident;  /* instances resident at once, 1..256            */
  uint32_t flags;        /* MEG_SERVER_FLAG_*                               */
  int32_t fixed_team;    /* > 0: every instance runs on this many workgroups
                            (at most one 64-row block each) instead of the
                            autotuner's choice; 0: autotune                */
} meg_server_params;

typedef struct {
  int32_t kind;          /* MEG_GRAD_DENOISE_DENSE or MEG_GRAD_LINEAR_DENSE  */
  int32_t r;             /* 1 <= r, with r + 1 + oversample <= 16           */
  int64_t n;             /* 16 <= n <= 32768                               */
  const float* M;        /* DEVICE n x n row-major FP32 (C or M), leading
                            dimension ld >= n.  BORROWED until the request
                            leaves the queue (state >= 1): it is split into
                            bf16 planes at admission                        */
  int64_t ld;
  int32_t q;             /* start columns, 1 <= q <= r                      */
  int32_t max_iters;     /* iteration cap, >= 1                            */
  const double* V0;      /* HOST n x q column-major orthonormal; copied     */
  const double* lambda0; /* HOST q weights >= 0 summing to 1; copied        */
  double eta;            /* step size > 0                                  */
  double eps_scale, eps_c, eps_pow; /* as in meg_params                    */
  double tol;            /* stop after the first step with
                            max(2 eps_t, cert_L) <= tol (<= 0: never)      */
  int32_t oversample;    /* p >= 0                                         */
  int32_t max_inner;     /* subspace sweeps per step, 1..64                 */
  uint64_t seed;         /* seeds the extra start columns                   */
} meg_request;

typedef struct {
  int32_t state;         /* 0 queued, 1 resident, 2 done, 3 failed          */
  int32_t status;        /* meg_status of a failed request, else MEG_OK      */
  int64_t iterations;    /* iterations performed                           */
  double submit_ms;      /* server clock (ms since meg_server_create) at
                            submission, admission and retirement            */
  double admit_ms;
  double done_ms;
  int32_t team;          /* workgroups of its team (resident or done)       */
  int32_t reserved;
  meg_step_info last;    /* last step's info (f = NaN)                      */
  int64_t applies;       /* operator applies (subspace sweeps) performed    */
} meg_request_status;

typedef struct {
  int64_t submitted, completed, failed;
  int64_t launches;      /* serving-kernel launches                        */
  int64_t iterations;    /* iterations over all instances                  */
  double kernel_ms;      /* summed HIP-event time of the serving launches   */
  int32_t resident, queued;
  int32_t capacity_wg;   /* co-resident workgroups of the serving kernel    */
  int32_t graph_node;    /* graph mode: 0 not captured yet, 1 the captured
                            kernel node is a cooperative launch, 2 an
                            ordinary launch of at most capacity_wg         */
  int64_t arena_bytes, arena_used, arena_peak;
} meg_server_stats;

meg_status meg_server_create(meg_server* out, const meg_server_params* params, void* stream);
/* Queue a request (validated here); *id identifies it from now on. */
meg_status meg_server_submit(meg_server s, const meg_request* req, int64_t* id);
/* `rounds` scheduling rounds: retire finished instances, admit queued
 * requests, launch the serving kernel once (if anything is resident) and
 * wait for it.  *pending (optional) = resident + queued requests after. */
meg_status meg_server_run(meg_server s, int32_t rounds, int32_t* pending);
meg_status meg_server_query(meg_server s, int64_t id, meg_request_status* out);
/* Result of a done request: HOST V n x r column-major, d[r], alpha (any may
 * be NULL), as meg_get_iterate. */
meg_status meg_server_result(meg_server s, int64_t id, double* V, double* d, double* alpha);
/* Forget a done or failed request (its host result). */
meg_status meg_server_release(meg_server s, int64_t id);
/* Team sizes for dimension n (autotuned on first use): latency and
 * throughput choices (either pointer may be NULL). */
meg_status meg_server_team(meg_server s, int64_t n, int32_t* latency_team, int32_t* throughput_team);
meg_status meg_server_get_stats(meg_server s, meg_server_stats* out);
void meg_server_destroy(meg_server s);

#ifdef __cplusplus
}
#endif
#endif /* MEG_H */
