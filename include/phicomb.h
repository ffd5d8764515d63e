/*
 * phicomb.h -- C ABI of the MI355X (gfx950) library for linear combinations
 * of phi-function actions,
 *
 *     w_i = sum_{j=0..p} beta_ij phi_j(t_i A) v_j,   i = 1..r,
 *
 * by the block truncated-Taylor scaling-and-recovering method of
 * A. H. Al-Mohy, "Computing Linear Combinations of phi-Function Actions for
 * Exponential Integrators" (arXiv 2509.26475).  The paper's problem statement
 * is Sec. 1, eq. (phi.comb), with beta_ij = alpha_i^j; phi_j is defined in
 * eq. (def.phik).  Any weight table beta is accepted (Corollary of Theorem 1:
 * the weights are folded into the columns of V).
 *
 * Conventions
 *  - Every function returns an int status: PHICOMB_OK (0), PHICOMB_PENDING
 *    (1, phicomb_poll only) or a negative error.  No exception crosses the
 *    ABI; phicomb_strerror() names a status.
 *  - "host" pointers are ordinary CPU memory, read during the call only.
 *    "device" pointers are HIP device memory of the current device; the
 *    caller owns them and keeps them alive until the call returns (solve) or
 *    until phicomb_poll returns something other than PHICOMB_PENDING.
 *  - Matrices are row-major.  V is [n][p+1] in natural order v_0..v_p; W is
 *    [n][r].  Everything is IEEE double unless stated.
 *  - The spectral shift is called xi* in the paper (Sec. 3, Algorithm 1); the
 *    field is named "shift".  (The paper's mu is the undo factor
 *    exp(t xi/s) of Sec. 3, eq. (rec.F.shift); it is internal.)
 *  - Handles are opaque and owned by the library.  An operator handle may be
 *    used by several threads; calls on one handle are serialised.
 */
#ifndef PHICOMB_H
#define PHICOMB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PHICOMB_OK 0
#define PHICOMB_PENDING 1
#define PHICOMB_EINVAL (-1)    /* bad argument: sizes, non-finite input, tol<=0, ceil(s max|t|) > INT_MAX */
#define PHICOMB_ENOMEM (-2)    /* device allocation failed */
#define PHICOMB_EADMIT (-3)    /* request can never fit the serving memory budget */
#define PHICOMB_ENOCONV (-4)   /* a Taylor loop hit the term cap (150 terms) */
#define PHICOMB_EOVERFLOW (-5) /* Algorithm 1 accepted no power of A (||Av|| beyond the overflow guard) */
#define PHICOMB_EDEVICE (-6)   /* HIP runtime error, missing device, or a non-finite result */

/* precision of the Taylor terms (the parameter search is always FP64) */
#define PHICOMB_FP64 0
/* Mixed: in every Taylor loop (the S-series and each recovery step), once
 * the previous term's block norm is below tol / (80 u32) (u32 = 2^-24) of
 * the smaller of the partial sum and the loop's starting block, later terms
 * and their products with A are FP32 (an FP64 head and an FP32 tail).
 * Partial sums, the stopping test and everything carried from one loop to
 * the next stay FP64, so the result agrees with FP64 to about 10 tol in the
 * block norm.  Terms stay FP64 when the partial sum is outside [1e-20,
 * 1e30 / (||A||_inf + |xi|)] (FP32 range).  Shapes with no mixed kernel run
 * FP64. */
#define PHICOMB_MIXED 1

/* limits of this build */
#define PHICOMB_MAX_P 7  /* p <= 7 */
#define PHICOMB_MAX_R 4  /* r <= 4 */
#define PHICOMB_MAX_M 100
#define PHICOMB_MAX_N (1 << 28)  /* rows of an operator (columns are addressed with 32-bit byte offsets) */

typedef struct phicomb_op_s *phicomb_op;
typedef struct phicomb_req_s *phicomb_req;

/* Result of Algorithm 1 (Sec. 3).  Plain data: may be stored and reused for
 * every later solve with the same operator (Sec. 6: the pair is computed once
 * and reused across calls). */
typedef struct {
    double shift;    /* xi*, minimiser of the power objective f (Alg. 1) */
    double s0;       /* preliminary scale from the last accepted growth ratios */
    double zstar;    /* minimiser in the reduced variable z = -xi/s0 */
    double fstar;    /* f(xi*) */
    double s;        /* real scaling parameter s = s0 f(xi*) / (tol m!)^(1/m) */
    double tol;      /* tolerance the pair was chosen for */
    int32_t m;       /* Taylor degree used by the objective (default 61) */
    int32_t r_acc;   /* last accepted power of the guarded basis */
    int32_t n_feval; /* objective evaluations spent by Brent's method */
    int32_t status;  /* PHICOMB_OK when valid */
} phicomb_params_t;

/* Per-solve statistics. */
typedef struct {
    int32_t s_int;          /* integer scaling max(1, ceil(s max|t_i|)) (Alg. 3) */
    int32_t terms_S;        /* k at exit of the S-series loop (Alg. 3, rec.D) */
    int32_t terms_rec;      /* Taylor terms summed over the s_int-1 recovery steps */
    int32_t max_terms_step; /* largest term count of one recovery step */
    int32_t status;
    int32_t fp32_terms;     /* mixed precision: Taylor terms evaluated in FP32 (S-series and recovery) */
    double bytes_alg;       /* algorithmic HBM bytes of the solve (see design notes) */
    double ms;              /* device time of the solve kernel, milliseconds */
} phicomb_stats_t;

/* ---------------------------------------------------------------- operators
 * An operator is copied to the current HIP device and stays resident until
 * phicomb_op_destroy.  Products are the only access to A (Alg. 1-3 take "a
 * matrix or linear operator"); the library applies A - xi I with the shift
 * folded into the diagonal.
 */

/* CSR matrix, host arrays: rowptr[n+1] (rowptr[0] = 0, non-decreasing),
 * col[nnz] in [0, n), val[nnz].  1 <= n <= PHICOMB_MAX_N, nnz < 2^31.  EINVAL
 * on a malformed structure, a non-finite value or n out of range. */
int phicomb_op_create_csr(int64_t n, const int32_t *rowptr, const int32_t *col,
                          const double *val, phicomb_op *out);

/* Constant-coefficient stencil on a Dirichlet grid.  dim = 2 (5-point, grid =
 * {nx, ny, 1}) or 3 (7-point, grid = {nx, ny, nz}); grid index i = x + nx*(y +
 * ny*z).  coef[7] = {centre, -x, +x, -y, +y, -z, +z} neighbour weights;
 * superdiag is added to every matrix entry (i, i+1), i < n-1 (a non-normal
 * perturbation; at the end of a grid line it is a new entry).  n = nx*ny*nz
 * must be <= PHICOMB_MAX_N (EINVAL otherwise). */
int phicomb_op_create_stencil(int dim, const int32_t grid[3], const double coef[7],
                              double superdiag, phicomb_op *out);

/* Dense n x n matrix, host row-major.  Products use FP64 MFMA. */
int phicomb_op_create_dense(int64_t n, const double *A, phicomb_op *out);

/* Low-rank operator A = U W^T (Sec. 5, third experiment: a fixed orthonormal
 * basis U and W = U M^T for a small core M), applied matrix-free as
 * x -> U (W^T x) with O(n rank) work per product.  U and W: host arrays,
 * row-major n x rank, copied to the device.  1 <= rank <= 16,
 * 1 <= n <= PHICOMB_MAX_N;
 * a solve additionally needs rank * max((p+1) r + r, 2r) <= 256 (EINVAL
 * otherwise).  The batched entry points do not take this kind (EINVAL).
 * EINVAL on a bad size or a non-finite entry. */
int phicomb_op_create_lowrank(int64_t n, int rank, const double *U, const double *W,
                              phicomb_op *out);

int phicomb_op_destroy(phicomb_op op);
int64_t phicomb_op_n(phicomb_op op);

/* ---------------------------------------------------------------- Algorithm 1
 * Choose the shift xi* and the scaling s for tolerance tol and degree m
 * (Sec. 3, Algorithm 1): guarded power basis of a unit vector, preliminary
 * scale s0, normalised basis extended to degree m, Brent minimisation of
 * f(xi) = ||(A - xi I)^m v||^(1/m) / s0 over z = -xi/s0 in [-sqrt(n), sqrt(n)],
 * then s = s0 f(xi*) / (tol m!)^(1/m).
 *   v      host [n] start vector (normalised by the library), or NULL for the
 *          library's own deterministic vector derived from seed
 *          (SplitMix64 of (seed, i) mapped to [-1, 1)).
 *   m      1..PHICOMB_MAX_M (the paper's default is 61).
 *   stream hipStream_t or NULL; the call is blocking.
 * Errors: EINVAL, EOVERFLOW (no power accepted), ENOMEM, EDEVICE.
 * A zero operator returns shift 0, s 1. */
int phicomb_params(phicomb_op op, double tol, int m, const double *v, uint64_t seed,
                   void *stream, phicomb_params_t *out);

/* ---------------------------------------------------------------- Algorithm 3
 * W[:, i] = sum_j beta[i][j] phi_j(t_i A) v_j, i < r (Sec. 4, Algorithm 3, the
 * block variant; r = 1 is Algorithm 2).  Blocking: returns when W is written.
 *   prm       result of phicomb_params for this operator (any tol).
 *   p, r      0 <= p <= PHICOMB_MAX_P, 1 <= r <= PHICOMB_MAX_R.
 *   t         host [r] abscissae (any sign, finite).
 *   beta      host [r][p+1] weights; the paper's case is beta[i][j] = alpha_i^j.
 *   V         device [n][p+1] row-major, double.
 *   tol       stopping tolerance of the Taylor loops (stopTm), > 0.
 *   precision PHICOMB_FP64 or PHICOMB_MIXED.
 *   W         device [n][r] row-major, double, written.
 *   stream    hipStream_t or NULL.
 *   stats     optional, may be NULL.
 * p = 0 returns exp(t_i A) v_0; v_0 = 0 returns sum_{j>=1} beta_ij phi_j v_j.
 * Errors: EINVAL, ENOCONV, ENOMEM,
 * EDEVICE (W then undefined).  Non-finite entries of V (or weighted columns
 * beyond the double range) are found by the device in its first pass over V,
 * before any Taylor term, and reported as EINVAL. */
int phicomb_solve(phicomb_op op, const phicomb_params_t *prm, int p, int r,
                  const double *t, const double *beta, const void *V, double tol,
                  int precision, void *W, void *stream, phicomb_stats_t *stats);

/* --------------------------------------------------- solve without allocation
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as phicomb_solve (same kernels, same results), with the work blocks
 * in a static device array of PHICOMB_STATIC_BYTES per device instead of
 * the operator's grow-only workspace.  The call allocates nothing: no
 * hipMalloc, hipFree or allocating library routine (the array's address and
 * two timing events are set up once per device, at the first call).  The
 * caller still passes V and W.  EINVAL when the work blocks of this shape
 * (phicomb_request_bytes minus V and W, i.e. about 8 n ((p+1) r + 2 max((p+1)
 * r, 2r) + 2r) bytes, plus the FP32 blocks of mixed precision) exceed the
 * array, or when the operator was created on another device than the
 * current one; otherwise as phicomb_solve.  Every call on a device shares
 * that device's array, which keeps the last call's contents; calls that
 * would overlap on one device are serialised by the library (each waits for
 * the previous one to finish). */
#define PHICOMB_STATIC_BYTES (64ll << 20)

int phicomb_solve_static(phicomb_op op, const phicomb_params_t *prm, int p, int r,
                         const double *t, const double *beta, const void *V, double tol,
                         int precision, void *W, void *stream, phicomb_stats_t *stats);

/* ---------------------------------------------------------------- serving
 * Asynchronous form of phicomb_solve for a request stream (continuous
 * batching; the paper computes the parameters once per operator and reuses
 * them across calls, Sec. 6).  A request is admitted, in arrival order
 * except that one waiting for memory does not block smaller ones behind it,
 * as soon as its device footprint (phicomb_request_bytes) fits what the
 * running requests leave of the budget and a slot is free.  Admitted
 * requests of any operator run at the same time on their own streams; each
 * is guaranteed CUs/slots of the device's CUs and takes up to one CU per 512
 * rows when more are free.  The result of a request does not depend on what
 * runs beside it.  Same arguments as phicomb_solve minus the stream.  V and W
 * must stay valid, and the operator alive, until poll reports completion.
 * Returns at once: OK with *out set, EINVAL, ENOMEM, or EADMIT if the
 * request can never fit the budget. */
int phicomb_submit(phicomb_op op, const phicomb_params_t *prm, int p, int r,
                   const double *t, const double *beta, const void *V, double tol,
                   int precision, void *W, phicomb_req *out);

/* PHICOMB_PENDING while queued or running; otherwise the request's final
 * status, with stats filled (optional) and the ticket released. */
int phicomb_poll(phicomb_req req, phicomb_stats_t *stats);

/* Serving limits: device bytes the admitted requests may hold at once
 * (budget_bytes <= 0 keeps the current one; default half of the free device
 * memory at the first call), and the number of requests that may run
 * concurrently (slots, 1..64, <= 0 keeps the current one; default 4).  Slots
 * can grow but not shrink once requests have run (EINVAL). */
int phicomb_serve_config(int64_t budget_bytes, int slots);

/* Device footprint in bytes of one request (V, W and work blocks). */
int64_t phicomb_request_bytes(int64_t n, int p, int r, int precision);

/* ---------------------------------------------------------------- batches
 * Many independent solves (Sec. 4, Algorithm 3 each) of uneven size in one
 * persistent launch.  The library splits the launch into groups of
 * workgroups, each running an ordered list of the instances, with group sizes
 * (and with them the rows each thread owns) and lists chosen from a cost
 * model of one Taylor term (phicomb_batch_model) and the expected term count
 * of every instance (s_int steps of the length tol implies), so that the
 * predicted finishing time of the last group is smallest: every instance
 * gets the fewest workgroups that meet a trial makespan and joins, first fit,
 * the smallest group of at least that size with time left.  The launch is
 * captured into a HIP graph and replayed by every run (recaptured when a
 * refit of the model changes the schedule).
 *   items     [count] solves: same fields as phicomb_solve; every operator of
 *             the kind stencil or CSR (dense operators are CSR inside), all of
 *             one kind and on the current device.  t and beta are copied at
 *             create; V and W are device pointers kept by the plan: their
 *             contents may change between runs, the pointers may not.
 *   count     1..PHICOMB_MAX_BATCH.
 * The plan holds its own work blocks (sum of solve_workspace sizes).
 * Errors: EINVAL (bad item, mixed kinds or devices), ENOMEM, EDEVICE. */
#define PHICOMB_MAX_BATCH 4096

typedef struct phicomb_batch_s *phicomb_batch;

typedef struct {
    phicomb_op op;
    const phicomb_params_t *prm;
    int32_t p, r;
    const double *t;     /* host [r] */
    const double *beta;  /* host [r][p+1] */
    const void *V;       /* device [n][p+1] row-major */
    void *W;             /* device [n][r] row-major, written by runs */
    double tol;
} phicomb_batch_item;

int phicomb_batch_create(int count, const phicomb_batch_item *items, int precision,
                         phicomb_batch *out);

/* Runs every solve of the plan on stream (blocking).  stats: optional
 * [count]; ms is the duration of the whole launch.  Returns OK or the first
 * failing instance's status (every instance still runs). */
int phicomb_batch_run(phicomb_batch b, void *stream, phicomb_stats_t *stats);

/* The plan's schedule: number of groups, workgroups of the launch, and the
 * cost model's predicted duration (milliseconds). */
int phicomb_batch_info(phicomb_batch b, int *groups, int *workgroups, double *predicted_ms);

/* The plan's cost model of one Taylor term on G workgroups, in microseconds:
 *   (G = 1 ? m[0] : m[1] + m[2] G) + ceil(n / (512 G)) (m[3] + m[4] 2r),
 * an exchange latency plus the rounds of rows each thread works through one
 * after another.  Every successful run refits it from the device clocks of
 * its instances (the per-round constants by least squares over instances of
 * 4 or more rounds, then the exchange constants from the remainders of
 * instances of few rounds, where the exchange dominates; every instance
 * weighted by its term count), rebuilds the schedule when the refit
 * predicts a makespan 10 % below the measured one (at most 3 times), and
 * returns to the fastest plan measured when a rebuilt one ran slower.  get (optional, 5 doubles)
 * receives the current model; set (optional, 5 non-negative doubles, e.g. a
 * model saved from an earlier plan by an autotuner) replaces it and rebuilds
 * the schedule (EINVAL for a negative or non-finite value). */
int phicomb_batch_model(phicomb_batch b, double *get, const double *set);

/* The last run's launch time, the model's prediction for that run's plan
 * before the refit (with the run's measured term counts), and after it. */
int phicomb_batch_fit(phicomb_batch b, double *measured_ms, double *predicted_ms_before,
                      double *predicted_ms_after);

/* Per instance of the last run (optional arrays of count entries): its
 * duration in microseconds from the device clock, and the workgroups of the
 * group that ran it (the data the cost model is fitted to). */
int phicomb_batch_times(phicomb_batch b, double *us, int *group_size);

int phicomb_batch_destroy(phicomb_batch b);

/* Block product Y = (A - shift I) X, the operation every Taylor term of
 * Algorithms 1-3 is built from (A is accessed only through products).  X and
 * Y: device arrays, column-major n x ncols (column c at offset c n), caller
 * owned, not overlapping; 1 <= ncols <= 64.  Stencil, CSR and dense operators
 * (dense through its CSR form); EINVAL for a low-rank operator.  Enqueued on
 * stream; when ms is not NULL the call waits for the product and stores its
 * device time in milliseconds. */
int phicomb_op_apply(phicomb_op op, const void *X, int ncols, double shift, void *Y,
                     void *stream, double *ms);

/* The single block series of the Proposition in Sec. 4 with g_i = phi_i:
 * W[:, k] = sum_i beta[k][i] phi_i(t_k A) v_i evaluated as
 * sum_j A^j V D_j Gamma T^j (D_j = diag(1/(i+j)!), Gamma[i][k] = beta[k][i]),
 * without shift or scaling and without Algorithm 1 parameters: the products
 * act on the p+1 columns of V only, whatever r is.  Terms are added until two
 * consecutive ones fall below tol times the block infinity norm, as in
 * Algorithm 3.  Meant for small |t_k| ||A|| (say up to about 1); for larger
 * steps it needs many terms and loses accuracy to cancellation (ENOCONV at
 * the term cap), and phicomb_solve is the method to use.  Arguments, layouts
 * and ownership as for phicomb_solve; every operator kind (dense through its
 * CSR form; low rank with W^T P_j summed in each term's exchange, which needs
 * rank (p+1) <= 256).  stats: s_int = 1,
 * terms_S = terms summed, the rest 0 apart from status, bytes_alg and ms. */
int phicomb_solve_series(phicomb_op op, int p, int r, const double *t, const double *beta,
                         const void *V, double tol, void *W, void *stream,
                         phicomb_stats_t *stats);

/* ------------------------------------------------------- exponential integrator
 * expRK4s6 (Sec. 1, eq. (expRK4s6): Luan's fourth-order six-stage exponential
 * Runge-Kutta scheme, nodes c2 = c3 = 1/2, c4 = c6 = 1/3, c5 = 5/6) for
 * u' = A u + g(u) with a pointwise cubic reaction
 * g(u) = g[0] + g[1] u + g[2] u^2 + g[3] u^3, as in the fourth experiment of
 * Sec. 5.  nsteps steps of size h advance the device vector u (n FP64,
 * overwritten in place).  Each step makes four block calls of Algorithm 3,
 * with the stages the scheme allows to be formed together in one call
 * (U2; U3 and U4; U5 and U6; u_{n+1}), all with the parameters prm of
 * Algorithm 1 (computed once for A and tol and reused, Sec. 6); tol and
 * precision as for phicomb_solve.  The operator must be a stencil, CSR or
 * dense operator (EINVAL for low rank).  Stage buffers (8 n doubles) stay
 * with the operator.  The workgroup slots of the solves are held for the
 * whole integration and the host does not wait for individual calls.
 * Blocking; the first failing call's status is returned and u then holds
 * the last completed step (a failure is noticed within 64 steps; the steps
 * after it leave u unchanged).  stats may be NULL. */
typedef struct {
    int32_t steps;          /* steps completed */
    int32_t calls;          /* Algorithm 3 calls (4 per step) */
    int32_t max_s_int;      /* largest scaling count of any call */
    int32_t status;
    int64_t terms;          /* Taylor terms over all calls (S-series + recovery) */
    int64_t fp32_terms;     /* mixed precision: Taylor terms evaluated in FP32 */
    double ms;              /* device time of the whole integration, milliseconds */
} phicomb_exprk_stats_t;

int phicomb_exprk4s6(phicomb_op op, const phicomb_params_t *prm, const double g[4], double h,
                     int nsteps, double tol, int precision, void *u, void *stream,
                     phicomb_exprk_stats_t *stats);

/* ---------------------------------------------------------- complex data
 * Sec. 1 poses the problem over C: A in C^{n x n}, V in C^{n x (p+1)}, complex
 * t_i and weights; Algorithm 3 takes a shift xi in C; Algorithm 1's listing
 * searches xi on the real line from a real start vector, so its xi* is real.
 * Complex arrays are interleaved (re, im) doubles (the layout of C99
 * double complex and of torch.complex128).  FP64 only. */
typedef struct phicomb_zop_s *phicomb_zop;

/* Complex CSR operator (host arrays, copied): rowptr [n+1], col [nnz],
 * val [2 nnz] interleaved.  1 <= n, 2n <= PHICOMB_MAX_N.  The operator also
 * keeps its real 2n x 2n representation [[Re A, -Im A], [Im A, Re A]] for
 * Algorithm 1.  Errors: EINVAL (bad structure, non-finite value), ENOMEM,
 * EDEVICE. */
int phicomb_zop_create_csr(int64_t n, const int32_t *rowptr, const int32_t *col,
                           const double *val, phicomb_zop *out);

/* Complex dense operator, A [n][n] row-major interleaved (host, copied);
 * n <= 16384. */
int phicomb_zop_create_dense(int64_t n, const double *A, phicomb_zop *out);

int phicomb_zop_destroy(phicomb_zop op);

/* Algorithm 1 (Sec. 3) for a complex operator: the real parameter kernel on
 * the operator's real representation from the start vector [v; 0], which
 * gives the same powers' 2-norms, objective and (real) xi*, s as the complex
 * listing.  v: host [n] real, or NULL for SplitMix64(seed, i) in [-1, 1). */
int phicomb_zparams(phicomb_zop op, double tol, int m, const double *v, uint64_t seed,
                    void *stream, phicomb_params_t *out);

/* Algorithm 3 (Sec. 4) over C, beta-prescaled form:
 *   w_i = sum_j beta_ij phi_j(t_i A) v_j,  i = 1..r.
 *   prm    parameters of phicomb_zparams (s, and the shift unless given)
 *   shift  host [2] complex shift xi, or NULL for prm->shift
 *   t      host [r] complex;  beta host [r][p+1] complex
 *   V      device [n][p+1] complex row-major;  W device [n][r] complex, written
 *   stats  optional (s_int, term counts, kernel time; bytes_alg not set)
 * One persistent launch, blocking on stream; the operator's device must be
 * the current one.  Errors: EINVAL (arguments, another device, non-finite V
 * found on the device), ENOCONV (a Taylor loop reached 150
 * terms), EDEVICE (launch, barrier time-out, or a non-finite norm later). */
int phicomb_zsolve(phicomb_zop op, const phicomb_params_t *prm, const double *shift, int p,
                   int r, const double *t, const double *beta, const void *V, double tol,
                   void *W, void *stream, phicomb_stats_t *stats);

const char *phicomb_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* PHICOMB_H */
