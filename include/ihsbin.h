/*
 * ihsbin.h - C ABI of the MI355X ridge-regularization-path solver (IHS-BIN).
 *
 * Problem (Section 1, Eq. (least-square); matrix right-hand sides: Section 5.3,
 * Eq. (least-square-max)):
 *     x(lam) = argmin_x 0.5*||A x - b||^2 + 0.5*lam*||x||^2  for every lam in a
 *     grid Lambda inside [lam_min, lam_max],
 * solved by the iterative Hessian sketch with binomial decomposition
 * (Section 4: the Proposition, Algorithms 2 and 3; Algorithms 5 and 6 for a
 * matrix B).  The build step sketches A, factors the sketched Hessian once per
 * lambda sub-interval (Section 4.2), runs the basis recursion Eq. (equ:upd)
 * and keeps the lambda-independent basis on the device; the evaluation step
 * composes x(lam) for any lam in [lam_min, lam_max] from that basis.
 *
 * Conventions for every call:
 *  - Pointers documented "device" must point to device memory of the context's
 *    device; "host" pointers to host memory.  The caller owns A, B, X and every
 *    output buffer; the library owns what it allocates inside opaque handles.
 *  - All device work is enqueued on the stream given to ihsbin_create; a call
 *    returns after the results it documents are complete on that stream unless
 *    stated otherwise.  Calls on one context must not overlap.
 *  - Dense matrices are row-major with a row stride (ld, in elements).
 *  - Every call returns an ihsbin_status code; no C++ exception crosses the
 *    ABI.  On failure ihsbin_last_error(ctx) holds a message and the output
 *    buffers hold unspecified values (except IHSBIN_ENOCONV, see below).
 *  - Under-determined problems (n < d) with a dense A are solved through the
 *    dual problem of Section 5.2, Eq. (ls_reg:d); n < d with a CSR matrix
 *    returns IHSBIN_EUNSUP.
 *  - Arithmetic: the sketch, its factors, the basis and every product with A
 *    run in FP64, and so does the sketched Hessian unless gram_prec selects
 *    its split-BF16 form; A and B are read in their stored type (FP32 or
 *    FP64, converted exactly on load).
 */
#ifndef IHSBIN_H
#define IHSBIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
typedef enum {
  IHSBIN_OK = 0,
  IHSBIN_EINVAL = -1,   /* bad argument (null pointer, size, lam range, CSR) */
  IHSBIN_ENOMEM = -2,   /* device allocation failed                          */
  IHSBIN_EHIP = -3,     /* a HIP runtime call failed                         */
  IHSBIN_ENOTSPD = -4,  /* a sketched Hessian was not positive definite      */
  IHSBIN_ENOCONV = -5,  /* an interval hit k_max before its stop test passed;
                           the path is still built and usable                */
  IHSBIN_ERANGE = -6,   /* a lam outside the prepared [lam_min, lam_max]     */
  IHSBIN_EUNSUP = -7,   /* unsupported combination (n < d CSR, dtype, ...)    */
  IHSBIN_EAGAIN = -8    /* a served request is not finished yet               */
} ihsbin_status;

enum { IHSBIN_DENSE = 0, IHSBIN_CSR = 1 };
enum { IHSBIN_F32 = 0, IHSBIN_F64 = 1 };

/* Sketch families of Section 4 (bullets 1-4). */
enum {
  IHSBIN_GAUSSIAN = 0,    /* S_ij ~ N(0, 1/m)                                  */
  IHSBIN_SRHT = 1,        /* sqrt(n'/m) R (H/sqrt(n')) D, rows with replacement */
  IHSBIN_COUNTSKETCH = 2, /* one +-1 per column of S                           */
  IHSBIN_SJLT = 3         /* s stacked CountSketches of m/s rows, 1/sqrt(s)    */
};

typedef struct ihsbin_ctx ihsbin_ctx;
typedef struct ihsbin_path ihsbin_path;

/* The data matrix A (n x d).  Dense: row-major, vals = device pointer to
 * n*ld elements of dtype.  CSR: row_ptr (n+1, device int32, non-decreasing,
 * row_ptr[0] = 0, row_ptr[n] = nnz), col_idx (nnz, device int32 in [0, d)),
 * vals (nnz, device, dtype).  Duplicate column entries are summed. */
typedef struct {
  int32_t format;          /* IHSBIN_DENSE or IHSBIN_CSR          */
  int32_t dtype;           /* IHSBIN_F32 or IHSBIN_F64            */
  int64_t n, d;
  int64_t ld;              /* dense row stride, >= d               */
  int64_t nnz;             /* CSR only                             */
  const void* vals;
  const int32_t* row_ptr;
  const int32_t* col_idx;
} ihsbin_matrix;

/* Build options.  Fill with ihsbin_opts_default, then override. */
typedef struct {
  int32_t sketch;          /* IHSBIN_GAUSSIAN ... IHSBIN_SJLT                   */
  int32_t sjlt_s;          /* SJLT blocks s (m must be a multiple), else ignored */
  int64_t m;               /* initial sketch dimension m (Section 4)            */
  uint64_t seed;           /* sketch seed (SplitMix64 counter-based draws)       */
  double tol;              /* per-interval stop test: increment bound at both
                              interval ends relative to ||x|| (default 1e-8)    */
  int32_t k_max;           /* cap on basis steps k per interval (default 96)    */
  int32_t k_fixed;         /* > 0: every interval runs exactly k_fixed steps    */
  int32_t L;               /* intervals; 0 = floor(2 ln(lam_max/lam_min))       */
  int32_t centred;         /* 1: expand about the interval centre lam0 (default);
                              0: the printed expansion in powers of tau*lam     */
  int32_t adaptive_m;      /* sketch dimension policy: 0 = m as given;
                              1 (default) = grow m until the predicted rate of
                              the lowest interval is <= rate_target;
                              2 = Algorithm 4 (Section 5.1) at lam_min, from
                              m0 = m (0: max(16, d / 4)), parameters
                              from alg4;
                              3 = as 1, but a Gaussian sketch that would need
                              more rows than it takes to form A^T A at the same
                              cost (8 d for the BF16/FP8 forms, d for FP64)
                              is replaced by S = I (the exact Hessian, m = n;
                              dense A, single builds)                         */
  double rate_target;      /* default 0.6                                      */
  int64_t m_max;           /* cap for adaptive m; 0 = library default           */
  int32_t lanczos_steps;   /* Lanczos steps of each spectrum estimate (default
                              12); one run per interval end: the smallest
                              eigenvalue at the lower end and the largest at
                              the upper end bound the whole interval          */
  int32_t timing;          /* 1: time the A^T A product kernels with events     */
  const double* taus;      /* host, optional: fixed step size per interval (L)  */
  int32_t gram_prec;       /* sketched Gram (SA)^T SA: IHSBIN_GRAM_F64 (default)
                              or IHSBIN_GRAM_BF16X3 (BF16 matrix cores, three-
                              term splits, ~1e-6 relative; the factor is still
                              FP64 and used consistently, so the path keeps its
                              fixed point)                                       */
  const struct ihsbin_alg4_opts* alg4; /* host, optional: Algorithm 4 parameters
                              for adaptive_m = 2 (NULL: the defaults)            */
  int32_t sketch_prec;     /* Gaussian S A: IHSBIN_SKETCH_F64 (default),
                              IHSBIN_SKETCH_BF16 (BF16 matrix cores: S rounded
                              to BF16 - still a Gaussian-type sketch - and A in
                              two BF16 terms, FP32 sums of <= 2048 rows, FP32
                              sums of those, FP64 across K-splits) or
                              IHSBIN_SKETCH_FP8 (FP8 matrix cores: S rounded to
                              e4m3, A in three e4m3 terms under a per-column
                              power-of-two scale, about 12 bits relative to the
                              column's largest entry; same sums); dense A only,
                              other sketches ignore it                           */
  double sigma_d2;         /* >= 0: sigma_d^2 of A (smallest squared singular
                              value) or an estimate; > 0 centres each interval
                              [lo, hi] at lam0 = sqrt((lo+s)(hi+s)) - s (the
                              remark after Theorem 1); 0 (default): sqrt(lo hi) */
  int32_t basis_prec;      /* arithmetic of the basis steps' A^T A products
                              (dense FP32 A; other inputs always use FP64):
                              IHSBIN_BASIS_F64 (default), IHSBIN_BASIS_F32 (every
                              step on the FP32 matrix cores: the recursion
                              refines with FP32 products, so its accuracy is
                              limited near 1e-5), IHSBIN_BASIS_MIXED (FP64 until
                              the largest increment of x at the ends of the
                              active intervals, relative to x, is <= f32_switch;
                              FP32 afterwards, when the products only refine
                              what is left)                                     */
  double f32_switch;       /* IHSBIN_BASIS_MIXED threshold (default 1e-2)       */
  int32_t graph_steps;     /* ihsbin_path_build_batch: > 0 captures that many
                              basis steps at a time into one HIP graph (on a
                              private stream of the context) and launches it
                              as one unit, reading the stop test once per
                              graph; 0 (default): step by step                  */
} ihsbin_opts;

/* Arithmetic of the basis products. */
enum { IHSBIN_BASIS_F64 = 0, IHSBIN_BASIS_F32 = 1, IHSBIN_BASIS_MIXED = 2 };

/* Arithmetic of the Gaussian sketch product. */
enum { IHSBIN_SKETCH_F64 = 0, IHSBIN_SKETCH_BF16 = 1, IHSBIN_SKETCH_FP8 = 2 };

/* Algorithm 4 (Section 5.1): IHS at lam with the direction
 * D_k = (A^T S^T S A + lam I)^-1 grad f(X_k), delta_k = <D_k, grad f(X_k)>,
 * the Armijo step of Eq. (armijo), and m doubled (S redrawn at 2m from the
 * same seed) whenever an update leaves delta_{k+1} >= gamma3 delta_k.
 * Fill with ihsbin_alg4_opts_default, then override. */
typedef struct ihsbin_alg4_opts {
  double gamma1;           /* Armijo steps tau = gamma1^j, in (0,1) (0.5)       */
  double gamma2;           /* Armijo sufficient decrease, in (0,1) (1e-4)       */
  double gamma3;           /* doubling threshold on delta_{k+1}/delta_k (0.5)    */
  double eps;              /* stop once delta_k <= eps * delta_0 (1e-8)          */
  int32_t max_iter;        /* IHS updates at most (50)                           */
  int32_t max_armijo;      /* trial steps per line search at most (60); none
                              accepted returns IHSBIN_ENOCONV                    */
} ihsbin_alg4_opts;

/* Filled by ihsbin_sketch_size. */
typedef struct {
  int64_t m;               /* sketch dimension at exit (n when S = I was used)  */
  int32_t iters;           /* IHS updates taken                                  */
  int32_t doublings;       /* times m was doubled                                */
  double delta0;           /* delta of the first direction (X_0 = 0)            */
  double delta;            /* delta at exit                                      */
  double ms;               /* wall time of the call                              */
} ihsbin_alg4_result;

/* Precision of the sketched Gram. */
enum { IHSBIN_GRAM_F64 = 0, IHSBIN_GRAM_BF16X3 = 1 };

/* Filled by ihsbin_path_build. */
typedef struct {
  int64_t m_used;          /* final sketch dimension (n when a sketch of m >= n
                              rows was replaced by S = I, the exact Hessian)    */
  int32_t L;               /* number of intervals                                */
  int32_t k_max_used;      /* largest k over intervals                           */
  int32_t k_sum;           /* sum of k over intervals                            */
  int32_t n_unconverged;   /* intervals that hit k_max                           */
  int32_t sketch_trials;   /* sketches drawn (adaptive m)                        */
  int32_t steps;           /* outer basis steps run (max k - 1)                  */
  double ms_sketch, ms_factor, ms_spectrum, ms_basis, ms_total;
  /* A^T A product kernels of the basis steps (Y = A U, then W = A^T Y) on
   * the FP64 matrix cores, timing = 1 only:                                */
  int64_t ata_launches;    /* launches of each of the two product kernels        */
  double ata_flops;        /* algorithmic flops of all those launches (4*nnz*w)  */
  double ata_ms_y;         /* summed event time of the Y = A U launches          */
  double ata_ms_w;         /* summed event time of the W = A^T Y launches (the
                              product kernel; its split-K reduction excluded)   */
  double ata_bytes_a;      /* algorithmic bytes of A read by those launches      */
  int64_t peak_bytes;      /* device memory held through the context at the
                              build's peak: its pool, workspaces (including those
                              kept from earlier calls) and the path's buffers    */
  double est_rel_err;      /* the stop test's bound on the relative error left
                              in x(lam), the largest over every interval and
                              both of its ends at the step the interval stopped:
                              ||last increment|| * r / (1 - r) / ||x||, r the
                              interval's predicted rate (the worst case over an
                              interval is at its ends, proof of Theorem 1); for
                              IHSBIN_ENOCONV it is the estimate of the intervals
                              that hit k_max; n < d: of the dual iterate; NaN
                              when every interval has one term (k = 1)          */
  int64_t ata_f32_launches; /* basis product launches on the FP32 matrix cores
                              (timing = 1; the ata_* fields above count the FP64
                              launches only)                                    */
  double ata_f32_flops, ata_f32_ms_y, ata_f32_ms_w;
  double bytes_moved;      /* algorithmic device-memory bytes of the passes over
                              A: A read once per product (sketch, A^T B, every
                              A U and A^T Y), the n x w intermediate Y written
                              and read once, U read and W written once          */
} ihsbin_report;

/* Per-interval description of a built path (host arrays of length L). */
typedef struct {
  int32_t L, K;
  int64_t d, m_used;
  double lam_min, lam_max;
  int32_t centred;
  int32_t dual;            /* 1: n < d, built on the dual problem (Section 5.2) */
} ihsbin_path_info;

/* ------------------------------------------------------------------ calls */

/* Static string for a status code. */
const char* ihsbin_status_str(int status);

/* Library version string. */
const char* ihsbin_version(void);

/* Default options: Gaussian sketch, m = 0 (= 2 d), seed 0, tol 1e-8,
 * k_max 96, L from Section 4.2, centred, adaptive m, rate 0.6, 12 Lanczos
 * steps, no timing. */
void ihsbin_opts_default(ihsbin_opts* opts);
void ihsbin_alg4_opts_default(ihsbin_alg4_opts* opts);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t the
 * library enqueues on (borrowed, not destroyed); NULL means the null stream.
 * Errors: EINVAL (null out pointer, bad device), EHIP. */
int ihsbin_create(ihsbin_ctx** ctx, int device, void* hip_stream);

/* Free the context and its workspace.  Paths built on it stay valid until
 * freed.  NULL is allowed. */
int ihsbin_destroy(ihsbin_ctx* ctx);

/* Message of the last failed call on ctx (static empty string when none). */
const char* ihsbin_last_error(const ihsbin_ctx* ctx);

/* Build the lambda-independent basis for [lam_min, lam_max] (Algorithm 3
 * with the basis hoisted out of the lambda loop; Algorithm 6 for K > 1).
 * B: device, n x K row-major with row stride ldb (>= K), dtype of A.
 * n < d (dense A only): the basis is built on the dual problem of Section
 * 5.2, (A A^T + lam I) z = b with x = A^T z; sketch, factors and step sizes
 * then live in R^n, the stored basis is mapped to x, and the stop test
 * measures the dual iterate.  The path reports dual = 1.
 * On success *path owns the basis on the device.  report may be NULL.
 * Errors: EINVAL (0 < lam_min <= lam_max violated, sizes), EUNSUP (n < d
 * with a CSR matrix), ENOTSPD, ENOMEM, EHIP.  ENOCONV: some interval reached
 * k_max; *path is still returned and usable, and report->est_rel_err holds
 * the stop test's bound on its remaining relative error. */
int ihsbin_path_build(ihsbin_ctx* ctx, const ihsbin_matrix* A, const void* B,
                      int64_t K, int64_t ldb, double lam_min, double lam_max,
                      const ihsbin_opts* opts, ihsbin_path** path,
                      ihsbin_report* report);

/* ihsbin_path_build for P problems of one shape at once (Algorithm 3 / 6 for
 * each; the problems are independent): dense A_p = A->vals + p * strideA
 * (elements of A's dtype; every A_p is n x d with row stride A->ld, n >= d)
 * and B_p = B + p * strideB (n x K, row stride ldb).  All problems share the
 * interval plan, the sketch family, its dimension m (adaptive_m 0 or 1: the
 * probe grows m until the slowest problem's lowest interval meets
 * rate_target) and, for the Gaussian sketch, the sketch matrix itself; each
 * problem has its own sketched Gram, factors, step sizes and basis.  Every
 * step runs as one launch sequence over all P L intervals, so many small
 * problems cost about as many launches as one; the basis steps run in
 * lockstep (every interval takes the number of steps after which all of them
 * pass the stop test, or k_fixed).  paths: host array of P handles receiving
 * independent paths (their bases share one device allocation, released with
 * the last of them).  report (optional) describes the whole batch.
 * Errors: EINVAL (sizes, strides, lambda range), EUNSUP (CSR, n < d,
 * adaptive_m = 2, taus, gram_prec other than FP64), ENOTSPD, ENOMEM, EHIP;
 * ENOCONV as for ihsbin_path_build (paths are returned). */
int ihsbin_path_build_batch(ihsbin_ctx* ctx, int32_t P, const ihsbin_matrix* A, int64_t strideA,
                            const void* B, int64_t K, int64_t ldb, int64_t strideB,
                            double lam_min, double lam_max, const ihsbin_opts* opts,
                            ihsbin_path** paths, ihsbin_report* report);

/* Compose x(lam_t) = tau sum_j (tau (lam_t - ref))^j ut_j for every t
 * (Algorithm 3 / 6, the lambda loop).  lambdas: host, T values, any order,
 * each inside [lam_min, lam_max] (else ERANGE).  X: device, T blocks of
 * d x K row-major (row stride ldx >= K, block stride d*ldx), element type
 * x_dtype (IHSBIN_F32 or IHSBIN_F64). */
int ihsbin_path_eval(ihsbin_path* path, const double* lambdas, int64_t T,
                     void* X, int64_t ldx, int32_t x_dtype);

/* ihsbin_path_eval without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, layout and results as
 * ihsbin_path_eval, but the lambdas and the per-lambda evaluation items are
 * staged in one fixed 8 MiB device array per GPU (taken by the library when
 * it first runs on that GPU and held until the process ends) instead of the
 * path's own buffer: T <= 262144 (more: EINVAL), no hipMalloc, hipFree or
 * allocating library call.  Every call on a GPU uses that GPU's one array,
 * so calls that overlap on the same GPU (different threads, streams or
 * paths) race: the caller serializes them.  Returns after X is complete. */
int ihsbin_path_eval_noalloc(ihsbin_path* path, const double* lambdas, int64_t T,
                             void* X, int64_t ldx, int32_t x_dtype);

/* Sizes of a built path. */
int ihsbin_path_get_info(const ihsbin_path* path, ihsbin_path_info* info);

/* Per-interval plan and result, host arrays of length info.L (any may be
 * NULL): boundaries lo/hi, centre lam0, step size tau, predicted rate, k. */
int ihsbin_path_intervals(const ihsbin_path* path, double* lo, double* hi,
                          double* lam0, double* tau, double* rate, int32_t* k);

/* Copy the basis ut_{l,0..k_l-1} of interval l to `out` (device, k_l blocks
 * of d x K row-major doubles, contiguous). */
int ihsbin_path_basis(const ihsbin_path* path, int32_t l, double* out);

/* Free a path (NULL allowed). */
int ihsbin_path_free(ihsbin_path* path);

/* Algorithm 3 (Algorithm 6 for K > 1) in one call: build the basis for
 * [min(lambdas), max(lambdas)], evaluate x(lam_t) for every lambda into X
 * (layout of ihsbin_path_eval) and free the path.  Errors as for
 * ihsbin_path_build and ihsbin_path_eval; with ENOCONV X is still written. */
int ihsbin_solve_path(ihsbin_ctx* ctx, const ihsbin_matrix* A, const void* B,
                      int64_t K, int64_t ldb, const double* lambdas, int64_t T,
                      const ihsbin_opts* opts, void* X, int64_t ldx,
                      int32_t x_dtype, ihsbin_report* report);

/* ---------------------------------------------------- step-level calls */

/* The integer draws of a sketch (Section 4), bit-exact with the SplitMix64
 * specification in the documentation: COUNTSKETCH/SJLT: idx (device int32,
 * n*s entries, row-major n x s) and sign (device int8, n*s); SRHT: sign
 * (device int8, n entries, diagonal D) and idx (device int32, m entries,
 * sampled rows of the order-n' transform).  GAUSSIAN: EINVAL. */
int ihsbin_sketch_draws(ihsbin_ctx* ctx, int32_t sketch, uint64_t seed,
                        int64_t n, int64_t m, int32_t sjlt_s, int32_t* idx,
                        int8_t* sign);

/* The same draws computed on the host, for checking a device copy bit for
 * bit (Section 4, sketch list; SplitMix64 counter draws).  Layouts as for
 * ihsbin_sketch_draws: COUNTSKETCH/SJLT fill idx (n*s int32, bucket in
 * [0, m), SJLT block b of row i in [b*m/s, (b+1)*m/s)) and sign (n*s int8,
 * +-1); SRHT fills sign (n int8, the diagonal D) and idx (m int32, rows of
 * the order-n' transform, n' = 2^ceil(log2 n), drawn with replacement).
 * idx and sign are host buffers owned by the caller.  EINVAL for bad sizes,
 * null pointers, an SJLT s that does not divide m, or GAUSSIAN (whose
 * values go through log/cos and are not defined bit for bit). */
int ihsbin_sketch_indices_host(uint64_t seed, int32_t sketch, int64_t n, int64_t m,
                               int32_t sjlt_s, int32_t* idx, int8_t* sign);

/* ihsbin_sketch_draws with the argument order of ihsbin_sketch_indices_host
 * (idx and sign are device buffers). */
int ihsbin_sketch_indices_device(ihsbin_ctx* ctx, uint64_t seed, int32_t sketch, int64_t n,
                                 int64_t m, int32_t sjlt_s, int32_t* idx, int8_t* sign);

/* The column-major copy of a CSR matrix that the transposed products A^T Y
 * gather from (built inside every CSR build).  col_ptr (device int32, d+1),
 * row (device int32, nnz) and vals (device, nnz elements of A's dtype) receive
 * it: the entries of column c at positions [col_ptr[c], col_ptr[c+1]) in the
 * order of their position in the CSR arrays (so by increasing row, and a
 * row's duplicates in their stored order), which makes it the stable
 * transpose of A.  EINVAL for a dense or malformed matrix. */
int ihsbin_csr_transpose(ihsbin_ctx* ctx, const ihsbin_matrix* A, int32_t* col_ptr,
                         int32_t* row, void* vals);

/* SA = S A (Section 4, Algorithm 3 first line), FP64, m x d row-major into
 * SA (device, m*d doubles).  ihsbin_sketch_apply_prec selects the Gaussian
 * product's arithmetic (IHSBIN_SKETCH_F64; IHSBIN_SKETCH_BF16, for which
 * S = BF16(FP32(z)) / sqrt(m) of the same draws z; IHSBIN_SKETCH_FP8, for
 * which S = E4M3(FP32(z)) / sqrt(m) and A enters as its three-term e4m3 split;
 * dense A only for the last two; EINVAL for another value). */
int ihsbin_sketch_apply_prec(ihsbin_ctx* ctx, const ihsbin_matrix* A, int32_t sketch,
                             int32_t sjlt_s, int64_t m, uint64_t seed, int32_t prec,
                             double* SA);
int ihsbin_sketch_apply(ihsbin_ctx* ctx, const ihsbin_matrix* A, int32_t sketch,
                        int32_t sjlt_s, int64_t m, uint64_t seed, double* SA);

/* Lower Cholesky factors of (SA)^T SA + lam0_i I for i < nl (the matrix whose
 * inverse is P_S, Section 4), and their inverses.  SA: device m x d doubles.
 * lam0: host, nl values > 0.  Lfac, Linv: device, nl blocks of d x d doubles
 * row-major (upper triangles zero); Linv may be NULL.  ENOTSPD on failure. */
int ihsbin_precond_factor(ihsbin_ctx* ctx, const double* SA, int64_t m,
                          int64_t d, const double* lam0, int32_t nl,
                          double* Lfac, double* Linv);

/* G = (SA)^T SA for the preconditioner (Section 4, P_S).  SA: device m x d
 * doubles (row-major, contiguous).  G: device d x d doubles; its lower triangle
 * (and the diagonal 128 x 128 or 64 x 64 tiles) is written.  prec: IHSBIN_GRAM_*.
 * EINVAL on bad sizes or prec. */
int ihsbin_gram(ihsbin_ctx* ctx, const double* SA, int64_t m, int64_t d, int32_t prec,
                double* G);

/* The sketched Gram G = (SA)^T SA exactly as a path build forms it for a
 * sketch of m rows (Section 4: the Gram P_S is built from): the sketch
 * (sketch, sjlt_s, seed, sketch_prec as in ihsbin_opts), then the Gram
 * (gram_prec).  For CountSketch / SJLT of a CSR matrix with d <= 8192 the
 * sketch is kept sparse and G is formed from its entries in FP64 (gram_prec
 * does not apply); m >= n gives G = A^T A.  A: device matrix; G: device d x d
 * doubles (row-major), of which the lower triangle and the diagonal 64 x 64
 * tiles are written.  EINVAL on bad arguments (SJLT: sjlt_s must divide m),
 * EUNSUP as ihsbin_sketch_apply_prec. */
int ihsbin_sketch_gram(ihsbin_ctx* ctx, const ihsbin_matrix* A, int32_t sketch, int32_t sjlt_s,
                       int64_t m, uint64_t seed, int32_t sketch_prec, int32_t gram_prec,
                       double* G);

/* Adaptive sketch dimension (Section 5.1, Algorithm 4) for the problem at
 * lam (the path's lam_min): runs the search from m0 = opts->m (0: max(16, d / 4),
 * rounded up to a multiple of sjlt_s) with opts->sketch, sjlt_s, seed,
 * gram_prec and the cap opts->m_max (0: min(n, 32 d); SRHT also at most the
 * padded order), and returns the m it ends with.  A sketch of m >= n rows is
 * replaced by S = I.  X (device, optional) receives the last iterate, d x K
 * FP64 with row stride ldx (n < d: the dual iterate z, n x K).  trace (host,
 * optional) receives 5 doubles per update, at most trace_rows updates:
 * m in effect, tau_k, delta_k, delta_{k+1} from that sketch, 1.0 if m then
 * doubled.  res (host) must not be NULL. */
int ihsbin_sketch_size(ihsbin_ctx* ctx, const ihsbin_matrix* A, const void* B,
                       int64_t K, int64_t ldb, double lam, const ihsbin_opts* opts,
                       const ihsbin_alg4_opts* alg4, ihsbin_alg4_result* res,
                       double* X, int64_t ldx, double* trace, int32_t trace_rows);

/* W = A^T A U: the two products of every basis step (Algorithm 2).  U: device
 * d x w doubles with row stride ldu; the buffer spans d * ldu doubles, and
 * columns [w, ldu) may be read (their values are ignored) so that ragged
 * widths run whole column tiles.  W: device d x w doubles (row stride ldw);
 * only columns [0, w) are written. */
int ihsbin_ata_apply(ihsbin_ctx* ctx, const ihsbin_matrix* A, const double* U,
                     int64_t w, int64_t ldu, double* W, int64_t ldw);

/* The same product (dense A) with a chosen column tiling, for tuning: prec
 * IHSBIN_BASIS_F64 or IHSBIN_BASIS_F32 (FP32 matrix cores, FP32 A only), q in
 * [1, 7] the tile width in 16-column blocks and splits in [1, 256] the split-K
 * count of W = A^T Y (0 for either: the library's choice, from its tuned
 * table or its cost model).  Results equal ihsbin_ata_apply's up to the
 * summation order. */
int ihsbin_ata_apply_tiled(ihsbin_ctx* ctx, const ihsbin_matrix* A, const double* U, int64_t w,
                           int64_t ldu, double* W, int64_t ldw, int32_t prec, int32_t q,
                           int32_t splits);

/* ----------------------------------------------------------------- serving
 * Independent path builds on one device, run concurrently by worker slots
 * (each a context with its own stream) and admitted in arrival order while
 * the sum of the admitted builds' ihsbin_build_footprint estimates stays
 * within hbm_budget.  A build that still fails with IHSBIN_ENOMEM is queued
 * again at the front and runs with nothing else in flight.  Every build runs
 * the same kernels as it would alone, so a result does not depend on what
 * else is served (CountSketch/SJLT and CSR products add with atomics, whose
 * order can change the last bits).  The path of a finished request is the
 * caller's: its basis stays resident for any number of ihsbin_path_eval
 * calls until ihsbin_path_free.  Thread-safe: submit and wait may be called
 * from any threads. */
typedef struct ihsbin_server ihsbin_server;

typedef struct {
  int32_t workers;         /* concurrent builds (1..16, default 4)              */
  int32_t reserved;
  int64_t hbm_budget;      /* bytes the admitted builds may need together
                              (0: 90 % of the free device memory at creation) */
  int64_t keep_bytes;      /* device memory a worker keeps between builds
                              (default 1 GiB); above it the worker trims       */
} ihsbin_server_opts;

typedef struct {
  int32_t status;          /* the build's status (ihsbin_server_wait's result) */
  int32_t worker;          /* worker slot that ran it                           */
  int64_t footprint;       /* its admission estimate (bytes)                    */
  double ms_queue;         /* submission to start of the build                  */
  double ms_build;         /* the build                                         */
  double ms_total;         /* submission to completion                          */
  ihsbin_report report;
  char message[160];       /* error text when status is not IHSBIN_OK           */
} ihsbin_request_info;

typedef struct {
  int64_t submitted, completed;
  int64_t retried;         /* builds re-run alone after IHSBIN_ENOMEM           */
  int32_t workers, queued, inflight, max_concurrent;
  int64_t budget, inflight_bytes, max_inflight_bytes;
} ihsbin_server_stats;

/* Upper estimate of the device memory one ihsbin_path_build allocates for a
 * problem of this shape and these options (every buffer at its largest size,
 * the sketch at its cap; A, B and outputs are the caller's).  Only A's
 * format, dtype, n and d are read (its pointers may be NULL). */
int ihsbin_build_footprint(const ihsbin_matrix* A, int64_t K, double lam_min,
                           double lam_max, const ihsbin_opts* opts, int64_t* bytes);
/* Bind a path to another stream for its later calls (waits for the old one). */
int ihsbin_path_set_stream(ihsbin_path* path, void* hip_stream);

void ihsbin_server_opts_default(ihsbin_server_opts* opts);
int ihsbin_server_create(ihsbin_server** server, int device, const ihsbin_server_opts* opts);
/* Queue a build (the arguments of ihsbin_path_build; opts may be NULL, and
 * its taus / alg4 arrays are copied).  A and B must hold their values on the
 * device when this is called and stay valid until the request is collected
 * by ihsbin_server_wait.  IHSBIN_ENOMEM: the estimate exceeds the budget. */
int ihsbin_server_submit(ihsbin_server* server, const ihsbin_matrix* A, const void* B,
                         int64_t K, int64_t ldb, double lam_min, double lam_max,
                         const ihsbin_opts* opts, int64_t* id);
/* Wait for request id (timeout_ms < 0: without limit; IHSBIN_EAGAIN when it
 * is not finished in time).  Once finished it is collected: path (optional)
 * receives the built path bound to hip_stream (NULL: the null stream; freed
 * here when path is NULL), info (optional) its timings and report; the return
 * value is the build's status.  An id is collected once. */
int ihsbin_server_wait(ihsbin_server* server, int64_t id, int64_t timeout_ms,
                       void* hip_stream, ihsbin_path** path, ihsbin_request_info* info);
int ihsbin_server_get_stats(ihsbin_server* server, ihsbin_server_stats* stats);
const char* ihsbin_server_last_error(ihsbin_server* server);
/* Finishes every queued request, then frees the workers and every path not
 * yet collected. */
int ihsbin_server_destroy(ihsbin_server* server);

#ifdef __cplusplus
}
#endif

#endif /* IHSBIN_H */
