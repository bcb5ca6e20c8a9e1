// IHS-BIN path build and evaluation (Section 4, Algorithms 2, 3, 5, 6) and the
// C ABI.
//
// Build:
//  1. C = A^T B.
//  2. Sketch SA = S A and the sketched Gram G_S = (SA)^T SA.  With adaptive m
//     the predicted contraction rate of the lowest interval decides whether m
//     grows (Section 5.1 motivates growing m until the sketch is good enough).
//  3. For every interval l (Section 4.2) factor G_S + lam0_l I = L_l L_l^T
//     and form L_l^-1, so P_S R = L^-T (L^-1 R).
//  4. Lanczos on L^-1 (A^T A + lam0 I) L^-T estimates the spectrum
//     [mu_min, mu_max] of P_S (A^T A + lam0 I) per interval; the step size
//     tau = 2 / (mu_min lo/lam0 + mu_max hi/lam0) minimizes the worst
//     contraction over the interval (the optimality condition in the proof
//     of Theorem 1, with measured instead of theoretical eigenvalue bounds).
//  5. Basis recursion of the Proposition for all intervals and right-hand
//     sides at once: one A^T A product over every live column per step; an
//     interval leaves the batch when its increment at both interval ends is
//     small enough.
// Evaluate: x(lam) = tau sum_j (tau (lam - ref))^j ut_j per lambda.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "basis.hpp"
#include "path.hpp"

#include <cstdarg>
#include <cstdlib>

namespace ihs {

bool log_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("IHSBIN_LOG");
    return e && e[0] && e[0] != '0';
  }();
  return on;
}

void logf(const char* fmt, ...) {
  if (!log_enabled()) return;
  va_list ap;
  va_start(ap, fmt);
  std::fputs("[ihsbin] ", stderr);
  std::vfprintf(stderr, fmt, ap);
  std::fputc('\n', stderr);
  va_end(ap);
}

MatView check_matrix(const ihsbin_matrix* A) {
  if (!A) fail(IHSBIN_EINVAL, "A is NULL");
  MatView v{A->format, A->dtype, A->n, A->d, A->ld, A->nnz, A->vals, A->row_ptr, A->col_idx};
  if (v.format != IHSBIN_DENSE && v.format != IHSBIN_CSR) fail(IHSBIN_EINVAL, "bad format");
  if (v.dtype != IHSBIN_F32 && v.dtype != IHSBIN_F64) fail(IHSBIN_EINVAL, "bad dtype");
  if (v.n <= 0 || v.d <= 0) fail(IHSBIN_EINVAL, "n and d must be positive");
  if (v.n > INT32_MAX || v.d > INT32_MAX) fail(IHSBIN_EUNSUP, "n, d must fit int32");
  if (v.format == IHSBIN_DENSE) {
    if (v.ld < v.d) fail(IHSBIN_EINVAL, "ld < d");
    if (!v.vals) fail(IHSBIN_EINVAL, "vals is NULL");
  } else {
    if (v.nnz < 0 || v.nnz > INT32_MAX) fail(IHSBIN_EINVAL, "bad nnz");
    if (!v.row_ptr || (v.nnz > 0 && (!v.col_idx || !v.vals)))
      fail(IHSBIN_EINVAL, "CSR arrays are NULL");
  }
  return v;
}

// CSR structure check on the device: row_ptr monotone from 0 to nnz, columns in range.
__global__ void csr_check_kernel(const int32_t* rp, const int32_t* ci, int64_t n, int64_t d,
                                 int64_t nnz, int* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i == 0 && rp[0] != 0) bad[0] = 1;
    if (i == n && rp[n] != nnz) bad[0] = 1;
    if (i < n) {
      const int32_t a = rp[i], b = rp[i + 1];
      if (b < a || a < 0 || b > nnz) {
        bad[0] = 1;
        continue;
      }
      for (int32_t p = a; p < b; ++p)
        if (ci[p] < 0 || ci[p] >= d) bad[0] = 1;
    }
  }
}

static void validate_csr(Ctx& c, const MatView& A) {
  int* bad = static_cast<int*>(c.ws_status.ensure(64));
  IHS_HIP(hipMemsetAsync(bad, 0, sizeof(int), c.stream));
  int64_t blocks = cdiv(A.n + 1, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(csr_check_kernel, dim3((unsigned)blocks), dim3(256), 0, c.stream, A.row_ptr,
                     A.col_idx, A.n, A.d, A.nnz, bad);
  IHS_CHECK_LAUNCH();
  int h = 0;
  IHS_HIP(hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  IHS_HIP(hipStreamSynchronize(c.stream));
  if (h) fail(IHSBIN_EINVAL, "CSR structure invalid (row_ptr or col_idx)");
}

static int64_t next_pow2(int64_t n) {
  int64_t p = 1;
  while (p < n) p <<= 1;
  return p;
}

// ------------------------------------------------------------------ sketch
// reuse_transform: the SRHT transform D-signs + Walsh-Hadamard of A for this
// seed is still in the context's sketch scratch (only the row sample depends on m).
// r_begin (Gaussian only): rows [r_begin, m) of SA are formed and earlier
// rows are left as they are (a Gaussian row depends on its index alone, so
// a grown sketch keeps the rows already formed, rescaled by the caller).
// SRHT: reuse_transform gathers from the transform a previous call kept
// whole; keep_transform keeps this call's transform whole for such reuse
// (otherwise its last pass writes the sampled rows straight into SA).
static void sketch_apply_impl(Ctx& c, const MatView& A, int kind, int s, int64_t m, uint64_t seed,
                              double* SA, bool reuse_transform = false,
                              int prec = IHSBIN_SKETCH_F64, int64_t r_begin = 0,
                              bool keep_transform = false) {
  hipStream_t st = c.stream;
  if (m <= 0) fail(IHSBIN_EINVAL, "m must be positive");
  if (m > INT32_MAX) fail(IHSBIN_EUNSUP, "m too large");
  if (r_begin < 0 || r_begin >= m || (r_begin > 0 && kind != IHSBIN_GAUSSIAN))
    fail(IHSBIN_EINVAL, "sketch rows out of range");
  c.bytes_moved += matrix_bytes(A) + 8.0 * (double)(m - r_begin) * (double)A.d;
  if (prec != IHSBIN_SKETCH_F64 && prec != IHSBIN_SKETCH_BF16 && prec != IHSBIN_SKETCH_FP8)
    fail(IHSBIN_EINVAL, "unknown sketch precision");
  if (kind == IHSBIN_GAUSSIAN && prec == IHSBIN_SKETCH_BF16) {
    void* work = c.ws_sketch.ensure((size_t)sketch_bf16_work_bytes(m, A.n, A.d));
    const int64_t pd = gaussian_sketch_bf16_part_doubles(m, A.n, A.d);
    double* part = static_cast<double*>(c.ws_part.ensure(sizeof(double) * (size_t)pd));
    gaussian_sketch_bf16(A, seed, m, SA, work, part, pd, st, r_begin);
  } else if (kind == IHSBIN_GAUSSIAN && prec == IHSBIN_SKETCH_FP8) {
    void* work = c.ws_sketch.ensure((size_t)sketch_fp8_work_bytes(m, A.n, A.d));
    const int64_t pd = gaussian_sketch_fp8_part_doubles(m, A.n, A.d);
    double* part = static_cast<double*>(c.ws_part.ensure(sizeof(double) * (size_t)pd));
    gaussian_sketch_fp8(A, seed, m, SA, work, part, pd, st, r_begin);
  } else if (kind == IHSBIN_GAUSSIAN && A.format == IHSBIN_CSR) {
    // (SA)^T = A^T S^T, O(m nnz(A)): each chunk of rows of S is drawn
    // transposed (n x rows), gathered through the column-major copy of A in
    // fixed order (d x rows), and transposed into its rows of SA
    PoolBuf cb(c.pool);
    Csc local;
    const Csc* csc = A.csc;
    if (!csc) {
      build_csc(A, cb.ensure((size_t)csc_work_bytes(A)), local, st);
      csc = &local;
    }
    int64_t rows = (int64_t)((size_t(1) << 30) / (sizeof(double) * (size_t)A.n));
    rows = std::max<int64_t>(1, std::min<int64_t>(rows, 256));
    if (rows > m) rows = m;
    double* St = static_cast<double*>(c.ws_sketch.ensure(sizeof(double) * (size_t)rows * A.n));
    double* Wt = static_cast<double*>(c.ws_tmp.ensure(sizeof(double) * (size_t)rows * A.d));
    double* part = static_cast<double*>(c.ws_part.ensure(
        sizeof(double) * (size_t)std::max<int64_t>(1, csc_partial_doubles(*csc, rows))));
    for (int64_t r0 = r_begin; r0 < m; r0 += rows) {
      const int64_t rn = std::min(rows, m - r0);
      launch_gaussian_fill_t(seed, m, r0, rn, A.n, St, st);
      launch_csc_atb(A, *csc, St, false, rn, rn, part, Wt, rn, st);
      MatView wv;
      wv.format = IHSBIN_DENSE;
      wv.dtype = IHSBIN_F64;
      wv.n = A.d;
      wv.d = rn;
      wv.ld = rn;
      wv.nnz = 0;
      wv.vals = Wt;
      wv.row_ptr = nullptr;
      wv.col_idx = nullptr;
      launch_transpose(wv, SA + r0 * A.d, st);
    }
  } else if (kind == IHSBIN_GAUSSIAN) {
    int64_t rows = (int64_t)((size_t(1) << 30) / (sizeof(double) * (size_t)A.n));
    rows = std::max<int64_t>(64, (rows / 64) * 64);
    if (rows > m) rows = m;
    double* S = static_cast<double*>(c.ws_sketch.ensure(sizeof(double) * (size_t)rows * A.n));
    const DT tb = A.dtype == IHSBIN_F32 ? DT::F32 : DT::F64;
    for (int64_t r0 = r_begin; r0 < m; r0 += rows) {
      const int64_t rn = std::min(rows, m - r0);
      launch_gaussian_fill(seed, m, r0, rn, A.n, S, st);
      const int splits = pick_splits(rn, A.d, A.n, 1);
      Gemm g;
      g.M = rn;
      g.N = A.d;
      g.K = A.n;
      g.A = S;
      g.lda = A.n;
      g.B = A.vals;
      g.ldb = A.ld;
      if (splits > 1) {
        double* part = static_cast<double*>(
            c.ws_part.ensure(sizeof(double) * (size_t)splits * (size_t)rn * (size_t)A.d));
        g.C = part;
        g.ldc = A.d;
        g.strideC = rn * A.d;
        g.splits = splits;
        gemm(g, DT::F64, false, tb, false, st);
        reduce_splits(part, splits, 1, rn, A.d, A.d, rn * A.d, SA + r0 * A.d, A.d, 0, 1.0, 0.0, st);
      } else {
        g.C = SA + r0 * A.d;
        g.ldc = A.d;
        gemm(g, DT::F64, false, tb, false, st);
      }
    }
  } else if (kind == IHSBIN_COUNTSKETCH || kind == IHSBIN_SJLT) {
    if (kind == IHSBIN_COUNTSKETCH) s = 1;
    if (s < 1 || m % s) fail(IHSBIN_EINVAL, "SJLT needs s >= 1 dividing m");
    void* work = c.ws_sketch.ensure((size_t)countsketch_work_bytes(A, m, s));
    countsketch_apply(A, seed, m, s, SA, work, st);
  } else if (kind == IHSBIN_SRHT) {
    const int64_t npad = next_pow2(A.n);
    if (npad > (int64_t(1) << 31)) fail(IHSBIN_EUNSUP, "SRHT order too large");
    char* base = static_cast<char*>(
        c.ws_sketch.ensure(sizeof(double) * (size_t)npad * A.d + (size_t)A.n + 256));
    double* Z = reinterpret_cast<double*>(base);
    int8_t* sg = reinterpret_cast<int8_t*>(base + sizeof(double) * (size_t)npad * A.d);
    int32_t* rows = static_cast<int32_t*>(c.ws_tmp.ensure(sizeof(int32_t) * (size_t)m));
    launch_draw_srht(seed, A.n, npad, m, sg, rows, st);
    const double scale = 1.0 / std::sqrt((double)m);
    if (reuse_transform || keep_transform) {
      if (!reuse_transform) launch_srht_transform(A, sg, npad, Z, st);
      launch_gather_rows(Z, A.d, rows, m, scale, SA, st);
    } else {
      PoolBuf wb(c.pool);
      const int32_t *rstart = nullptr, *rk = nullptr;
      build_row_sample(rows, m, npad, wb.ensure((size_t)row_sample_work_bytes(m, npad)), &rstart,
                       &rk, st);
      if (!launch_srht_transform(A, sg, npad, Z, st, rstart, rk, scale, SA))
        launch_gather_rows(Z, A.d, rows, m, scale, SA, st);
    }
  } else {
    fail(IHSBIN_EINVAL, "unknown sketch type");
  }
}

// Lower triangle (and the diagonal tiles) of G = (SA)^T SA; the strictly
// upper tiles are not computed and hold unspecified values.
// batch > 1: SA holds `batch` blocks of m x d at stride m * d, G `batch`
// blocks of d x d (FP64 only).
static void gram_impl(Ctx& c, const double* SA, int64_t m, int64_t d, double* G,
                      int prec = IHSBIN_GRAM_F64, int batch = 1) {
  if (batch > 1 && prec != IHSBIN_GRAM_F64) fail(IHSBIN_EUNSUP, "batched Gram is FP64 only");
  if (prec == IHSBIN_GRAM_BF16X3) {
    const int splits = gram_bf16x3_splits(m);
    PoolBuf wb(c.pool);
    void* work = wb.ensure((size_t)gram_bf16x3_work_bytes(m, d));
    double* part = static_cast<double*>(
        c.ws_part.ensure(sizeof(double) * (size_t)splits * (size_t)d * (size_t)d));
    gram_bf16x3(SA, m, d, d, work, part, splits, c.stream);
    reduce_splits(part, splits, 1, d, d, d, d * d, G, d, 0, 1.0, 0.0, c.stream);
    return;
  }
  if (prec != IHSBIN_GRAM_F64) fail(IHSBIN_EINVAL, "unknown Gram precision");
  // 64 x 64 lower tiles, ~64 workgroups per CU over the K-splits (a sweep at
  // 65536 x 2048: 8 splits 47, 16 splits 52, 32 splits 57 TFLOP/s)
  const int splits = pick_splits_lower(d, m, std::max<int64_t>(1, 16384 / batch));
  Gemm g;
  g.small_tiles = 1;
  g.M = d;
  g.N = d;
  g.K = m;
  g.A = SA;
  g.lda = d;
  g.strideA = m * d;
  g.B = SA;
  g.ldb = d;
  g.strideB = m * d;
  g.batch = batch;
  g.lower_only = 1;
  if (splits > 1) {
    double* part = static_cast<double*>(c.ws_part.ensure(
        sizeof(double) * (size_t)splits * (size_t)batch * (size_t)d * (size_t)d));
    g.C = part;
    g.ldc = d;
    g.strideC = d * d;
    g.splits = splits;
    gemm(g, DT::F64, true, DT::F64, false, c.stream);
    reduce_splits(part, splits, batch, d, d, d, d * d, G, d, d * d, 1.0, 0.0, c.stream);
  } else {
    g.C = G;
    g.ldc = d;
    g.strideC = d * d;
    gemm(g, DT::F64, true, DT::F64, false, c.stream);
  }
}

// Whether P_S keeps its factors in split form (PsFactors) at dimension d.  The
// split form skips two GEMMs of the inverse (about L d^3 / 4 flop) but applies
// through three products instead of one.  Where those run split-K (d >= 1024)
// their extra launches outweigh the saving until d reaches about 3000
// (measured: d = 2048 path 43.2 ms whole, 44.4 ms split; d = 4096 and 8192
// 7 ms and 59 ms faster split).  Below 1024 a single build is launch-bound
// (256 served 2048 x 256 builds: 796 paths/s split against 914 whole), while
// a batched build, whose launches cover every problem, gains (2990 -> 3167
// paths/s for the same 256 problems).
static bool split_factors(int64_t d, bool batched = false) {
  return d >= 3072 || (batched && d < 1024);
}

// H_l = G + lam0_l I, factor in place, and Linv_l = L_l^-1.
// gper > 0: matrix l is built from G block l / gper (blocks of d x d), so the
// factors of several Grams run in one batch.
// split: leave out the top split's lower-left block of L^-1 (applied through
// X11, L21, X22 instead, see PsFactors); returns that split (0: Linv is the
// whole inverse).
static int64_t factor_impl(Ctx& c, const double* G, int64_t d, const std::vector<double>& lam0s,
                           double* Lf, double* Linv, PoolBuf& dinv_buf, PoolBuf& lam_buf,
                           int gper = 0, bool split = false) {
  const int nl = (int)lam0s.size();
  double* lam_dev = static_cast<double*>(lam_buf.ensure(sizeof(double) * nl));
  IHS_HIP(hipMemcpyAsync(lam_dev, lam0s.data(), sizeof(double) * nl, hipMemcpyHostToDevice, c.stream));
  launch_build_shifted(G, d, lam_dev, nl, Lf, c.stream, gper > 0 ? gper : nl);
  const int64_t nblk = cdiv(d, kNB);
  double* dinv = static_cast<double*>(dinv_buf.ensure(sizeof(double) * nl * nblk * kNB * kNB));
  int* status = static_cast<int*>(c.ws_status.ensure(64));
  IHS_HIP(hipMemsetAsync(status, 0, sizeof(int), c.stream));
  PoolBuf work(c.pool);
  if (Linv) {
    // factor and inverse together, by halves
    double* wk = static_cast<double*>(work.ensure(
        sizeof(double) * (size_t)std::max<int64_t>(1, factor_inverse_work_doubles(d, nl))));
    factor_inverse_batched(Lf, Linv, d, nl, dinv, status, wk, c.stream, !split);
  } else {
    cholesky_batched(Lf, d, nl, dinv, status, c.stream);
  }
  int h = 0;
  IHS_HIP(hipMemcpyAsync(&h, status, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  IHS_HIP(hipStreamSynchronize(c.stream));
  if (h) fail(IHSBIN_ENOTSPD, "sketched Hessian not positive definite");
  return Linv && split ? factor_top_split(d) : 0;
}

// The preconditioner P_S = L^-T L^-1 of every interval: X holds L^-1 whole
// (n1 == 0) or only its diagonal blocks X11 = L11^-1 (n1 x n1) and
// X22 = L22^-1, with L21 read from the Cholesky factor Lf; then
//   L^-1 [v1; v2] = [X11 v1; X22 (v2 - L21 X11 v1)],
//   L^-T [y1; y2] = [X11^T (y1 - L21^T X22^T y2); X22^T y2],
// which reads the same bytes as the whole inverse (X11, L21, X22 are its
// quarters) without the two GEMMs that would form its lower-left block.
struct PsFactors {
  const double* X = nullptr;
  const double* Lf = nullptr;
  int64_t n1 = 0;
};

// Z = P R for every active position: P_a = Linv_{ids[a]}^T Linv_{ids[a]}.
// Each product reads a whole triangular factor for a few columns, so it is
// bound by that read: K is split until ~2048 workgroups stream the factors.
static int apply_p_splits(int na, int64_t d, int64_t cw) {
  const int64_t tiles = (int64_t)na * cdiv(d, 256) * cdiv(cw, cw <= 16 ? 16 : 32);
  int splits = (int)std::min<int64_t>(16, std::max<int64_t>(1, cdiv(2048, tiles)));
  if (d < 1024 || cw > 32) splits = 1;
  return splits;
}

// Grow the workspaces of apply_p for na positions of cw columns (the split-K
// partials at most 16 splits, the split factors' block temporary), so that
// calls captured into a graph allocate nothing.
static void apply_p_reserve(Ctx& c, int na, int64_t d, int64_t cw) {
  const int splits = apply_p_splits(na, d, cw);
  if (splits > 1) c.ws_part.ensure(sizeof(double) * (size_t)16 * na * (size_t)d * (size_t)cw);
  c.ws_ps.ensure(sizeof(double) * (size_t)d * na * (size_t)cw);
}

// C_a = alpha op(A_a) B_a + beta C_a for na positions: A_a = A0 + ids[a] d^2
// (row stride d), op(A_a) M x K; B_a, C_a = N columns from column a N of B, C
// (row strides ldb, ldc).  Skinny products split K over the factor's read
// (fixed-order reduction).
static void ps_product(Ctx& c, const double* A0, int64_t d, const int32_t* ids, int na, bool trans,
                       int tri, int64_t M, int64_t N, int64_t K, const double* B, int64_t ldb,
                       double* C, int64_t ldc, double alpha, double beta) {
  if (M <= 0 || N <= 0) return;
  const int splits = apply_p_splits(na, std::max(M, K), N);
  Gemm g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A0;
  g.lda = d;
  g.strideA = d * d;
  g.amap = ids;
  g.B = B;
  g.ldb = ldb;
  g.strideB = N;
  g.batch = na;
  g.tri = tri;
  if (splits > 1) {
    double* part = static_cast<double*>(
        c.ws_part.ensure(sizeof(double) * (size_t)splits * na * (size_t)M * (size_t)N));
    g.C = part;
    g.ldc = N;
    g.strideC = M * N;
    g.splits = splits;
    gemm(g, DT::F64, trans, DT::F64, false, c.stream);
    reduce_splits(part, splits, na, M, N, N, M * N, C, ldc, N, alpha, beta, c.stream);
  } else {
    g.C = C;
    g.ldc = ldc;
    g.strideC = N;
    g.alpha = alpha;
    g.beta = beta;
    gemm(g, DT::F64, trans, DT::F64, false, c.stream);
  }
}

// Y = L^-1 X (lower) or L^-T X (upper) for the split factors, na positions of
// N columns (row stride ld); tmp: max(n1, n2) x (na N) doubles.
static void ps_split_apply(Ctx& c, const PsFactors& F, const int32_t* ids, int na, int64_t d,
                           int64_t N, int64_t ld, bool upper, const double* X, double* Y,
                           double* tmp) {
  const int64_t n1 = F.n1, n2 = d - n1, ldt = (int64_t)na * N;
  const double* X11 = F.X;
  const double* X22 = F.X + n1 * d + n1;
  const double* L21 = F.Lf + n1 * d;
  hipStream_t st = c.stream;
  if (!upper) {
    ps_product(c, X11, d, ids, na, false, 1, n1, N, n1, X, ld, Y, ld, 1.0, 0.0);
    launch_copy_rect(X + n1 * ld, ld, n2, ldt, tmp, ldt, st);
    ps_product(c, L21, d, ids, na, false, 0, n2, N, n1, Y, ld, tmp, ldt, -1.0, 1.0);
    ps_product(c, X22, d, ids, na, false, 1, n2, N, n2, tmp, ldt, Y + n1 * ld, ld, 1.0, 0.0);
  } else {
    ps_product(c, X22, d, ids, na, true, 2, n2, N, n2, X + n1 * ld, ld, Y + n1 * ld, ld, 1.0, 0.0);
    launch_copy_rect(X, ld, n1, ldt, tmp, ldt, st);
    ps_product(c, L21, d, ids, na, true, 0, n1, N, n2, Y + n1 * ld, ld, tmp, ldt, -1.0, 1.0);
    ps_product(c, X11, d, ids, na, true, 2, n1, N, n1, tmp, ldt, Y, ld, 1.0, 0.0);
  }
}

static void apply_p(Ctx& c, const PsFactors& F, const int32_t* ids_dev, int na, int64_t d,
                    int64_t cw, int64_t ld, const double* R, double* T, double* Z) {
  if (F.n1 > 0) {
    double* tmp = static_cast<double*>(
        c.ws_ps.ensure(sizeof(double) * (size_t)std::max(F.n1, d - F.n1) * na * (size_t)cw));
    ps_split_apply(c, F, ids_dev, na, d, cw, ld, false, R, T, tmp);
    ps_split_apply(c, F, ids_dev, na, d, cw, ld, true, T, Z, tmp);
    return;
  }
  const double* Linv_all = F.X;
  const int splits = apply_p_splits(na, d, cw);
  double* part = splits > 1 ? static_cast<double*>(c.ws_part.ensure(
                                  sizeof(double) * (size_t)splits * na * (size_t)d * (size_t)cw))
                            : nullptr;
  auto tri_product = [&](bool trans, const double* X, double* Y) {
    Gemm g;
    g.M = d;
    g.N = cw;
    g.K = d;
    g.A = Linv_all;
    g.lda = d;
    g.strideA = d * d;
    g.amap = ids_dev;
    g.B = X;
    g.ldb = ld;
    g.strideB = cw;
    g.batch = na;
    g.tri = trans ? 2 : 1;
    if (splits > 1) {
      g.C = part;
      g.ldc = cw;
      g.strideC = d * cw;
      g.splits = splits;
      gemm(g, DT::F64, trans, DT::F64, false, c.stream);
      reduce_splits(part, splits, na, d, cw, cw, d * cw, Y, ld, cw, 1.0, 0.0, c.stream);
    } else {
      g.C = Y;
      g.ldc = ld;
      g.strideC = cw;
      gemm(g, DT::F64, trans, DT::F64, false, c.stream);
    }
  };
  tri_product(false, R, T);
  tri_product(true, T, Z);
}

// Symmetric eigen-decomposition of a small dense matrix by cyclic Jacobi.
static void jacobi_eig(int n, std::vector<double>& a, std::vector<double>& v) {
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double x = a[(size_t)i * n + j] * a[(size_t)i * n + j];
        tot += x;
        if (i != j) off += x;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
        const double th = (aqq - app) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {
          const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = cs * akp - sn * akq;
          a[(size_t)k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = cs * apk - sn * aqk;
          a[(size_t)q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
          v[(size_t)k * n + p] = cs * vkp - sn * vkq;
          v[(size_t)k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
}

struct Spec {
  double mu_min, mu_max;
};

// Ritz values of the Lanczos tridiagonal of column a after n steps:
// (theta_min, theta_max) and their residual bounds |beta_n s_n|.
struct Ritz {
  double tmin, tmax, rmin, rmax;
};

static Ritz ritz_extremes(const std::vector<double>& h, int na, int J, int a, int n_steps) {
  int n = n_steps;
  for (int j = 0; j < n_steps - 1; ++j)
    if (!(h[(size_t)na * J + (size_t)a * J + j] > 1e-14 * std::fabs(h[(size_t)a * J + j]) + 1e-300)) {
      n = j + 1;
      break;
    }
  std::vector<double> Tm((size_t)n * n, 0.0), V;
  for (int j = 0; j < n; ++j) {
    Tm[(size_t)j * n + j] = h[(size_t)a * J + j];
    if (j + 1 < n) {
      const double b = h[(size_t)na * J + (size_t)a * J + j];
      Tm[(size_t)j * n + j + 1] = b;
      Tm[(size_t)(j + 1) * n + j] = b;
    }
  }
  jacobi_eig(n, Tm, V);
  const double bres = n == n_steps ? h[(size_t)na * J + (size_t)a * J + n_steps - 1] : 0.0;
  int imin = 0, imax = 0;
  for (int i = 1; i < n; ++i) {
    if (Tm[(size_t)i * n + i] < Tm[(size_t)imin * n + imin]) imin = i;
    if (Tm[(size_t)i * n + i] > Tm[(size_t)imax * n + imax]) imax = i;
  }
  Ritz r;
  r.tmin = Tm[(size_t)imin * n + imin];
  r.tmax = Tm[(size_t)imax * n + imax];
  r.rmin = std::fabs(bres * V[(size_t)(n - 1) * n + imin]);
  r.rmax = std::fabs(bres * V[(size_t)(n - 1) * n + imax]);
  return r;
}

// Lanczos with full re-orthogonalization, one column a per operator
// B_a = Linv_{ids[a]} (A^T A + shifts[a] I) Linv_{ids[a]}^T.  early: when
// enabled, the run may stop once early(Ritz extremes of every column) returns
// true (Ritz values bound the spectrum from inside).
// nv = 2: columns a and a + na/2 share a factor (ids holds na/2 entries).
// The A^T A product of the working form (one matrix): S = A^T A T for w
// columns of row stride ld.
// f32: the products on the FP32 matrix cores (dense FP32 A; ignored
// otherwise).  The spectrum estimates take them when the basis may: their
// Ritz values move by ~1e-7 relative, far inside the bounds' 2 % slack.
struct AtaProd {
  Ctx& c;
  const MatView& A;
  bool f32 = false;
  int64_t d() const { return A.d; }
  int64_t slack(int64_t) const { return 0; }
  void operator()(const double* T, int64_t w, int64_t ld, double* S) const {
    ata_apply(c, A, T, w, ld, S, ld, nullptr, ld, f32);
  }
};

template <class Early, class Prod>
static std::vector<Spec> spectrum_impl(Ctx& c, const Prod& prod, const PsFactors& F,
                                       const std::vector<int32_t>& ids,
                                       const std::vector<double>& shifts, int J, uint64_t seed,
                                       Early early, int nv = 1) {
  hipStream_t st = c.stream;
  const int na = (int)shifts.size();
  if ((int)ids.size() * nv != na) fail(IHSBIN_EINVAL, "spectrum: ids and shifts disagree");
  const int64_t d = prod.d();
  if (J < 2) J = 2;
  if (J > d) J = (int)d;
  if (J > 63) J = 63;
  // padded so the A^T A product runs on whole tiles
  const int64_t ld = padded_width(na + prod.slack(na));
  const size_t vec = sizeof(double) * (size_t)d * ld;
  PoolBuf Qb(c.pool), Tb(c.pool), Sb(c.pool), Wb(c.pool), ab(c.pool), idb(c.pool), lb(c.pool), trb(c.pool);
  double* trs = static_cast<double*>(trb.ensure(sizeof(double) * trmv_scratch_doubles(d, na)));
  double* Q = static_cast<double*>(Qb.ensure(vec * (J + 1)));
  double* T = static_cast<double*>(Tb.ensure(vec));
  double* S = static_cast<double*>(Sb.ensure(vec));
  double* Wv = static_cast<double*>(Wb.ensure(vec));
  double* alpha = static_cast<double*>(ab.ensure(sizeof(double) * 2 * na * J));
  double* beta = alpha + (size_t)na * J;
  int32_t* ids_dev = static_cast<int32_t*>(idb.ensure(sizeof(int32_t) * na));
  double* lam_dev = static_cast<double*>(lb.ensure(sizeof(double) * na));
  // one id per column (column b + v nm takes ids[b]): the triangular
  // products read the first nm, the L21 products all na
  std::vector<int32_t> col_ids((size_t)na);
  for (int a = 0; a < na; ++a) col_ids[a] = ids[a % ids.size()];
  IHS_HIP(hipMemcpyAsync(ids_dev, col_ids.data(), sizeof(int32_t) * na, hipMemcpyHostToDevice, st));
  IHS_HIP(hipMemcpyAsync(lam_dev, shifts.data(), sizeof(double) * na, hipMemcpyHostToDevice, st));
  launch_lanczos_start(seed, d, na, ld, Q, st);
  std::vector<double> h(2 * (size_t)na * J);
  int steps = J;
  // Y = L^-1 X or L^-T X for every column (its interval's factor); the
  // split factors go through their diagonal blocks and L21 (PsFactors)
  PoolBuf tmb(c.pool);
  double* tmv = F.n1 > 0 ? static_cast<double*>(tmb.ensure(
                               sizeof(double) * (size_t)std::max(F.n1, d - F.n1) * ld))
                         : nullptr;
  auto linv = [&](bool transpose, const double* X, double* Y) {
    if (F.n1 == 0) {
      launch_trmv(F.X, d, ids_dev, na, transpose, X, ld, Y, ld, trs, st, nv);
      return;
    }
    const int64_t n1 = F.n1, n2 = d - n1;
    const double* X11 = F.X;
    const double* X22 = F.X + n1 * d + n1;
    const double* L21 = F.Lf + n1 * d;
    if (!transpose) {
      launch_trmv_block(X11, n1, d, d * d, ids_dev, na, false, X, ld, Y, ld, trs, st, nv);
      launch_copy_rect(X + n1 * ld, ld, n2, na, tmv, ld, st);
      ps_product(c, L21, d, ids_dev, na, false, 0, n2, 1, n1, Y, ld, tmv, ld, -1.0, 1.0);
      launch_trmv_block(X22, n2, d, d * d, ids_dev, na, false, tmv, ld, Y + n1 * ld, ld, trs, st,
                        nv);
    } else {
      launch_trmv_block(X22, n2, d, d * d, ids_dev, na, true, X + n1 * ld, ld, Y + n1 * ld, ld,
                        trs, st, nv);
      launch_copy_rect(X, ld, n1, na, tmv, ld, st);
      ps_product(c, L21, d, ids_dev, na, true, 0, n1, 1, n2, Y + n1 * ld, ld, tmv, ld, -1.0, 1.0);
      launch_trmv_block(X11, n1, d, d * d, ids_dev, na, true, tmv, ld, Y, ld, trs, st, nv);
    }
  };
  for (int j = 0; j < J; ++j) {
    linv(true, Q + (size_t)j * d * ld, T);           // T = Linv^T q
    prod(T, na, ld, S);                                // S = A^T A T
    launch_add_shift(S, T, d, na, ld, lam_dev, st);   // S += shift T
    linv(false, S, Wv);                                // W = Linv S
    launch_lanczos_orth(Q, Wv, d, na, ld, j, J, alpha, beta, st);
    // checked after every step from early.min_steps on (a sketch far too small
    // shows within two or three steps; converged extremes stop the run)
    if (early.enabled && j + 1 >= early.min_steps && j + 1 < J) {
      IHS_HIP(hipMemcpyAsync(h.data(), alpha, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
      IHS_HIP(hipStreamSynchronize(st));
      std::vector<Ritz> rz(na);
      for (int a = 0; a < na; ++a) rz[a] = ritz_extremes(h, na, J, a, j + 1);
      if (early(rz)) {
        steps = j + 1;
        break;
      }
    }
  }
  IHS_HIP(hipMemcpyAsync(h.data(), alpha, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
  IHS_HIP(hipStreamSynchronize(st));
  logf("lanczos: %d columns, %d of %d steps", na, steps, J);
  std::vector<Spec> out(na);
  for (int a = 0; a < na; ++a) {
    const Ritz rz = ritz_extremes(h, na, J, a, steps);
    if (log_enabled() && (a % 8 == 0 || a == na - 1))
      logf("  column %d: ritz [%.6g, %.6g] residual bounds [%.3g, %.3g]", a, rz.tmin, rz.tmax,
           rz.rmin, rz.rmax);
    Spec sp;
    sp.mu_max = (rz.tmax + rz.rmax) * 1.02;
    sp.mu_min = std::max(rz.tmin - rz.rmin, 0.5 * rz.tmin);
    if (!(sp.mu_min > 0.0) || !(sp.mu_max > sp.mu_min) || !std::isfinite(sp.mu_max))
      fail(IHSBIN_ENOTSPD, "spectrum estimate failed");
    out[a] = sp;
  }
  return out;
}

struct NoEarly {
  bool enabled = false;
  int min_steps = 0;
  bool operator()(const std::vector<Ritz>&) const { return false; }
};
// Columns 0 and 1 hold the lower and upper end of one interval: the Ritz
// values lie inside the spectra, so their rate is a lower bound.
struct EarlyIfSlow {
  bool enabled = true;
  int min_steps = 2;
  double target;
  bool operator()(const std::vector<Ritz>& r) const {
    const double cmin = r[0].tmin, cmax = r[1].tmax;
    return (cmax - cmin) / (cmax + cmin) > target;
  }
};

// The same for `groups` x P column blocks of problems of one shape: columns
// (g P + p) per .. + per - 1 belong to problem p (batched builds).
struct BatchProd {
  Ctx& c;
  const MatView& A;
  int64_t strideA;
  int P, groups;
  int64_t d() const { return A.d; }
  int64_t slack(int64_t na) const { return ata_batch_slack(std::max<int64_t>(1, na / (groups * P))); }
  void operator()(const double* T, int64_t w, int64_t ld, double* S) const {
    const int64_t per = w / ((int64_t)groups * P);
    if (per * groups * P != w) fail(IHSBIN_EINVAL, "batched product: ragged column blocks");
    ata_apply_batch(c, A, strideA, P, groups, per, T, ld, S, ld);
  }
};

// P problems probed together (columns p: lower end, P + p: upper end of the
// lowest interval of problem p): stop as soon as any of them is too slow.
struct EarlyIfAnySlow {
  bool enabled = true;
  int min_steps = 2;
  int P = 1;
  double target;
  bool operator()(const std::vector<Ritz>& r) const {
    for (int p = 0; p < P; ++p) {
      const double cmin = r[p].tmin, cmax = r[P + p].tmax;
      if ((cmax - cmin) / (cmax + cmin) > target) return true;
    }
    return false;
  }
};

// Spectrum bounds over whole intervals.  In the symmetric form
// Linv (A^T A + lam I) Linv^T = B_0 + lam Linv Linv^T every Rayleigh quotient
// grows with lam, so for lam in [lo, hi] the spectrum of P_S (A^T A + lam I)
// lies between the smallest eigenvalue at lo and the largest at hi.  One
// Lanczos column per interval end; fids[i] is the factor of interval i.
template <class Early, class Prod>
static std::vector<Spec> interval_spectra(Ctx& c, const Prod& prod, const PsFactors& F,
                                          const std::vector<int32_t>& fids,
                                          const std::vector<double>& los,
                                          const std::vector<double>& his, int J, uint64_t seed,
                                          Early early) {
  const int ni = (int)fids.size();
  std::vector<double> shifts(2 * ni);
  for (int i = 0; i < ni; ++i) {
    shifts[i] = los[i];
    shifts[ni + i] = his[i];
  }
  const std::vector<Spec> col = spectrum_impl(c, prod, F, fids, shifts, J, seed, early, 2);
  std::vector<Spec> out(ni);
  for (int i = 0; i < ni; ++i) {
    out[i].mu_min = col[i].mu_min;
    out[i].mu_max = col[ni + i].mu_max;
    if (!(out[i].mu_max > out[i].mu_min)) fail(IHSBIN_ENOTSPD, "spectrum estimate failed");
  }
  return out;
}

// SA = A in FP64 (n x d contiguous): dense rows widened, CSR rows scattered
// into their own rows.
static void copy_rows_f64(Ctx& c, const MatView& A, double* SA) {
  if (A.format == IHSBIN_DENSE) {
    launch_widen_rows(A.vals, A.dtype, A.n, A.d, A.ld, SA, c.stream);
    return;
  }
  launch_csr_densify(A, SA, c.stream);
}

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

// The primal form every step runs on: A itself, or for n < d the dual problem
// (Section 5.2, Eq. (ls_reg:d)).  The dual's optimality condition
// (A A^T + lam I) z = b is the primal form for the d x n matrix A^T with
// right-hand side b itself, and x = A^T z; A^T is materialized once.
// C = A^T B (dual: B widened), d x K.
struct Form {
  MatView A;
  bool dual = false;
  PoolBuf At, Cb, cscb, htb;
  Csc csc;     // CSR: the column-major copy the transposed products gather from
  HeadTail ht;  // CSR: its dense head columns and sparse tail
  double* C = nullptr;
  explicit Form(Pool& p) : At(p), Cb(p), cscb(p), htb(p) {}
};

static void make_form(Ctx& c, const MatView& A0, const void* B, int64_t K, int64_t ldb, Form& f) {
  if (!B) fail(IHSBIN_EINVAL, "B is NULL");
  if (K < 1 || ldb < K) fail(IHSBIN_EINVAL, "need K >= 1 and ldb >= K");
  f.dual = A0.n < A0.d;
  if (f.dual && A0.format != IHSBIN_DENSE)
    fail(IHSBIN_EUNSUP, "n < d with a CSR matrix (the dual is built for dense A)");
  f.A = A0;
  if (f.dual) {
    const size_t es = A0.dtype == IHSBIN_F32 ? 4 : 8;
    void* At = f.At.ensure(es * (size_t)A0.n * (size_t)A0.d);
    launch_transpose(A0, At, c.stream);
    f.A.n = A0.d;
    f.A.d = A0.n;
    f.A.ld = A0.n;
    f.A.vals = At;
  }
  if (f.A.format == IHSBIN_CSR) {
    validate_csr(c, f.A);
    build_csc(f.A, f.cscb.ensure((size_t)csc_work_bytes(f.A)), f.csc, c.stream);
    f.A.csc = &f.csc;
    build_head_tail(f.A, f.csc, f.htb, f.ht, c.stream);
    if (f.ht.h > 0) f.A.ht = &f.ht;
  }
  const int64_t d = f.A.d;
  f.C = static_cast<double*>(f.Cb.ensure(sizeof(double) * d * K));
  if (f.dual) launch_widen_rows(B, A0.dtype, d, K, ldb, f.C, c.stream);
  else atb_apply(c, f.A, B, K, ldb, f.C);
}

// Sketch of the working form at a given m into SA, then G = (SA)^T SA.  A
// sketch of m >= n rows is no cheaper than A itself and embeds it no better
// than S = I does: then SA = A and P_S is the exact (A^T A + lam0 I)^-1.
struct Sketcher {
  Ctx& c;
  const MatView& A;
  const ihsbin_opts& o;
  int s;
  int64_t m_cap;
  PoolBuf SAb, Gb;
  double* G;
  int trials = 0;
  Sketcher(Ctx& cc, const MatView& AA, const ihsbin_opts& oo)
      : c(cc), A(AA), o(oo), SAb(cc.pool), Gb(cc.pool) {
    s = o.sketch == IHSBIN_SJLT ? std::max(1, o.sjlt_s) : 1;
    const int64_t m = initial_m(2 * A.d);
    m_cap = o.m_max > 0 ? o.m_max : std::max<int64_t>(m, std::min<int64_t>(A.n, 32 * A.d));
    if (o.sketch == IHSBIN_SRHT) m_cap = std::min(m_cap, std::max(m, next_pow2(A.n)));
    if (exact_switch() && o.m_max <= 0) m_cap = std::max(m_cap, A.n);
    G = static_cast<double*>(Gb.ensure(sizeof(double) * A.d * A.d));
  }
  // adaptive_m = 3: a Gaussian sketch costs 2 m n d multiply-adds against
  // 2 n d^2 for A^T A itself; the BF16 and FP8 forms run at about 8 times the
  // FP64 Gram's rate (the FP64 form at the same rate), so past exact_rows()
  // rows the sketch is dearer than the exact Hessian, and m jumps to n (S = I;
  // dense A only: S = I copies A densely)
  bool exact_switch() const {
    return o.adaptive_m == 3 && o.sketch == IHSBIN_GAUSSIAN && A.format == IHSBIN_DENSE;
  }
  int64_t exact_rows() const { return (o.sketch_prec == IHSBIN_SKETCH_F64 ? 1 : 8) * A.d; }
  int64_t next_m(int64_t want) const {
    return exact_switch() && want > exact_rows() ? std::max(want, A.n) : want;
  }
  // o.m rounded up to a multiple of s, or dflt when o.m is 0
  int64_t initial_m(int64_t dflt) const {
    int64_t m = o.m > 0 ? o.m : std::max<int64_t>(1, dflt);
    if (m % s) m += s - m % s;
    return m;
  }
  // Rows of a Gaussian sketch already formed (0: none): row r of S depends
  // on r alone up to the common factor 1 / sqrt(m), so growing m keeps them,
  // rescaled by sqrt(m_old / m), and draws only the new rows.
  int64_t gauss_rows = 0;
  bool srht_whole = false;  // the SRHT transform of the last call is complete
  // CountSketch / SJLT of a CSR matrix: SA is kept sparse and its Gram is
  // formed from its entries (gram_prec does not apply)
  bool sparse_sketch() const {
    return A.format == IHSBIN_CSR &&
           (o.sketch == IHSBIN_COUNTSKETCH || o.sketch == IHSBIN_SJLT) && A.d <= kSparseGramMaxD;
  }
  void operator()(int64_t mm) {
    const int64_t rows = mm >= A.n ? A.n : mm;
    if (mm < A.n && sparse_sketch()) {
      if (mm > INT32_MAX || mm % s) fail(IHSBIN_EINVAL, "sketch size");
      void* work = c.ws_sketch.ensure((size_t)countsketch_sparse_work_bytes(A, mm, s));
      void* out = SAb.ensure((size_t)countsketch_sparse_out_bytes(A, mm, s));
      SparseRows sa;
      const int64_t nnz_s = countsketch_apply_sparse(A, o.seed, mm, s, work, out, sa, c.stream);
      c.bytes_moved += matrix_bytes(A) + 12.0 * (double)nnz_s;
      logf("m=%lld: sparse sketch with %lld entries", (long long)mm, (long long)nnz_s);
      sparse_gram(c, sa, G);
      gauss_rows = 0;
      ++trials;
      return;
    }
    if (mm >= A.n) {
      double* SA = static_cast<double*>(SAb.ensure(sizeof(double) * rows * A.d));
      logf("m=%lld >= n=%lld: exact Hessian (S = I)", (long long)mm, (long long)A.n);
      copy_rows_f64(c, A, SA);
      gauss_rows = 0;
    } else if (o.sketch == IHSBIN_GAUSSIAN && gauss_rows > 0 && mm > gauss_rows) {
      PoolBuf grown(c.pool);
      double* SA = static_cast<double*>(grown.ensure(sizeof(double) * rows * A.d));
      launch_scale_copy(static_cast<const double*>(SAb.p), gauss_rows * A.d,
                        std::sqrt((double)gauss_rows / (double)mm), SA, c.stream);
      std::swap(SAb.p, grown.p);  // the old rows go back to the pool (stream-ordered)
      std::swap(SAb.bytes, grown.bytes);
      logf("m=%lld: keeps the %lld Gaussian rows formed, draws %lld", (long long)mm,
           (long long)gauss_rows, (long long)(mm - gauss_rows));
      sketch_apply_impl(c, A, o.sketch, s, mm, o.seed, SA, false, o.sketch_prec, gauss_rows);
      gauss_rows = mm;
    } else {
      double* SA = static_cast<double*>(SAb.ensure(sizeof(double) * rows * A.d));
      // an SRHT keeps its whole transform only while a later probe could
      // sample it again (m below the cap)
      const bool srht = o.sketch == IHSBIN_SRHT;
      const bool keep = srht && o.adaptive_m != 0 && mm < m_cap;
      sketch_apply_impl(c, A, o.sketch, s, mm, o.seed, SA, trials > 0 && srht && srht_whole,
                        o.sketch_prec, 0, keep);
      if (srht) srht_whole = keep || (trials > 0 && srht_whole);
      gauss_rows = o.sketch == IHSBIN_GAUSSIAN ? mm : 0;
    }
    gram_impl(c, static_cast<const double*>(SAb.p), rows, A.d, G, o.gram_prec);
    ++trials;
  }
  void release() {
    SAb.release();
    Gb.release();
  }
};

// Adaptive sketch dimension (Section 5.1, Algorithm 4): IHS on
// f(X) = 1/2 ||A X - B||^2 + lam/2 ||X||^2 from X = 0 with the direction
// D = P_S grad f, delta = <D, grad f>, a backtracking (Armijo) step
// tau = gamma1^j, and m doubled (S redrawn at 2m) whenever an update leaves
// delta_{k+1} >= gamma3 delta_k.  f is quadratic, so with H D = A^T A D + lam D
// from one pass over A, f(X - tau D) - f(X) = -tau delta + tau^2 <D, H D> / 2
// decides every trial step, and grad f(X - tau D) = grad f - tau H D: one
// pass per update.  The final sketch is left in sk (its G and SA).
// trace (optional): 5 values per update (m, tau, delta_k, delta_{k+1} from
// the same sketch, 1 if m doubled).
static ihsbin_alg4_result alg4_impl(Ctx& c, const MatView& A, const double* C, int64_t K,
                                    double lam, int64_t m0, const ihsbin_alg4_opts& p,
                                    Sketcher& sk, double* X_out, int64_t ldx,
                                    std::vector<double>* trace) {
  if (!(p.gamma1 > 0.0 && p.gamma1 < 1.0) || !(p.gamma2 > 0.0 && p.gamma2 < 1.0) ||
      !(p.gamma3 > 0.0) || !(p.eps >= 0.0) || p.max_iter < 0 || p.max_armijo < 1)
    fail(IHSBIN_EINVAL, "Algorithm 4 parameters out of range");
  if (!(lam > 0.0) || !std::isfinite(lam)) fail(IHSBIN_EINVAL, "need lam > 0");
  Timer t0;
  hipStream_t st = c.stream;
  const int64_t d = A.d, cnt = d * K;
  PoolBuf xb(c.pool), gb(c.pool), db(c.pool), tb(c.pool), wb(c.pool), lfb(c.pool), lib(c.pool),
      dinvb(c.pool), lamb(c.pool), idb(c.pool), partb(c.pool);
  double* X = static_cast<double*>(xb.ensure(sizeof(double) * cnt));
  double* Gr = static_cast<double*>(gb.ensure(sizeof(double) * cnt));
  double* D = static_cast<double*>(db.ensure(sizeof(double) * cnt));
  double* T = static_cast<double*>(tb.ensure(sizeof(double) * cnt));
  double* W = static_cast<double*>(wb.ensure(sizeof(double) * cnt));
  double* Lf = static_cast<double*>(lfb.ensure(sizeof(double) * d * d));
  double* Li = static_cast<double*>(lib.ensure(sizeof(double) * d * d));
  int32_t* ids = static_cast<int32_t*>(idb.ensure(sizeof(int32_t)));
  IHS_HIP(hipMemsetAsync(ids, 0, sizeof(int32_t), st));
  double* part = static_cast<double*>(partb.ensure(sizeof(double) * (dots3_part_doubles() + 3)));
  double* dev_out = part + dots3_part_doubles();
  double h[3];
  auto dots = [&](const double* Wp) {
    launch_dots3(D, Gr, Wp, cnt, part, dev_out, st);
    IHS_HIP(hipMemcpyAsync(h, dev_out, sizeof(h), hipMemcpyDeviceToHost, st));
    IHS_HIP(hipStreamSynchronize(st));
  };
  PsFactors F;
  auto redraw = [&](int64_t m) {
    sk(m);
    F.n1 = factor_impl(c, sk.G, d, {lam}, Lf, Li, dinvb, lamb, 0, split_factors(d));
    F.X = Li;
    F.Lf = Lf;
  };
  // D = P_S Gr and delta = <D, Gr>
  auto direction = [&]() {
    apply_p(c, F, ids, 1, d, K, K, Gr, T, D);
    dots(nullptr);
    return h[0];
  };
  ihsbin_alg4_result r;
  std::memset(&r, 0, sizeof(r));
  int64_t m = m0;
  redraw(m);
  launch_alg4_init(C, X, Gr, cnt, st);
  double delta = direction();
  r.delta0 = delta;
  int k = 0;
  while (delta > p.eps * r.delta0 && k < p.max_iter) {
    ata_apply(c, A, D, K, K, W, K, nullptr);
    dots(W);
    const double q = h[1] + lam * h[2];  // <D, H D>
    double tau = 1.0;
    int j = 0;
    while (!(-tau * delta + 0.5 * tau * tau * q <= -p.gamma2 * tau * delta)) {
      if (++j >= p.max_armijo) fail(IHSBIN_ENOCONV, "Armijo search found no step");
      tau *= p.gamma1;
    }
    launch_alg4_step(X, Gr, D, W, cnt, tau, lam, st);
    const double dn = direction();
    const int64_t m_step = m;
    int doubled = 0;
    double delta_new = dn;
    if (dn >= p.gamma3 * delta && m < sk.m_cap) {
      int64_t m_new = std::min(2 * m, sk.m_cap);
      if (sk.s > 1 && m_new < A.n) m_new -= m_new % sk.s;
      if (m_new > m) {
        m = m_new;
        redraw(m);
        delta_new = direction();
        doubled = 1;
        ++r.doublings;
      }
    }
    if (trace) {
      trace->push_back((double)m_step);
      trace->push_back(tau);
      trace->push_back(delta);
      trace->push_back(dn);
      trace->push_back((double)doubled);
    }
    logf("alg4 k=%d m=%lld tau=%g delta=%.6g -> %.6g%s", k, (long long)m_step, tau, delta, dn,
         doubled ? " (m doubled)" : "");
    delta = delta_new;
    ++k;
  }
  if (X_out)
    IHS_HIP(hipMemcpy2DAsync(X_out, sizeof(double) * ldx, X, sizeof(double) * K,
                             sizeof(double) * K, d, hipMemcpyDeviceToDevice, st));
  IHS_HIP(hipStreamSynchronize(st));
  r.m = std::min<int64_t>(m, A.n);
  r.iters = k;
  r.delta = delta;
  r.ms = t0.ms();
  return r;
}

// Upper estimate of the device memory a build allocates (A, B and X are the
// caller's): every buffer of the build at its largest size, as if all were
// live at once, with the sketch at its cap.
static int64_t footprint_impl(const ihsbin_matrix* A0, int64_t K, double lam_min,
                              double lam_max, const ihsbin_opts& o) {
  if (!A0 || A0->n <= 0 || A0->d <= 0 || K < 1 || !(lam_min > 0.0) || !(lam_max >= lam_min))
    fail(IHSBIN_EINVAL, "footprint: bad shape or lambda range");
  if (A0->dtype != IHSBIN_F32 && A0->dtype != IHSBIN_F64) fail(IHSBIN_EINVAL, "bad dtype");
  const bool dual = A0->n < A0->d;
  const bool csr = A0->format == IHSBIN_CSR;
  const int64_t N = dual ? A0->d : A0->n, D = dual ? A0->n : A0->d;
  const int64_t es = A0->dtype == IHSBIN_F32 ? 4 : 8;
  const double beta = lam_max / lam_min;
  const int64_t L = o.L > 0 ? o.L : (beta > 1.0 ? std::max(1, (int)std::floor(2.0 * std::log(beta))) : 1);
  const int64_t kcap = o.k_fixed > 0 ? o.k_fixed : o.k_max;
  const int64_t s = o.sketch == IHSBIN_SJLT ? std::max(1, o.sjlt_s) : 1;
  int64_t m = o.m > 0 ? o.m : 2 * D;
  if (m % s) m += s - m % s;
  int64_t m_cap = o.m_max > 0 ? o.m_max : std::max<int64_t>(m, std::min<int64_t>(N, 32 * D));
  if (o.sketch == IHSBIN_SRHT) m_cap = std::min(m_cap, std::max(m, next_pow2(N)));
  if (o.adaptive_m == 3 && o.sketch == IHSBIN_GAUSSIAN && !csr && o.m_max <= 0)
    m_cap = std::max(m_cap, N);
  const int64_t mmax = o.adaptive_m ? std::max(m, m_cap) : m;
  const int64_t rows = std::min(mmax, N);
  double b = 0;
  if (dual) b += (double)es * N * D;
  b += 8.0 * D * K;  // C
  if (csr) {
    // the column-major copy and the dense head block (<= 256 columns) with
    // the tail entries
    const double nz = (double)std::max<int64_t>(0, A0->nnz);
    b += (8.0 + es + 16.0) * nz + 16.0 * D + double(8 << 20) +  // copy and its sort scratch
         (double)es * N * 256.0 + (4.0 + es) * nz + 8.0 * N;
  }
  // sketch scratch (also the identity draws of S = I for CSR)
  double sk = 5.0 * N + 256;
  if (o.sketch == IHSBIN_GAUSSIAN && o.sketch_prec == IHSBIN_SKETCH_BF16) {
    sk = std::max(sk, (double)sketch_bf16_work_bytes(mmax, N, D));
  } else if (o.sketch == IHSBIN_GAUSSIAN && o.sketch_prec == IHSBIN_SKETCH_FP8) {
    sk = std::max(sk, (double)sketch_fp8_work_bytes(mmax, N, D));
  } else if (o.sketch == IHSBIN_GAUSSIAN) {
    int64_t blk = (int64_t)((size_t(1) << 30) / (8 * (size_t)N));
    blk = std::min(mmax, std::max<int64_t>(64, (blk / 64) * 64));
    sk = std::max(sk, 8.0 * blk * N);
  } else if (o.sketch == IHSBIN_SRHT) {
    sk = std::max(sk, 8.0 * next_pow2(N) * D + N + 256);
  } else {
    // draws, then the bucket sort: dense 12 bytes per draw (+ sort scratch),
    // CSR 24 bytes per entry and block (+ sort scratch)
    const double nnz = csr ? (double)std::max<int64_t>(0, A0->nnz) : 0.0;
    sk = std::max(sk, 5.0 * N * s + (csr ? 28.0 * nnz * s : 12.0 * N * s + 4.0 * mmax) +
                          16.0 * (csr ? nnz * s : (double)N * s) + double(8 << 20));
  }
  b += sk + 4.0 * mmax;
  b += 2 * 8.0 * rows * D;  // SA (grown at most geometrically)
  b += 8.0 * D * D;         // G
  if (o.gram_prec == IHSBIN_GRAM_BF16X3) b += (double)gram_bf16x3_work_bytes(rows, D);
  b += 2 * 8.0 * D * D + 8.0 * cdiv(D, kNB) * kNB * kNB;  // probe or Algorithm 4 factor
  b += 2 * 8.0 * L * D * D + 8.0 * L * cdiv(D, kNB) * kNB * kNB +
       8.0 * factor_inverse_work_doubles(D, (int)L);
  // Lanczos at both ends of every interval
  const int64_t na = 2 * L, ld = padded_width(na);
  const int64_t J = std::min<int64_t>(63, std::max<int64_t>(8, o.lanczos_steps));
  b += 8.0 * D * ld * (J + 4) + 8.0 * trmv_scratch_doubles(D, (int)na) + 16.0 * na * J;
  // basis and the step vectors
  const int64_t wcap = padded_width(L * kcap * K);
  b += 8.0 * L * kcap * D * K + 6 * 8.0 * D * wcap;
  // Y = A U
  int64_t wc = (int64_t)((size_t(6) << 30) / (8 * (size_t)N));
  if (wc >= 64) wc = (wc / 64) * 64;
  wc = std::max<int64_t>(1, std::min(wc, std::max(wcap, ld)));
  b += 8.0 * N * (csr ? wc : padded_width(wc));
  // split-K partials (one buffer, sized by its largest use)
  double part = o.gram_prec == IHSBIN_GRAM_BF16X3
                    ? 8.0 * gram_bf16x3_splits(rows) * D * D
                    : 8.0 * pick_splits_lower(D, rows, 16384) * D * D;
  part = std::max(part, 8.0 * 1024 * 128 * 112);         // W = A^T Y column tiles
  part = std::max(part, 8.0 * 4096 * 8192);              // P_S products
  part = std::max(part, 8.0 * 4096 * 256 * 64);          // Gaussian S A
  part = std::max(part, 8.0 * pick_splits(D, K, N, 1) * D * K);  // A^T B
  b += part;
  if (dual) {
    const int64_t cpad = padded_width(L * kcap * K);
    b += 8.0 * L * kcap * A0->d * K + 8.0 * D * cpad + 8.0 * A0->d * cpad;
  }
  if (o.adaptive_m == 2) b += 5 * 8.0 * D * K;
  if (csr) {
    // column-major copy (sort scratch bounded by 16 bytes per entry + 4 MiB)
    const double nnz = (double)std::max<int64_t>(0, A0->nnz);
    b += 8.0 * (D + 1) + (4.0 + es) * nnz + 4.0 * (nnz / 1024 + D + 1) + 16.0 * nnz +
         4.0 * (D + 1) + 16.0 * nnz + double(4 << 20);
    // chunk partials of the gathered products (in the split-K buffer)
    const int64_t gw = o.sketch == IHSBIN_GAUSSIAN ? std::max<int64_t>(wc, 256) : wc;
    b += 8.0 * (nnz / 1024 + D + 1) * std::max(gw, K);
    // Gaussian sketch: the d x rows gathered block before its transpose
    if (o.sketch == IHSBIN_GAUSSIAN) b += 8.0 * 256 * D;
  }
  b += double(16 << 20);  // small buffers and the pool's 64 KiB rounding
  return (int64_t)b;
}

static int build_impl(Ctx& c, const ihsbin_matrix* Ain, const void* B, int64_t K, int64_t ldb,
                      double lam_min, double lam_max, const ihsbin_opts* o_in,
                      ihsbin_path** out, ihsbin_report* rep) {
  if (!out) fail(IHSBIN_EINVAL, "path out-pointer is NULL");
  *out = nullptr;
  ihsbin_opts o;
  if (o_in) o = *o_in;
  else ihsbin_opts_default(&o);
  const MatView A0 = check_matrix(Ain);
  if (!(lam_min > 0.0) || !(lam_max >= lam_min) || !std::isfinite(lam_max))
    fail(IHSBIN_EINVAL, "need 0 < lam_min <= lam_max");
  if (o.k_max < 1 || o.k_max > 4096) fail(IHSBIN_EINVAL, "k_max out of range");
  if (o.k_fixed < 0 || o.k_fixed > 4096) fail(IHSBIN_EINVAL, "k_fixed out of range");
  if (!(o.tol > 0.0)) fail(IHSBIN_EINVAL, "tol must be positive");
  if (o.adaptive_m < 0 || o.adaptive_m > 3) fail(IHSBIN_EINVAL, "adaptive_m out of range");
  if (!(o.sigma_d2 >= 0.0) || !std::isfinite(o.sigma_d2)) fail(IHSBIN_EINVAL, "need sigma_d2 >= 0");
  if (o.basis_prec < IHSBIN_BASIS_F64 || o.basis_prec > IHSBIN_BASIS_MIXED)
    fail(IHSBIN_EINVAL, "basis_prec out of range");
  if (o.basis_prec == IHSBIN_BASIS_MIXED && !(o.f32_switch > 0.0))
    fail(IHSBIN_EINVAL, "f32_switch must be positive");
  hipStream_t st = c.stream;
  Timer total;
  ihsbin_report r;
  std::memset(&r, 0, sizeof(r));
  c.mem.peak = c.mem.live;
  c.bytes_moved = 0.0;
  // path buffers (handed to the caller) count against the context while the
  // build runs
  struct Held {
    MemStats& s;
    int64_t b = 0;
    void add(int64_t x) {
      s.add(x);
      b += x;
    }
    ~Held() { s.sub(b); }
  } held{c.mem};
  Form form(c.pool);
  make_form(c, A0, B, K, ldb, form);
  const MatView& A = form.A;
  const bool dual = form.dual;
  const double* C = form.C;

  // ---- interval plan (Section 4.2)
  const double beta = lam_max / lam_min;
  int L = o.L > 0 ? o.L : (beta > 1.0 ? std::max(1, (int)std::floor(2.0 * std::log(beta))) : 1);
  std::vector<double> grid(L + 1), lam0(L);
  for (int l = 0; l <= L; ++l) grid[l] = lam_min * std::pow(beta, (double)l / L);
  grid[L] = lam_max;
  // centre of each interval; with sigma_d^2 known, the shifted geometric
  // centre of the remark after Theorem 1: (lam0 + s)^2 = (lo + s)(hi + s)
  // (written without the cancellation of sqrt(...) - s for large s)
  const double sd2 = o.sigma_d2;
  for (int l = 0; l < L; ++l) {
    const double lo = grid[l], hi = grid[l + 1];
    lam0[l] = (lo * hi + sd2 * (lo + hi)) / (std::sqrt((lo + sd2) * (hi + sd2)) + sd2);
  }
  const int64_t d = A.d;

  // ---- sketch, with adaptive m
  Timer tsk;
  Sketcher sketch_m(c, A, o);
  const int64_t m_cap = sketch_m.m_cap;
  int64_t m = sketch_m.initial_m(2 * d);
  if (o.adaptive_m == 3 && !o.taus) m = std::min(m_cap, sketch_m.next_m(m));
  const int& trials = sketch_m.trials;
  PoolBuf Lb(c.pool), Ib(c.pool), dinvb(c.pool), lamb(c.pool);
  double* G = sketch_m.G;
  std::vector<Spec> spec;
  // Predicted contraction rate of interval l from its spectrum estimate.
  auto rate_of = [&](const Spec& sp) { return (sp.mu_max - sp.mu_min) / (sp.mu_max + sp.mu_min); };
  // Next m when the lowest interval is too slow: the Gaussian theorem's edges
  // (1 -+ sqrt(rho))^2 with rho ~ d_e / m give rho from the measured condition
  // number; m is scaled (by a power of two in [2, 16]) to reach rate_target.
  auto grow = [&](const Spec& sp) {
    const double kap = sp.mu_max / sp.mu_min;
    const double kt = (1.0 + o.rate_target) / (1.0 - o.rate_target);
    double factor = 16.0;
    if (kt > 1.0 && kap > 1.0) {
      const double so = (std::sqrt(kap) - 1.0) / (std::sqrt(kap) + 1.0);
      const double sg = (std::sqrt(kt) - 1.0) / (std::sqrt(kt) + 1.0);
      factor = (so * so) / (sg * sg);
    }
    factor = std::min(16.0, std::max(2.0, factor));
    int64_t mult = 1;
    while (mult < factor) mult <<= 1;
    return std::min(m_cap, sketch_m.next_m(m * mult));
  };
  const bool adapt = (o.adaptive_m == 1 || o.adaptive_m == 3) && !o.taus;
  // spectrum estimates on the FP32 matrix cores when the basis products may
  // run there (dense FP32 A)
  const bool spec32 = o.basis_prec != IHSBIN_BASIS_F64 && A.format == IHSBIN_DENSE &&
                      A.dtype == IHSBIN_F32;
  // Sketches whose cost does not grow with m (SRHT: one transform;
  // CountSketch/SJLT: one pass over A) pay for m only through the 2 m d^2
  // Gram, while a larger m shrinks the spectrum of P_S (A^T A + lam I) and
  // with it k.  Measured on the dense 131072 x 2048 SRHT workload with m
  // fixed: path time falls monotonically from m = d/2 (k_max 96, no
  // convergence) to the cap m = 32 d (k_max 14, the fastest), while growing
  // from m0 by probes ends at m = 16 d after three probes (1.6x the time).
  // With m < d such a sketch therefore starts at the cap without a probe;
  // with m >= d the probe below decides.
  const bool cheap_sketch = o.sketch != IHSBIN_GAUSSIAN;
  if (adapt && cheap_sketch && m < d && m < m_cap) {
    logf("m=%lld < d=%lld: starting at the cap m=%lld", (long long)m, (long long)d,
         (long long)m_cap);
    m = m_cap;
  }
  if (o.adaptive_m == 2) {
    // Algorithm 4 at lam_min from m0 = m (default d / 4); it leaves its
    // final sketch in place
    ihsbin_alg4_opts ap;
    ihsbin_alg4_opts_default(&ap);
    if (o.alg4) ap = *o.alg4;
    const int64_t m0 = sketch_m.initial_m(std::max<int64_t>(16, d / 4));
    const ihsbin_alg4_result ar = alg4_impl(c, A, C, K, lam_min, m0, ap, sketch_m, nullptr, 0,
                                            nullptr);
    m = ar.m;
  } else {
    sketch_m(m);
  }
  // Probe: factor and estimate the lowest interval only (the Lanczos run stops
  // early once its Ritz values already show a rate above the target).  When m
  // is too small it grows by the factor the measured spectrum implies (a power
  // of two in [2, 16]) and the sketch is probed again (an SRHT keeps its
  // transform: only the row sample depends on m).
  while (adapt && m < m_cap && trials < 8) {
    double* Lf1 = static_cast<double*>(Lb.ensure(sizeof(double) * d * d));
    double* Li1 = static_cast<double*>(Ib.ensure(sizeof(double) * d * d));
    PsFactors F1;
    F1.n1 = factor_impl(c, G, d, {lam0[0]}, Lf1, Li1, dinvb, lamb, 0, split_factors(d));
    F1.X = Li1;
    F1.Lf = Lf1;
    EarlyIfSlow early;
    early.target = o.rate_target;
    auto sp = interval_spectra(c, AtaProd{c, A, spec32}, F1, {0}, {grid[0]}, {grid[1]},
                               std::max(8, o.lanczos_steps),
                               o.seed, early);
    logf("probe m=%lld: c=[%.4g, %.4g] rate0=%.3f (target %.3f)", (long long)m, sp[0].mu_min,
         sp[0].mu_max, rate_of(sp[0]), o.rate_target);
    if (rate_of(sp[0]) <= o.rate_target) break;
    const int64_t m_new = grow(sp[0]);
    if (m_new <= m) break;
    m = m_new;
    sketch_m(m);
  }
  IHS_HIP(hipStreamSynchronize(st));
  r.ms_sketch = tsk.ms();

  // ---- factor every interval and estimate its spectrum; the batched estimate
  // of the lowest interval re-checks the sketch size
  std::vector<double> tau(L), rate(L), ref(L);
  std::vector<int32_t> all(L);
  for (int l = 0; l < L; ++l) all[l] = l;
  double* Lf = nullptr;
  double* Linv = nullptr;
  PsFactors PF;
  int regrows = 0;
  const int kcap_steps = o.k_fixed > 0 ? o.k_fixed : o.k_max;
  for (;;) {
    Timer tf;
    Lf = static_cast<double*>(Lb.ensure(sizeof(double) * d * d * L));
    Linv = static_cast<double*>(Ib.ensure(sizeof(double) * d * d * L));
    PF.n1 = factor_impl(c, G, d, lam0, Lf, Linv, dinvb, lamb, 0, split_factors(d));
    PF.X = Linv;
    PF.Lf = Lf;
    IHS_HIP(hipStreamSynchronize(st));
    r.ms_factor += tf.ms();
    Timer tspec;
    spec = interval_spectra(c, AtaProd{c, A, spec32}, PF, all,
                            std::vector<double>(grid.begin(), grid.end() - 1),
                            std::vector<double>(grid.begin() + 1, grid.end()),
                            std::max(2, o.lanczos_steps), o.seed + 1, NoEarly{});
    r.ms_spectrum += tspec.ms();
    // the batched estimate of the lowest interval can still be well above the
    // probe's (different start vector): grow once more in that case.  After
    // Algorithm 4 the guard is looser: its m stands unless the lowest
    // interval could not pass the stop test within the step cap at all (its
    // progress measure can shrink quickly while slow directions stall, e.g.
    // when m < d leaves most directions to the 1/lam0 part of P_S).
    const bool recheck =
        adapt ? trials < 8 && rate_of(spec[0]) > o.rate_target + 0.1
              : o.adaptive_m == 2 && regrows < 4 &&
                    rate_of(spec[0]) > std::exp(std::log(o.tol) / std::max(1, kcap_steps));
    if (recheck && m < m_cap) {
      ++regrows;
      const int64_t m_new = grow(spec[0]);
      if (m_new > m) {
        Timer t2;
        m = m_new;
        sketch_m(m);
        IHS_HIP(hipStreamSynchronize(st));
        r.ms_sketch += t2.ms();
        continue;
      }
    }
    break;
  }
  sketch_m.release();
  r.m_used = std::min<int64_t>(m, A.n);
  r.sketch_trials = trials;
  for (int l = 0; l < L && log_enabled(); ++l)
    logf("interval %d [%.4g, %.4g]: c=[%.4g, %.4g]", l, grid[l], grid[l + 1], spec[l].mu_min,
         spec[l].mu_max);
  if (o.taus) {
    for (int l = 0; l < L; ++l) {
      tau[l] = o.taus[l];
      if (!(tau[l] > 0.0)) fail(IHSBIN_EINVAL, "taus must be positive");
    }
  }
  for (int l = 0; l < L; ++l) {
    const double cmin = spec[l].mu_min, cmax = spec[l].mu_max;
    if (!o.taus) tau[l] = 2.0 / (cmin + cmax);
    const double rr = std::max(std::fabs(1.0 - tau[l] * cmin), std::fabs(1.0 - tau[l] * cmax));
    rate[l] = std::min(rr, 0.999);
  }
  for (int l = 0; l < L; ++l) ref[l] = o.centred ? lam0[l] : 0.0;

  // ---- basis recursion
  Timer tb;
  auto path = new ihsbin_path();
  std::unique_ptr<ihsbin_path> guard(path);
  path->device = c.device;
  path->stream = st;
  path->basis.bind(st, nullptr);
  path->items.bind(st, nullptr);
  path->plan.bind(st, nullptr);
  path->d = d;
  path->K = K;
  path->L = L;
  path->m_used = std::min<int64_t>(m, A.n);
  path->lam_min = lam_min;
  path->lam_max = lam_max;
  path->centred = o.centred ? 1 : 0;
  path->grid = grid;
  path->lam0 = lam0;
  path->tau = tau;
  path->rate = rate;
  path->ref = ref;
  path->k.assign(L, 1);
  const int64_t kcap = o.k_fixed > 0 ? o.k_fixed : o.k_max;
  path->kcap = kcap;
  double* basis = static_cast<double*>(path->basis.ensure(sizeof(double) * L * kcap * d * K));
  held.add((int64_t)path->basis.bytes);
  IHS_HIP(hipMemsetAsync(basis, 0, sizeof(double) * L * kcap * d * K, st));

  const int64_t wcap = padded_width((int64_t)L * kcap * K);
  PoolBuf Ub0(c.pool), Ub1(c.pool), Rb(c.pool), Tt(c.pool), Zb(c.pool), Wb(c.pool), pb(c.pool), parb(c.pool), partial_b(c.pool);
  double* Ucur = static_cast<double*>(Ub0.ensure(sizeof(double) * d * wcap));
  double* Unext = static_cast<double*>(Ub1.ensure(sizeof(double) * d * wcap));
  double* R = static_cast<double*>(Rb.ensure(sizeof(double) * d * wcap));
  double* Tm = static_cast<double*>(Tt.ensure(sizeof(double) * d * wcap));
  double* Z = static_cast<double*>(Zb.ensure(sizeof(double) * d * wcap));
  double* W = static_cast<double*>(Wb.ensure(sizeof(double) * d * wcap));
  // per-position parameters: ids, keep (int32), tau, ref, mu_lo, mu_hi (double)
  char* pbase = static_cast<char*>(pb.ensure((sizeof(int32_t) * 2 + sizeof(double) * 4) * L + 256));
  int32_t* ids_dev = reinterpret_cast<int32_t*>(pbase);
  int32_t* keep_dev = ids_dev + L;
  double* tau_dev = reinterpret_cast<double*>(pbase + ((sizeof(int32_t) * 2 * L + 63) / 64) * 64);
  double* ref_dev = tau_dev + L;
  double* mlo_dev = ref_dev + L;
  double* mhi_dev = mlo_dev + L;

  std::vector<int32_t> act = all;
  auto upload = [&]() {
    const int na = (int)act.size();
    std::vector<double> t(na), rf(na), ml(na), mh(na);
    for (int a = 0; a < na; ++a) {
      const int l = act[a];
      t[a] = tau[l];
      rf[a] = ref[l];
      ml[a] = tau[l] * (grid[l] - ref[l]);
      mh[a] = tau[l] * (grid[l + 1] - ref[l]);
    }
    IHS_HIP(hipMemcpyAsync(ids_dev, act.data(), sizeof(int32_t) * na, hipMemcpyHostToDevice, st));
    IHS_HIP(hipMemcpyAsync(tau_dev, t.data(), sizeof(double) * na, hipMemcpyHostToDevice, st));
    IHS_HIP(hipMemcpyAsync(ref_dev, rf.data(), sizeof(double) * na, hipMemcpyHostToDevice, st));
    IHS_HIP(hipMemcpyAsync(mlo_dev, ml.data(), sizeof(double) * na, hipMemcpyHostToDevice, st));
    IHS_HIP(hipMemcpyAsync(mhi_dev, mh.data(), sizeof(double) * na, hipMemcpyHostToDevice, st));
    IHS_HIP(hipStreamSynchronize(st));
  };
  upload();
  // u_{0,0} = P_S C for every interval
  launch_seed_rhs(C, d, K, L, R, wcap, st);
  apply_p(c, PF, ids_dev, L, d, K, wcap, R, Tm, Ucur);
  launch_store_first(Ucur, wcap, d, K, L, ids_dev, kcap, basis, st);

  std::vector<hipEvent_t> events;
  std::vector<double> flops_per_launch;
  std::vector<double> host_part;
  // stop-test bound per interval at its latest step (k = 1: no estimate yet)
  std::vector<double> est(L, 0.0);
  // FP32 products (dense FP32 A): from the start, or once the increments
  // they refine are small (basis_prec)
  const bool f32_ok = A.format == IHSBIN_DENSE && A.dtype == IHSBIN_F32;
  bool use32 = f32_ok && o.basis_prec == IHSBIN_BASIS_F32;
  std::vector<char> launch_f32;
  int unconverged = 0;
  int steps = 0;
  for (int i = 1; i < kcap && !act.empty(); ++i) {
    const int na = (int)act.size();
    const int64_t w_old = (int64_t)na * i * K;
    if (log_enabled()) {
      const ColTiles ct = pick_col_tiles(w_old);
      logf("step %d: active %d, product width %lld (%d column tiles of %d)", i, na,
           (long long)w_old, ct.c, 16 * ct.q);
    }
    const size_t ev0 = events.size();
    ata_apply(c, A, Ucur, w_old, wcap, W, wcap, o.timing ? &events : nullptr, wcap, use32);
    if (o.timing) {
      const double per = A.format == IHSBIN_DENSE ? 4.0 * A.n * A.d : 4.0 * A.nnz;
      const size_t chunks = (events.size() - ev0) / 3;
      const int64_t wc = w_old / (int64_t)std::max<size_t>(1, chunks);
      for (size_t q = 0; q < chunks; ++q) {
        flops_per_launch.push_back(per * (double)wc);
        launch_f32.push_back(use32 ? 1 : 0);
      }
    }
    launch_form_r(W, Ucur, wcap, d, K, na, i, tau_dev, ref_dev, R, st);
    apply_p(c, PF, ids_dev, na, d, (int64_t)(i + 1) * K, wcap, R, Tm, Z);
    double* part = static_cast<double*>(partial_b.ensure(sizeof(double) * 4 * na * 64));
    const int nbx = launch_update(Ucur, Z, Unext, wcap, d, K, na, i, ids_dev, kcap, basis, mlo_dev,
                                  mhi_dev, part, st);
    host_part.resize((size_t)4 * na * nbx);
    IHS_HIP(hipMemcpyAsync(host_part.data(), part, sizeof(double) * host_part.size(),
                           hipMemcpyDeviceToHost, st));
    IHS_HIP(hipStreamSynchronize(st));
    steps = i;
    std::vector<int32_t> keep_pos, next_act;
    double max_inc = 0.0;  // largest relative increment at the active interval ends
    for (int a = 0; a < na; ++a) {
      const int l = act[a];
      path->k[l] = i + 1;
      double sums[4] = {0, 0, 0, 0};
      for (int b = 0; b < nbx; ++b)
        for (int q = 0; q < 4; ++q) sums[q] += host_part[((size_t)a * nbx + b) * 4 + q];
      bool stop;
      const bool finite = std::isfinite(sums[0]) && std::isfinite(sums[1]) && std::isfinite(sums[2]) &&
                          std::isfinite(sums[3]);
      {
        const double fac = rate[l] / (1.0 - rate[l]);
        const double e_lo = std::sqrt(sums[0]) * fac / std::sqrt(sums[2]);
        const double e_hi = std::sqrt(sums[1]) * fac / std::sqrt(sums[3]);
        est[l] = finite ? std::max(e_lo, e_hi) : INFINITY;
        max_inc = std::max(max_inc, finite ? std::max(std::sqrt(sums[0] / sums[2]),
                                                      std::sqrt(sums[1] / sums[3]))
                                           : INFINITY);
      }
      if (o.k_fixed > 0) {
        stop = (i + 1 >= o.k_fixed);
      } else if (!finite) {
        stop = true;
        ++unconverged;
      } else {
        const double rr = rate[l];
        const double fac = rr / (1.0 - rr);
        stop = std::sqrt(sums[0]) * fac <= o.tol * std::sqrt(sums[2]) &&
               std::sqrt(sums[1]) * fac <= o.tol * std::sqrt(sums[3]);
      }
      if (!stop) {
        keep_pos.push_back(a);
        next_act.push_back(l);
      }
    }
    if (f32_ok && o.basis_prec == IHSBIN_BASIS_MIXED && !use32 && max_inc <= o.f32_switch) {
      use32 = true;
      logf("step %d: largest relative increment %.3g <= %.3g: FP32 products from here", i,
           max_inc, o.f32_switch);
    }
    if ((int)next_act.size() < na && !next_act.empty()) {
      IHS_HIP(hipMemcpyAsync(keep_dev, keep_pos.data(), sizeof(int32_t) * keep_pos.size(),
                             hipMemcpyHostToDevice, st));
      launch_compact(Unext, Ucur, wcap, d, (int64_t)(i + 1) * K, (int)next_act.size(), keep_dev, st);
      act = next_act;
      upload();
    } else {
      std::swap(Ucur, Unext);
      act = next_act;
    }
  }
  if (o.k_fixed == 0) unconverged += (int)act.size();
  IHS_HIP(hipStreamSynchronize(st));
  if (dual) {
    // x = A^T z for every stored basis vector (blocks j < k_l of each
    // interval): gathered into one n x (blocks K) matrix, one product with
    // the d0 x n matrix A^T, scattered back as d0 x K blocks
    const int64_t d0 = A.n;
    std::vector<int32_t> blk;
    for (int l = 0; l < L; ++l)
      for (int j = 0; j < path->k[l]; ++j) blk.push_back((int32_t)(l * kcap + j));
    const int nb = (int)blk.size();
    const int64_t cols = (int64_t)nb * K;
    const int64_t cpad = padded_width(cols);
    ihs::DevBuf bx;
    bx.bind(st, nullptr);
    PoolBuf zb(c.pool), xb(c.pool), ib(c.pool);
    double* bxp = static_cast<double*>(bx.ensure(sizeof(double) * L * kcap * d0 * K));
    held.add((int64_t)bx.bytes);
    double* Zt = static_cast<double*>(zb.ensure(sizeof(double) * d * cpad));
    double* Xt = static_cast<double*>(xb.ensure(sizeof(double) * d0 * cpad));
    int32_t* blk_dev = static_cast<int32_t*>(ib.ensure(sizeof(int32_t) * nb));
    IHS_HIP(hipMemcpyAsync(blk_dev, blk.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
    IHS_HIP(hipMemsetAsync(bxp, 0, sizeof(double) * L * kcap * d0 * K, st));
    // Zt has row stride cpad so the product may read whole column tiles
    if (cpad != cols) IHS_HIP(hipMemsetAsync(Zt, 0, sizeof(double) * d * cpad, st));
    launch_gather_blocks(basis, blk_dev, nb, d, K, Zt, cpad, st);
    int64_t done = 0;
    const int64_t chunk = 8192;  // column chunks keep the tiling within its range
    while (done < cols) {
      const int64_t cw = std::min(chunk, cols - done);
      const ColTiles ct = pick_col_tiles(cw);
      Gemm g;
      g.M = d0;
      g.N = cw;
      g.K = d;
      g.A = A.vals;
      g.lda = A.ld;
      g.B = Zt + done;
      g.ldb = cpad;
      g.n_read = std::min<int64_t>(cpad - done, (int64_t)ct.c * 16 * ct.q);
      g.C = Xt + done;
      g.ldc = cpad;
      gemm_cols(g, A.dtype == IHSBIN_F32 ? DT::F32 : DT::F64, false, ct, st);
      done += cw;
    }
    launch_scatter_blocks(Xt, cpad, blk_dev, nb, d0, K, bxp, st);
    IHS_HIP(hipStreamSynchronize(st));
    std::swap(path->basis.p, bx.p);
    std::swap(path->basis.bytes, bx.bytes);
    path->d = d0;
    path->dual = 1;
  }
  r.ms_basis = tb.ms();
  if (o.timing && !events.empty()) {
    for (size_t q = 0, t = 0; q + 2 < events.size(); q += 3, ++t) {
      float ty = 0.f, tw = 0.f;
      IHS_HIP(hipEventElapsedTime(&ty, events[q], events[q + 1]));
      IHS_HIP(hipEventElapsedTime(&tw, events[q + 1], events[q + 2]));
      const double f = t < flops_per_launch.size() ? flops_per_launch[t] : 0.0;
      if (t < launch_f32.size() && launch_f32[t]) {
        r.ata_f32_ms_y += ty;
        r.ata_f32_ms_w += tw;
        r.ata_f32_launches += 1;
        r.ata_f32_flops += f;
      } else {
        r.ata_ms_y += ty;
        r.ata_ms_w += tw;
        r.ata_launches += 1;
        r.ata_flops += f;
      }
    }
    const double abytes = A.format == IHSBIN_DENSE
                              ? (double)A.n * A.d * (A.dtype == IHSBIN_F32 ? 4.0 : 8.0)
                              : (double)A.nnz * ((A.dtype == IHSBIN_F32 ? 4.0 : 8.0) + 4.0);
    r.ata_bytes_a = abytes * (double)r.ata_launches;
  }
  for (auto e : events) (void)hipEventDestroy(e);
  r.L = L;
  r.steps = steps;
  for (int l = 0; l < L; ++l) {
    r.k_max_used = std::max(r.k_max_used, path->k[l]);
    r.k_sum += path->k[l];
  }
  {
    // the plan on the device, read by ihsbin_path_eval_noalloc
    const size_t nd = (size_t)(3 * L + 1);
    char* pl = static_cast<char*>(path->plan.ensure(sizeof(double) * nd + sizeof(int32_t) * L));
    std::vector<double> hp;
    hp.reserve(nd);
    hp.insert(hp.end(), path->grid.begin(), path->grid.end());
    hp.insert(hp.end(), path->tau.begin(), path->tau.end());
    hp.insert(hp.end(), path->ref.begin(), path->ref.end());
    IHS_HIP(hipMemcpyAsync(pl, hp.data(), sizeof(double) * nd, hipMemcpyHostToDevice, st));
    IHS_HIP(hipMemcpyAsync(pl + sizeof(double) * nd, path->k.data(), sizeof(int32_t) * L,
                           hipMemcpyHostToDevice, st));
    IHS_HIP(hipStreamSynchronize(st));
    held.add((int64_t)path->plan.bytes);
  }
  r.n_unconverged = unconverged;
  for (int l = 0; l < L; ++l) r.est_rel_err = std::max(r.est_rel_err, est[l]);
  if (kcap == 1) r.est_rel_err = NAN;  // one term: no increment to bound it with
  r.bytes_moved = c.bytes_moved;
  r.ms_total = total.ms();
  r.peak_bytes = c.mem.peak;
  if (rep) *rep = r;
  *out = guard.release();
  return unconverged > 0 ? IHSBIN_ENOCONV : IHSBIN_OK;
}

// Many problems of one shape in one set of launches: P dense n x d problems
// (A_p = A + p strideA, B_p = B + p strideB) share the interval plan, the
// sketch family and its dimension m, and every step runs as one batched
// launch over all P L intervals (GEMMs with a problem dimension, factors and
// triangular products over P L matrices).  The basis steps run in lockstep:
// every interval takes the same number of steps, the first after which all
// of them pass the stop test (so each gets at least the steps it needs).
// Each problem gets its own path; their bases share one allocation.
static int build_batch_impl(Ctx& c, int P, const ihsbin_matrix* Ain, int64_t strideA,
                            const void* B, int64_t K, int64_t ldb, int64_t strideB,
                            double lam_min, double lam_max, const ihsbin_opts* o_in,
                            ihsbin_path** paths, ihsbin_report* rep) {
  if (!paths) fail(IHSBIN_EINVAL, "paths is NULL");
  if (P < 1 || P > 65535) fail(IHSBIN_EINVAL, "need 1 <= P <= 65535");
  for (int p = 0; p < P; ++p) paths[p] = nullptr;
  ihsbin_opts o;
  if (o_in) o = *o_in;
  else ihsbin_opts_default(&o);
  const MatView A = check_matrix(Ain);
  if (A.format != IHSBIN_DENSE) fail(IHSBIN_EUNSUP, "batched builds take dense matrices");
  if (A.n < A.d) fail(IHSBIN_EUNSUP, "batched builds need n >= d");
  if (strideA < (A.n - 1) * A.ld + A.d) fail(IHSBIN_EINVAL, "strideA smaller than one matrix");
  if (!B || K < 1 || ldb < K || strideB < (A.n - 1) * ldb + K)
    fail(IHSBIN_EINVAL, "need B, K >= 1, ldb >= K and strideB covering one right-hand side block");
  if (!(lam_min > 0.0) || !(lam_max >= lam_min) || !std::isfinite(lam_max))
    fail(IHSBIN_EINVAL, "need 0 < lam_min <= lam_max");
  if (o.k_max < 1 || o.k_max > 4096) fail(IHSBIN_EINVAL, "k_max out of range");
  if (o.k_fixed < 0 || o.k_fixed > 4096) fail(IHSBIN_EINVAL, "k_fixed out of range");
  if (!(o.tol > 0.0)) fail(IHSBIN_EINVAL, "tol must be positive");
  if (o.adaptive_m < 0 || o.adaptive_m > 1)
    fail(IHSBIN_EUNSUP, "batched builds use adaptive_m 0 or 1");
  if (o.taus) fail(IHSBIN_EUNSUP, "batched builds estimate their step sizes");
  if (o.gram_prec != IHSBIN_GRAM_F64) fail(IHSBIN_EUNSUP, "batched builds form the Gram in FP64");
  if (o.graph_steps < 0 || o.graph_steps > 64) fail(IHSBIN_EINVAL, "graph_steps in [0, 64]");
  if (!(o.sigma_d2 >= 0.0) || !std::isfinite(o.sigma_d2)) fail(IHSBIN_EINVAL, "need sigma_d2 >= 0");
  hipStream_t st = c.stream;
  Timer total;
  ihsbin_report r;
  std::memset(&r, 0, sizeof(r));
  c.mem.peak = c.mem.live;
  c.bytes_moved = 0.0;
  const int64_t n = A.n, d = A.d;
  const size_t es = A.dtype == IHSBIN_F32 ? 4 : 8;
  auto problem = [&](int p) {
    MatView v = A;
    v.vals = static_cast<const char*>(A.vals) + (size_t)p * (size_t)strideA * es;
    return v;
  };

  // ---- interval plan (Section 4.2), shared by every problem
  const double beta = lam_max / lam_min;
  const int L = o.L > 0 ? o.L
                        : (beta > 1.0 ? std::max(1, (int)std::floor(2.0 * std::log(beta))) : 1);
  std::vector<double> grid(L + 1), lam0(L);
  for (int l = 0; l <= L; ++l) grid[l] = lam_min * std::pow(beta, (double)l / L);
  grid[L] = lam_max;
  for (int l = 0; l < L; ++l) {
    const double lo = grid[l], hi = grid[l + 1], sd2 = o.sigma_d2;
    lam0[l] = (lo * hi + sd2 * (lo + hi)) / (std::sqrt((lo + sd2) * (hi + sd2)) + sd2);
  }
  const int nl = P * L;  // slots: problem p, interval l -> p L + l

  // ---- C_p = A_p^T B_p
  PoolBuf Cb(c.pool);
  double* C = static_cast<double*>(Cb.ensure(sizeof(double) * (size_t)P * d * K));
  atb_apply_batch(c, A, strideA, P, B, K, ldb, strideB, C);

  // ---- sketch with one m for all problems
  Timer tsk;
  const int s = o.sketch == IHSBIN_SJLT ? std::max(1, o.sjlt_s) : 1;
  auto round_s = [&](int64_t mm) { return mm % s ? mm + (s - mm % s) : mm; };
  int64_t m = round_s(o.m > 0 ? o.m : 2 * d);
  int64_t m_cap = o.m_max > 0 ? o.m_max : std::max<int64_t>(m, std::min<int64_t>(n, 32 * d));
  if (o.sketch == IHSBIN_SRHT) m_cap = std::min(m_cap, std::max(m, next_pow2(n)));
  const bool adapt = o.adaptive_m == 1;
  const bool cheap_sketch = o.sketch != IHSBIN_GAUSSIAN;
  if (adapt && cheap_sketch && m < d && m < m_cap) m = m_cap;
  PoolBuf SAb(c.pool), Gb(c.pool), Sb(c.pool);
  double* G = static_cast<double*>(Gb.ensure(sizeof(double) * (size_t)P * d * d));
  int trials = 0;
  auto sketch_all = [&](int64_t mm) {
    const int64_t rows = std::min(mm, n);
    double* SA = static_cast<double*>(SAb.ensure(sizeof(double) * (size_t)P * rows * d));
    if (mm >= n) {
      for (int p = 0; p < P; ++p) copy_rows_f64(c, problem(p), SA + (size_t)p * rows * d);
    } else if (o.sketch == IHSBIN_GAUSSIAN && o.sketch_prec == IHSBIN_SKETCH_F64) {
      // one S for every problem: S A_p as a batched product per chunk of rows
      c.bytes_moved += (double)P * (matrix_bytes(A) + 8.0 * (double)mm * (double)d);
      int64_t rb = (int64_t)((size_t(1) << 30) / (sizeof(double) * (size_t)n));
      rb = std::max<int64_t>(64, (rb / 64) * 64);
      if (rb > mm) rb = mm;
      double* S = static_cast<double*>(Sb.ensure(sizeof(double) * (size_t)rb * n));
      for (int64_t r0 = 0; r0 < mm; r0 += rb) {
        const int64_t rn = std::min(rb, mm - r0);
        launch_gaussian_fill(o.seed, mm, r0, rn, n, S, st);
        const int splits = pick_splits(rn, d, n, P);
        Gemm g;
        g.M = rn;
        g.N = d;
        g.K = n;
        g.A = S;
        g.lda = n;
        g.strideA = 0;
        g.B = A.vals;
        g.ldb = A.ld;
        g.strideB = strideA;
        g.batch = P;
        const DT tb = A.dtype == IHSBIN_F32 ? DT::F32 : DT::F64;
        if (splits > 1) {
          double* part = static_cast<double*>(c.ws_part.ensure(
              sizeof(double) * (size_t)splits * (size_t)P * (size_t)rn * (size_t)d));
          g.C = part;
          g.ldc = d;
          g.strideC = rn * d;
          g.splits = splits;
          gemm(g, DT::F64, false, tb, false, st);
          reduce_splits(part, splits, P, rn, d, d, rn * d, SA + r0 * d, d, rows * d, 1.0, 0.0, st);
        } else {
          g.C = SA + r0 * d;
          g.ldc = d;
          g.strideC = rows * d;
          gemm(g, DT::F64, false, tb, false, st);
        }
      }
    } else {
      for (int p = 0; p < P; ++p)
        sketch_apply_impl(c, problem(p), o.sketch, s, mm, o.seed, SA + (size_t)p * rows * d, false,
                          o.sketch_prec);
    }
    gram_impl(c, SA, rows, d, G, IHSBIN_GRAM_F64, P);
    ++trials;
  };
  auto rate_of = [&](const Spec& sp) { return (sp.mu_max - sp.mu_min) / (sp.mu_max + sp.mu_min); };
  auto grow = [&](const Spec& sp) {
    const double kap = sp.mu_max / sp.mu_min;
    const double kt = (1.0 + o.rate_target) / (1.0 - o.rate_target);
    double factor = 16.0;
    if (kt > 1.0 && kap > 1.0) {
      const double so = (std::sqrt(kap) - 1.0) / (std::sqrt(kap) + 1.0);
      const double sg = (std::sqrt(kt) - 1.0) / (std::sqrt(kt) + 1.0);
      factor = (so * so) / (sg * sg);
    }
    factor = std::min(16.0, std::max(2.0, factor));
    int64_t mult = 1;
    while (mult < factor) mult <<= 1;
    return round_s(std::min(m_cap, m * mult));
  };
  sketch_all(m);
  PoolBuf Lb(c.pool), Ib(c.pool), dinvb(c.pool), lamb(c.pool);
  const BatchProd prod{c, A, strideA, P, 2};
  std::vector<int32_t> pid(P);
  for (int p = 0; p < P; ++p) pid[p] = p;
  while (adapt && m < m_cap && trials < 8) {
    // the lowest interval of every problem, probed together
    double* Lf1 = static_cast<double*>(Lb.ensure(sizeof(double) * (size_t)P * d * d));
    double* Li1 = static_cast<double*>(Ib.ensure(sizeof(double) * (size_t)P * d * d));
    PsFactors F1;
    F1.n1 = factor_impl(c, G, d, std::vector<double>(P, lam0[0]), Lf1, Li1, dinvb, lamb, 1,
                        split_factors(d, true));
    F1.X = Li1;
    F1.Lf = Lf1;
    EarlyIfAnySlow early;
    early.P = P;
    early.target = o.rate_target;
    auto sp = interval_spectra(c, prod, F1, pid, std::vector<double>(P, grid[0]),
                               std::vector<double>(P, grid[1]), std::max(8, o.lanczos_steps),
                               o.seed, early);
    int worst = 0;
    for (int p = 1; p < P; ++p)
      if (rate_of(sp[p]) > rate_of(sp[worst])) worst = p;
    logf("batch probe m=%lld: worst rate %.3f (problem %d, target %.3f)", (long long)m,
         rate_of(sp[worst]), worst, o.rate_target);
    if (rate_of(sp[worst]) <= o.rate_target) break;
    const int64_t m_new = grow(sp[worst]);
    if (m_new <= m) break;
    m = m_new;
    sketch_all(m);
  }
  IHS_HIP(hipStreamSynchronize(st));
  r.ms_sketch = tsk.ms();

  // ---- factors and spectra of every interval of every problem
  std::vector<double> lam0s(nl), los(nl), his(nl);
  std::vector<int32_t> all(nl);
  for (int p = 0; p < P; ++p)
    for (int l = 0; l < L; ++l) {
      lam0s[p * L + l] = lam0[l];
      los[p * L + l] = grid[l];
      his[p * L + l] = grid[l + 1];
      all[p * L + l] = p * L + l;
    }
  std::vector<Spec> spec;
  double* Lf = nullptr;
  double* Linv = nullptr;
  PsFactors PF;
  for (;;) {
    Timer tf;
    Lf = static_cast<double*>(Lb.ensure(sizeof(double) * (size_t)nl * d * d));
    Linv = static_cast<double*>(Ib.ensure(sizeof(double) * (size_t)nl * d * d));
    PF.n1 = factor_impl(c, G, d, lam0s, Lf, Linv, dinvb, lamb, L, split_factors(d, true));
    PF.X = Linv;
    PF.Lf = Lf;
    IHS_HIP(hipStreamSynchronize(st));
    r.ms_factor += tf.ms();
    Timer tspec;
    spec = interval_spectra(c, prod, PF, all, los, his, std::max(2, o.lanczos_steps), o.seed + 1,
                            NoEarly{});
    r.ms_spectrum += tspec.ms();
    int worst = 0;
    for (int p = 1; p < P; ++p)
      if (rate_of(spec[p * L]) > rate_of(spec[worst * L])) worst = p;
    if (adapt && trials < 8 && m < m_cap && rate_of(spec[worst * L]) > o.rate_target + 0.1) {
      const int64_t m_new = grow(spec[worst * L]);
      if (m_new > m) {
        Timer t2;
        m = m_new;
        sketch_all(m);
        IHS_HIP(hipStreamSynchronize(st));
        r.ms_sketch += t2.ms();
        continue;
      }
    }
    break;
  }
  SAb.release();
  Gb.release();
  r.m_used = std::min<int64_t>(m, n);
  r.sketch_trials = trials;
  std::vector<double> tau(nl), rate(nl), ref(nl);
  for (int a = 0; a < nl; ++a) {
    tau[a] = 2.0 / (spec[a].mu_min + spec[a].mu_max);
    const double rr = std::max(std::fabs(1.0 - tau[a] * spec[a].mu_min),
                               std::fabs(1.0 - tau[a] * spec[a].mu_max));
    rate[a] = std::min(rr, 0.999);
    ref[a] = o.centred ? lam0s[a] : 0.0;
  }

  // ---- basis recursion, all P L intervals in lockstep
  Timer tb;
  const int64_t kcap = o.k_fixed > 0 ? o.k_fixed : o.k_max;
  auto basis_buf = std::make_shared<DevBuf>();
  double* basis =
      static_cast<double*>(basis_buf->ensure(sizeof(double) * (size_t)nl * kcap * d * K));
  c.mem.add((int64_t)basis_buf->bytes);
  struct Unheld {
    MemStats& s;
    int64_t b;
    ~Unheld() { s.sub(b); }
  } unheld{c.mem, (int64_t)basis_buf->bytes};
  IHS_HIP(hipMemsetAsync(basis, 0, sizeof(double) * (size_t)nl * kcap * d * K, st));
  const int64_t wcap = padded_width((int64_t)nl * kcap * K + 128);
  PoolBuf Ub0(c.pool), Ub1(c.pool), Rb(c.pool), Tt(c.pool), Zb(c.pool), Wb(c.pool), pb(c.pool),
      partial_b(c.pool);
  double* Ucur = static_cast<double*>(Ub0.ensure(sizeof(double) * d * wcap));
  double* Unext = static_cast<double*>(Ub1.ensure(sizeof(double) * d * wcap));
  double* R = static_cast<double*>(Rb.ensure(sizeof(double) * d * wcap));
  double* Tm = static_cast<double*>(Tt.ensure(sizeof(double) * d * wcap));
  double* Z = static_cast<double*>(Zb.ensure(sizeof(double) * d * wcap));
  double* W = static_cast<double*>(Wb.ensure(sizeof(double) * d * wcap));
  // the product's tiles may read columns past the last block: keep them finite
  IHS_HIP(hipMemsetAsync(Ucur, 0, sizeof(double) * d * wcap, st));
  IHS_HIP(hipMemsetAsync(Unext, 0, sizeof(double) * d * wcap, st));
  char* pbase = static_cast<char*>(pb.ensure((sizeof(int32_t) + sizeof(double) * 4) * nl + 256));
  int32_t* ids_dev = reinterpret_cast<int32_t*>(pbase);
  double* tau_dev = reinterpret_cast<double*>(pbase + ((sizeof(int32_t) * nl + 63) / 64) * 64);
  double* ref_dev = tau_dev + nl;
  double* mlo_dev = ref_dev + nl;
  double* mhi_dev = mlo_dev + nl;
  {
    std::vector<double> ml(nl), mh(nl);
    for (int a = 0; a < nl; ++a) {
      ml[a] = tau[a] * (los[a] - ref[a]);
      mh[a] = tau[a] * (his[a] - ref[a]);
    }
    IHS_HIP(hipMemcpyAsync(ids_dev, all.data(), sizeof(int32_t) * nl, hipMemcpyHostToDevice, st));
    IHS_HIP(hipMemcpyAsync(tau_dev, tau.data(), sizeof(double) * nl, hipMemcpyHostToDevice, st));
    IHS_HIP(hipMemcpyAsync(ref_dev, ref.data(), sizeof(double) * nl, hipMemcpyHostToDevice, st));
    IHS_HIP(hipMemcpyAsync(mlo_dev, ml.data(), sizeof(double) * nl, hipMemcpyHostToDevice, st));
    IHS_HIP(hipMemcpyAsync(mhi_dev, mh.data(), sizeof(double) * nl, hipMemcpyHostToDevice, st));
  }
  launch_seed_rhs(C, d, K, nl, R, wcap, st, L);
  apply_p(c, PF, ids_dev, nl, d, K, wcap, R, Tm, Ucur);
  launch_store_first(Ucur, wcap, d, K, nl, ids_dev, kcap, basis, st);
  const BatchProd prod1{c, A, strideA, P, 1};
  std::vector<double> host_part, est(nl, 0.0);
  std::vector<char> passed(nl, 0);
  int steps = 0;
  bool all_passed = false;
  double* part = static_cast<double*>(partial_b.ensure(sizeof(double) * 4 * nl * 64));
  // one basis step of every interval on stream s (the context's own stream
  // or the capture stream); returns the blocks of partial norms it wrote
  auto step = [&](int i, hipStream_t s) {
    const int64_t w_old = (int64_t)nl * i * K;
    prod1(Ucur, w_old, wcap, W);
    launch_form_r(W, Ucur, wcap, d, K, nl, i, tau_dev, ref_dev, R, s);
    apply_p(c, PF, ids_dev, nl, d, (int64_t)(i + 1) * K, wcap, R, Tm, Z);
    const int nbx = launch_update(Ucur, Z, Unext, wcap, d, K, nl, i, ids_dev, kcap, basis, mlo_dev,
                                  mhi_dev, part, s);
    std::swap(Ucur, Unext);
    return nbx;
  };
  const int gsteps = o.graph_steps;
  int graphs = 0;
  for (int i = 1; i < kcap;) {
    int chunk = 1, nbx = 0;
    if (gsteps > 0) {
      // steps i .. i + chunk - 1 captured into one HIP graph and launched as
      // one unit (the stop test reads the last step's norms): nothing may
      // allocate while capturing, so the workspaces are grown first
      chunk = std::min<int>(gsteps, (int)(kcap - i));
      for (int j = 0; j < chunk; ++j) {
        ata_batch_reserve(c, A, P, (int64_t)L * (i + j) * K);
        apply_p_reserve(c, nl, d, (int64_t)(i + j + 1) * K);
      }
      if (!c.capture_stream)
        IHS_HIP(hipStreamCreateWithFlags(&c.capture_stream, hipStreamNonBlocking));
      hipEvent_t ready;
      IHS_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
      IHS_HIP(hipEventRecord(ready, st));
      IHS_HIP(hipStreamWaitEvent(c.capture_stream, ready, 0));
      (void)hipEventDestroy(ready);
      hipGraph_t graph = nullptr;
      c.stream = c.capture_stream;
      IHS_HIP(hipStreamBeginCapture(c.capture_stream, hipStreamCaptureModeThreadLocal));
      try {
        for (int j = 0; j < chunk; ++j) nbx = step(i + j, c.capture_stream);
      } catch (...) {
        (void)hipStreamEndCapture(c.capture_stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        c.stream = st;
        throw;
      }
      const hipError_t ec = hipStreamEndCapture(c.capture_stream, &graph);
      c.stream = st;
      IHS_HIP(ec);
      hipGraphExec_t exec = nullptr;
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      IHS_HIP(ei);
      const hipError_t el = hipGraphLaunch(exec, st);
      if (el == hipSuccess) IHS_HIP(hipStreamSynchronize(st));
      (void)hipGraphExecDestroy(exec);
      IHS_HIP(el);
      ++graphs;
    } else {
      nbx = step(i, st);
    }
    host_part.resize((size_t)4 * nl * nbx);
    IHS_HIP(hipMemcpyAsync(host_part.data(), part, sizeof(double) * host_part.size(),
                           hipMemcpyDeviceToHost, st));
    IHS_HIP(hipStreamSynchronize(st));
    i += chunk;
    steps = i - 1;
    all_passed = true;
    for (int a = 0; a < nl; ++a) {
      double sums[4] = {0, 0, 0, 0};
      for (int b = 0; b < nbx; ++b)
        for (int q = 0; q < 4; ++q) sums[q] += host_part[((size_t)a * nbx + b) * 4 + q];
      const bool finite = std::isfinite(sums[0]) && std::isfinite(sums[1]) &&
                          std::isfinite(sums[2]) && std::isfinite(sums[3]);
      const double fac = rate[a] / (1.0 - rate[a]);
      const double e_lo = std::sqrt(sums[0]) * fac / std::sqrt(sums[2]);
      const double e_hi = std::sqrt(sums[1]) * fac / std::sqrt(sums[3]);
      est[a] = finite ? std::max(e_lo, e_hi) : INFINITY;
      passed[a] = finite && e_lo <= o.tol && e_hi <= o.tol;
      if (!passed[a]) all_passed = false;
    }
    if (o.k_fixed > 0 ? steps + 1 >= o.k_fixed : all_passed) break;
  }
  if (graphs) logf("batch basis: %d steps in %d HIP graphs", steps, graphs);
  const int k_all = steps + 1;
  int unconverged = 0;
  if (o.k_fixed == 0)
    for (int a = 0; a < nl; ++a) unconverged += passed[a] ? 0 : 1;
  r.ms_basis = tb.ms();

  // ---- one path per problem, sharing the basis and plan allocations
  const size_t plan_doubles = (size_t)(3 * L + 1);
  const size_t plan_bytes = ((sizeof(double) * plan_doubles + sizeof(int32_t) * L + 255) / 256) * 256;
  auto plan_buf = std::make_shared<DevBuf>();
  char* plan = static_cast<char*>(plan_buf->ensure(plan_bytes * (size_t)P));
  {
    std::vector<char> hp(plan_bytes * (size_t)P, 0);
    for (int p = 0; p < P; ++p) {
      double* dp = reinterpret_cast<double*>(hp.data() + plan_bytes * p);
      for (int l = 0; l <= L; ++l) dp[l] = grid[l];
      for (int l = 0; l < L; ++l) {
        dp[L + 1 + l] = tau[p * L + l];
        dp[2 * L + 1 + l] = ref[p * L + l];
      }
      int32_t* kp = reinterpret_cast<int32_t*>(dp + plan_doubles);
      for (int l = 0; l < L; ++l) kp[l] = k_all;
    }
    IHS_HIP(hipMemcpyAsync(plan, hp.data(), hp.size(), hipMemcpyHostToDevice, st));
    IHS_HIP(hipStreamSynchronize(st));
  }
  std::vector<std::unique_ptr<ihsbin_path>> made;
  for (int p = 0; p < P; ++p) {
    auto path = std::make_unique<ihsbin_path>();
    path->device = c.device;
    path->stream = st;
    path->items.bind(st, nullptr);
    path->d = d;
    path->K = K;
    path->L = L;
    path->m_used = r.m_used;
    path->lam_min = lam_min;
    path->lam_max = lam_max;
    path->centred = o.centred ? 1 : 0;
    path->grid = grid;
    path->lam0 = lam0;
    path->tau.assign(tau.begin() + (size_t)p * L, tau.begin() + (size_t)(p + 1) * L);
    path->rate.assign(rate.begin() + (size_t)p * L, rate.begin() + (size_t)(p + 1) * L);
    path->ref.assign(ref.begin() + (size_t)p * L, ref.begin() + (size_t)(p + 1) * L);
    path->k.assign(L, k_all);
    path->kcap = kcap;
    path->shared_basis = basis_buf;
    path->basis_off = sizeof(double) * (size_t)p * L * kcap * d * K;
    path->shared_plan = plan_buf;
    path->plan_off = plan_bytes * (size_t)p;
    made.push_back(std::move(path));
  }
  r.L = L;
  r.steps = steps;
  r.k_max_used = k_all;
  r.k_sum = k_all * nl;
  r.n_unconverged = unconverged;
  for (int a = 0; a < nl; ++a) r.est_rel_err = std::max(r.est_rel_err, est[a]);
  if (kcap == 1) r.est_rel_err = NAN;
  r.bytes_moved = c.bytes_moved;
  r.ms_total = total.ms();
  r.peak_bytes = c.mem.peak;
  if (rep) *rep = r;
  for (int p = 0; p < P; ++p) paths[p] = made[p].release();
  return unconverged > 0 ? IHSBIN_ENOCONV : IHSBIN_OK;
}

static int interval_of(const std::vector<double>& grid, double lam) {
  const int L = (int)grid.size() - 1;
  int l = (int)(std::lower_bound(grid.begin() + 1, grid.end(), lam) - (grid.begin() + 1));
  return std::min(std::max(l, 0), L - 1);
}

static void eval_impl(ihsbin_path* p, const double* lambdas, int64_t T, void* X, int64_t ldx,
                      int x_dtype) {
  if (!p) fail(IHSBIN_EINVAL, "path is NULL");
  if (T < 0 || (T > 0 && (!lambdas || !X))) fail(IHSBIN_EINVAL, "bad lambdas / X");
  if (ldx < p->K) fail(IHSBIN_EINVAL, "ldx < K");
  if (x_dtype != IHSBIN_F32 && x_dtype != IHSBIN_F64) fail(IHSBIN_EINVAL, "bad x_dtype");
  if (T == 0) return;
  DeviceGuard dg(p->device);
  std::vector<EvalItem> items((size_t)T);
  const double slack = 1e-12;
  for (int64_t t = 0; t < T; ++t) {
    const double lam = lambdas[t];
    if (!(lam >= p->lam_min * (1 - slack)) || !(lam <= p->lam_max * (1 + slack)))
      fail(IHSBIN_ERANGE, "lambda outside the prepared range");
    const int l = interval_of(p->grid, lam);
    items[t].l = l;
    items[t].k = p->k[l];
    items[t].tau = p->tau[l];
    items[t].mu = p->tau[l] * (lam - p->ref[l]);
  }
  EvalItem* it = static_cast<EvalItem*>(p->items.ensure(sizeof(EvalItem) * (size_t)T));
  IHS_HIP(hipMemcpyAsync(it, items.data(), sizeof(EvalItem) * (size_t)T, hipMemcpyHostToDevice,
                         p->stream));
  launch_eval(p->basis_ptr(), p->kcap, p->d, p->K, it, T, X, ldx, x_dtype, p->stream);
  IHS_HIP(hipStreamSynchronize(p->stream));
}

}  // namespace ihs

// ====================================================================== ABI
using namespace ihs;

template <class F>
static int guarded(ihsbin_ctx* ctx, F&& f) {
  try {
    int rc = f();
    if (ctx && rc == IHSBIN_ENOCONV) ctx->c.last_error = "some interval reached k_max";
    return rc;
  } catch (const Error& e) {
    if (ctx) ctx->c.last_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->c.last_error = "host allocation failed";
    return IHSBIN_ENOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->c.last_error = e.what();
    return IHSBIN_EHIP;
  }
}

extern "C" {

const char* ihsbin_status_str(int s) {
  switch (s) {
    case IHSBIN_OK: return "ok";
    case IHSBIN_EINVAL: return "invalid argument";
    case IHSBIN_ENOMEM: return "out of device memory";
    case IHSBIN_EHIP: return "HIP runtime error";
    case IHSBIN_ENOTSPD: return "sketched Hessian not positive definite";
    case IHSBIN_ENOCONV: return "tolerance not reached within k_max";
    case IHSBIN_ERANGE: return "lambda outside the prepared range";
    case IHSBIN_EUNSUP: return "unsupported";
    case IHSBIN_EAGAIN: return "not finished yet";
    default: return "unknown status";
  }
}

const char* ihsbin_version(void) { return "ihsbin 0.1 (gfx950)"; }

void ihsbin_opts_default(ihsbin_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->sketch = IHSBIN_GAUSSIAN;
  o->sjlt_s = 1;
  o->m = 0;
  o->seed = 0;
  o->tol = 1e-8;
  o->k_max = 96;
  o->k_fixed = 0;
  o->L = 0;
  o->centred = 1;
  o->adaptive_m = 1;
  o->rate_target = 0.6;
  o->m_max = 0;
  o->lanczos_steps = 12;
  o->gram_prec = IHSBIN_GRAM_F64;
  o->timing = 0;
  o->taus = nullptr;
  o->alg4 = nullptr;
  o->sketch_prec = IHSBIN_SKETCH_F64;
  o->sigma_d2 = 0.0;
  o->basis_prec = IHSBIN_BASIS_F64;
  o->f32_switch = 1e-2;
  o->graph_steps = 0;
}

void ihsbin_alg4_opts_default(ihsbin_alg4_opts* a) {
  if (!a) return;
  std::memset(a, 0, sizeof(*a));
  a->gamma1 = 0.5;
  a->gamma2 = 1e-4;
  a->gamma3 = 0.5;
  a->eps = 1e-8;
  a->max_iter = 50;
  a->max_armijo = 60;
}

int ihsbin_create(ihsbin_ctx** ctx, int device, void* stream) {
  if (!ctx) return IHSBIN_EINVAL;
  *ctx = nullptr;
  try {
    int n = 0;
    IHS_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return IHSBIN_EINVAL;
    {
      // the allocation-free entry point's scratch address on this device
      DeviceGuard g(device);
      noalloc_scratch(device);
    }
    auto c = new ihsbin_ctx();
    c->c.device = device;
    c->c.stream = static_cast<hipStream_t>(stream);
    c->c.bind();
    *ctx = c;
    return IHSBIN_OK;
  } catch (const Error& e) {
    return e.status;
  } catch (...) {
    return IHSBIN_EHIP;
  }
}

int ihsbin_destroy(ihsbin_ctx* ctx) {
  if (!ctx) return IHSBIN_OK;
  try {
    DeviceGuard g(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    if (ctx->c.capture_stream) {
      (void)hipStreamSynchronize(ctx->c.capture_stream);
      (void)hipStreamDestroy(ctx->c.capture_stream);
    }
    delete ctx;
  } catch (...) {
    delete ctx;
    return IHSBIN_EHIP;
  }
  return IHSBIN_OK;
}

const char* ihsbin_last_error(const ihsbin_ctx* ctx) { return ctx ? ctx->c.last_error.c_str() : ""; }

int ihsbin_path_build(ihsbin_ctx* ctx, const ihsbin_matrix* A, const void* B, int64_t K,
                      int64_t ldb, double lam_min, double lam_max, const ihsbin_opts* opts,
                      ihsbin_path** path, ihsbin_report* report) {
  if (!ctx) return IHSBIN_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    return build_impl(ctx->c, A, B, K, ldb, lam_min, lam_max, opts, path, report);
  });
}

int ihsbin_path_build_batch(ihsbin_ctx* ctx, int32_t P, const ihsbin_matrix* A, int64_t strideA,
                            const void* B, int64_t K, int64_t ldb, int64_t strideB,
                            double lam_min, double lam_max, const ihsbin_opts* opts,
                            ihsbin_path** paths, ihsbin_report* report) {
  if (!ctx) return IHSBIN_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    return build_batch_impl(ctx->c, P, A, strideA, B, K, ldb, strideB, lam_min, lam_max, opts,
                            paths, report);
  });
}

int ihsbin_path_eval(ihsbin_path* path, const double* lambdas, int64_t T, void* X, int64_t ldx,
                     int32_t x_dtype) {
  return guarded(nullptr, [&] {
    eval_impl(path, lambdas, T, X, ldx, x_dtype);
    return IHSBIN_OK;
  });
}

int ihsbin_path_get_info(const ihsbin_path* p, ihsbin_path_info* info) {
  if (!p || !info) return IHSBIN_EINVAL;
  info->L = p->L;
  info->K = (int32_t)p->K;
  info->d = p->d;
  info->m_used = p->m_used;
  info->lam_min = p->lam_min;
  info->lam_max = p->lam_max;
  info->centred = p->centred;
  info->dual = p->dual;
  return IHSBIN_OK;
}

int ihsbin_path_intervals(const ihsbin_path* p, double* lo, double* hi, double* lam0, double* tau,
                          double* rate, int32_t* k) {
  if (!p) return IHSBIN_EINVAL;
  for (int l = 0; l < p->L; ++l) {
    if (lo) lo[l] = p->grid[l];
    if (hi) hi[l] = p->grid[l + 1];
    if (lam0) lam0[l] = p->lam0[l];
    if (tau) tau[l] = p->tau[l];
    if (rate) rate[l] = p->rate[l];
    if (k) k[l] = p->k[l];
  }
  return IHSBIN_OK;
}

int ihsbin_path_basis(const ihsbin_path* p, int32_t l, double* out) {
  if (!p || !out || l < 0 || l >= p->L) return IHSBIN_EINVAL;
  return guarded(nullptr, [&] {
    DeviceGuard g(p->device);
    const size_t blk = sizeof(double) * (size_t)p->d * p->K;
    IHS_HIP(hipMemcpyAsync(out, p->basis_ptr() + (size_t)l * p->kcap * p->d * p->K,
                           blk * p->k[l], hipMemcpyDeviceToDevice, p->stream));
    IHS_HIP(hipStreamSynchronize(p->stream));
    return IHSBIN_OK;
  });
}

int ihsbin_path_free(ihsbin_path* p) {
  if (!p) return IHSBIN_OK;
  try {
    DeviceGuard g(p->device);
    (void)hipStreamSynchronize(p->stream);
  } catch (...) {
  }
  delete p;
  return IHSBIN_OK;
}

int ihsbin_solve_path(ihsbin_ctx* ctx, const ihsbin_matrix* A, const void* B, int64_t K,
                      int64_t ldb, const double* lambdas, int64_t T, const ihsbin_opts* opts,
                      void* X, int64_t ldx, int32_t x_dtype, ihsbin_report* report) {
  if (!ctx) return IHSBIN_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    if (T < 1 || !lambdas) fail(IHSBIN_EINVAL, "need T >= 1 lambdas");
    double lo = lambdas[0], hi = lambdas[0];
    for (int64_t t = 1; t < T; ++t) {
      lo = std::min(lo, lambdas[t]);
      hi = std::max(hi, lambdas[t]);
    }
    ihsbin_path* p = nullptr;
    const int rc = build_impl(ctx->c, A, B, K, ldb, lo, hi, opts, &p, report);
    std::unique_ptr<ihsbin_path> guard(p);
    eval_impl(p, lambdas, T, X, ldx, x_dtype);
    return rc;
  });
}

int ihsbin_sketch_draws(ihsbin_ctx* ctx, int32_t sketch, uint64_t seed, int64_t n, int64_t m,
                        int32_t sjlt_s, int32_t* idx, int8_t* sign) {
  if (!ctx) return IHSBIN_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    if (n <= 0 || m <= 0 || n > INT32_MAX || m > INT32_MAX || !idx || !sign)
      fail(IHSBIN_EINVAL, "bad sizes or pointers");
    if (sketch == IHSBIN_COUNTSKETCH || sketch == IHSBIN_SJLT) {
      const int s = sketch == IHSBIN_SJLT ? sjlt_s : 1;
      if (s < 1 || m % s) fail(IHSBIN_EINVAL, "SJLT needs s >= 1 dividing m");
      launch_draw_countsketch(seed, n, m, s, idx, sign, ctx->c.stream);
    } else if (sketch == IHSBIN_SRHT) {
      launch_draw_srht(seed, n, next_pow2(n), m, sign, idx, ctx->c.stream);
    } else {
      fail(IHSBIN_EINVAL, "no integer draws for this sketch");
    }
    IHS_HIP(hipStreamSynchronize(ctx->c.stream));
    return IHSBIN_OK;
  });
}

int ihsbin_sketch_indices_host(uint64_t seed, int32_t sketch, int64_t n, int64_t m,
                               int32_t sjlt_s, int32_t* idx, int8_t* sign) {
  if (n <= 0 || m <= 0 || n > INT32_MAX || m > INT32_MAX || !idx || !sign) return IHSBIN_EINVAL;
  using namespace ihs;
  if (sketch == IHSBIN_COUNTSKETCH || sketch == IHSBIN_SJLT) {
    const int64_t s = sketch == IHSBIN_SJLT ? sjlt_s : 1;
    if (s < 1 || m % s) return IHSBIN_EINVAL;
    const uint64_t key = stream_key(seed, 0);
    const uint32_t mb = (uint32_t)(m / s);
    for (int64_t t = 0; t < n * s; ++t) {
      const uint64_t x = sm_draw(key, (uint64_t)t);
      idx[t] = (int32_t)((uint32_t)(t % s) * mb + sm_range(x, mb));
      sign[t] = (x & 1ull) ? (int8_t)-1 : (int8_t)1;
    }
    return IHSBIN_OK;
  }
  if (sketch == IHSBIN_SRHT) {
    const int64_t npad = next_pow2(n);
    if (npad > INT32_MAX) return IHSBIN_EUNSUP;
    const uint64_t k1 = stream_key(seed, 1), k2 = stream_key(seed, 2);
    for (int64_t i = 0; i < n; ++i) sign[i] = (sm_draw(k1, (uint64_t)i) & 1ull) ? (int8_t)-1 : (int8_t)1;
    for (int64_t r = 0; r < m; ++r) idx[r] = (int32_t)sm_range(sm_draw(k2, (uint64_t)r), (uint32_t)npad);
    return IHSBIN_OK;
  }
  return IHSBIN_EINVAL;
}

int ihsbin_sketch_indices_device(ihsbin_ctx* ctx, uint64_t seed, int32_t sketch, int64_t n,
                                 int64_t m, int32_t sjlt_s, int32_t* idx, int8_t* sign) {
  return ihsbin_sketch_draws(ctx, sketch, seed, n, m, sjlt_s, idx, sign);
}

int ihsbin_csr_transpose(ihsbin_ctx* ctx, const ihsbin_matrix* A, int32_t* col_ptr, int32_t* row,
                         void* vals) {
  if (!ctx) return IHSBIN_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    const MatView v = check_matrix(A);
    if (v.format != IHSBIN_CSR) fail(IHSBIN_EINVAL, "the column-major copy needs a CSR matrix");
    if (!col_ptr || (v.nnz > 0 && (!row || !vals))) fail(IHSBIN_EINVAL, "NULL output");
    validate_csr(ctx->c, v);
    PoolBuf cscb(ctx->c.pool);
    Csc csc;
    build_csc(v, cscb.ensure((size_t)csc_work_bytes(v)), csc, ctx->c.stream);
    hipStream_t st = ctx->c.stream;
    const size_t es = v.dtype == IHSBIN_F32 ? 4 : 8;
    IHS_HIP(hipMemcpyAsync(col_ptr, csc.col_ptr, sizeof(int32_t) * (size_t)(v.d + 1),
                           hipMemcpyDeviceToDevice, st));
    if (v.nnz > 0) {
      IHS_HIP(hipMemcpyAsync(row, csc.row, sizeof(int32_t) * (size_t)v.nnz, hipMemcpyDeviceToDevice, st));
      IHS_HIP(hipMemcpyAsync(vals, csc.val, es * (size_t)v.nnz, hipMemcpyDeviceToDevice, st));
    }
    IHS_HIP(hipStreamSynchronize(st));
    return IHSBIN_OK;
  });
}

int ihsbin_sketch_apply_prec(ihsbin_ctx* ctx, const ihsbin_matrix* A, int32_t sketch,
                             int32_t sjlt_s, int64_t m, uint64_t seed, int32_t prec, double* SA) {
  if (!ctx) return IHSBIN_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    const MatView v = check_matrix(A);
    if (!SA) fail(IHSBIN_EINVAL, "SA is NULL");
    if (v.format == IHSBIN_CSR) validate_csr(ctx->c, v);
    sketch_apply_impl(ctx->c, v, sketch, sjlt_s, m, seed, SA, false, prec);
    IHS_HIP(hipStreamSynchronize(ctx->c.stream));
    return IHSBIN_OK;
  });
}

int ihsbin_sketch_apply(ihsbin_ctx* ctx, const ihsbin_matrix* A, int32_t sketch, int32_t sjlt_s,
                        int64_t m, uint64_t seed, double* SA) {
  return ihsbin_sketch_apply_prec(ctx, A, sketch, sjlt_s, m, seed, IHSBIN_SKETCH_F64, SA);
}

int ihsbin_precond_factor(ihsbin_ctx* ctx, const double* SA, int64_t m, int64_t d,
                          const double* lam0, int32_t nl, double* Lfac, double* Linv) {
  if (!ctx) return IHSBIN_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    if (!SA || !lam0 || !Lfac || m <= 0 || d <= 0 || nl <= 0) fail(IHSBIN_EINVAL, "bad arguments");
    for (int i = 0; i < nl; ++i)
      if (!(lam0[i] > 0.0)) fail(IHSBIN_EINVAL, "lam0 must be positive");
    PoolBuf Gb(ctx->c.pool), dinvb(ctx->c.pool), lamb(ctx->c.pool);
    double* G = static_cast<double*>(Gb.ensure(sizeof(double) * d * d));
    gram_impl(ctx->c, SA, m, d, G);
    std::vector<double> l0(lam0, lam0 + nl);
    factor_impl(ctx->c, G, d, l0, Lfac, Linv, dinvb, lamb);
    IHS_HIP(hipStreamSynchronize(ctx->c.stream));
    return IHSBIN_OK;
  });
}

int ihsbin_build_footprint(const ihsbin_matrix* A, int64_t K, double lam_min, double lam_max,
                           const ihsbin_opts* opts, int64_t* bytes) {
  if (!bytes) return IHSBIN_EINVAL;
  return guarded(nullptr, [&] {
    ihsbin_opts o;
    if (opts) o = *opts;
    else ihsbin_opts_default(&o);
    *bytes = footprint_impl(A, K, lam_min, lam_max, o);
    return IHSBIN_OK;
  });
}

int ihsbin_path_set_stream(ihsbin_path* p, void* stream) {
  if (!p) return IHSBIN_EINVAL;
  try {
    DeviceGuard g(p->device);
    IHS_HIP(hipStreamSynchronize(p->stream));  // the basis is complete
    p->stream = static_cast<hipStream_t>(stream);
    p->basis.stream = p->stream;
    p->plan.stream = p->stream;
    p->items.stream = p->stream;
  } catch (const Error& e) {
    return e.status;
  }
  return IHSBIN_OK;
}

int ihsbin_sketch_size(ihsbin_ctx* ctx, const ihsbin_matrix* A, const void* B, int64_t K,
                       int64_t ldb, double lam, const ihsbin_opts* opts,
                       const ihsbin_alg4_opts* alg4, ihsbin_alg4_result* res, double* X,
                       int64_t ldx, double* trace, int32_t trace_rows) {
  if (!ctx) return IHSBIN_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    if (!res) fail(IHSBIN_EINVAL, "res is NULL");
    if (trace_rows < 0 || (trace_rows > 0 && !trace)) fail(IHSBIN_EINVAL, "bad trace buffer");
    ihsbin_opts o;
    if (opts) o = *opts;
    else ihsbin_opts_default(&o);
    ihsbin_alg4_opts ap;
    if (alg4) ap = *alg4;
    else ihsbin_alg4_opts_default(&ap);
    const MatView A0 = check_matrix(A);
    Form form(ctx->c.pool);
    make_form(ctx->c, A0, B, K, ldb, form);
    if (X && ldx < K) fail(IHSBIN_EINVAL, "ldx < K");
    Sketcher sk(ctx->c, form.A, o);
    const int64_t m0 = sk.initial_m(std::max<int64_t>(16, form.A.d / 4));
    std::vector<double> tr;
    *res = alg4_impl(ctx->c, form.A, form.C, K, lam, m0, ap, sk, X, ldx,
                     trace_rows > 0 ? &tr : nullptr);
    const size_t rows = std::min<size_t>(tr.size() / 5, (size_t)trace_rows);
    if (rows) std::memcpy(trace, tr.data(), sizeof(double) * 5 * rows);
    return IHSBIN_OK;
  });
}

int ihsbin_gram(ihsbin_ctx* ctx, const double* SA, int64_t m, int64_t d, int32_t prec,
                double* G) {
  if (!ctx) return IHSBIN_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    if (!SA || !G || m <= 0 || d <= 0) fail(IHSBIN_EINVAL, "bad arguments");
    gram_impl(ctx->c, SA, m, d, G, prec);
    IHS_HIP(hipStreamSynchronize(ctx->c.stream));
    return IHSBIN_OK;
  });
}

int ihsbin_sketch_gram(ihsbin_ctx* ctx, const ihsbin_matrix* A, int32_t sketch, int32_t sjlt_s,
                       int64_t m, uint64_t seed, int32_t sketch_prec, int32_t gram_prec,
                       double* G) {
  if (!ctx) return IHSBIN_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    const MatView v = check_matrix(A);
    if (!G || m <= 0) fail(IHSBIN_EINVAL, "bad arguments");
    if (v.format == IHSBIN_CSR) validate_csr(ctx->c, v);
    ihsbin_opts o;
    ihsbin_opts_default(&o);
    o.sketch = sketch;
    o.sjlt_s = sjlt_s;
    o.m = m;
    o.seed = seed;
    o.sketch_prec = sketch_prec;
    o.gram_prec = gram_prec;
    if (sketch == IHSBIN_SJLT && (sjlt_s < 1 || m % sjlt_s)) fail(IHSBIN_EINVAL, "SJLT needs s | m");
    Sketcher sk(ctx->c, v, o);
    sk(m);
    IHS_HIP(hipMemcpyAsync(G, sk.G, sizeof(double) * (size_t)v.d * (size_t)v.d,
                           hipMemcpyDeviceToDevice, ctx->c.stream));
    IHS_HIP(hipStreamSynchronize(ctx->c.stream));
    return IHSBIN_OK;
  });
}

int ihsbin_ata_apply_tiled(ihsbin_ctx* ctx, const ihsbin_matrix* A, const double* U, int64_t w,
                           int64_t ldu, double* W, int64_t ldw, int32_t prec, int32_t q,
                           int32_t splits) {
  if (!ctx) return IHSBIN_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    const MatView v = check_matrix(A);
    if (v.format != IHSBIN_DENSE) fail(IHSBIN_EUNSUP, "tiled products are dense only");
    if (!U || !W || w < 1 || ldu < w || ldw < w) fail(IHSBIN_EINVAL, "bad U / W");
    if (prec != IHSBIN_BASIS_F64 && prec != IHSBIN_BASIS_F32) fail(IHSBIN_EINVAL, "bad prec");
    if (q < 0 || q > kColTileMaxQ || splits < 0 || splits > 256)
      fail(IHSBIN_EINVAL, "q in [0, 7], splits in [0, 256]");
    if (prec == IHSBIN_BASIS_F32 && v.dtype != IHSBIN_F32)
      fail(IHSBIN_EUNSUP, "FP32 products need an FP32 matrix");
    TileForce f;
    f.q = q;
    f.splits = splits;
    ata_apply(ctx->c, v, U, w, ldu, W, ldw, nullptr, ldu, prec == IHSBIN_BASIS_F32, &f);
    IHS_HIP(hipStreamSynchronize(ctx->c.stream));
    return IHSBIN_OK;
  });
}

int ihsbin_ata_apply(ihsbin_ctx* ctx, const ihsbin_matrix* A, const double* U, int64_t w,
                     int64_t ldu, double* W, int64_t ldw) {
  if (!ctx) return IHSBIN_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    MatView v = check_matrix(A);
    if (!U || !W || w < 1 || ldu < w || ldw < w) fail(IHSBIN_EINVAL, "bad U / W");
    PoolBuf cscb(ctx->c.pool), htb(ctx->c.pool);
    Csc csc;
    HeadTail ht;
    if (v.format == IHSBIN_CSR) {
      validate_csr(ctx->c, v);
      build_csc(v, cscb.ensure((size_t)csc_work_bytes(v)), csc, ctx->c.stream);
      v.csc = &csc;
      build_head_tail(v, csc, htb, ht, ctx->c.stream);
      if (ht.h > 0) v.ht = &ht;
    }
    ata_apply(ctx->c, v, U, w, ldu, W, ldw, nullptr, ldu);
    IHS_HIP(hipStreamSynchronize(ctx->c.stream));
    return IHSBIN_OK;
  });
}

}  // extern "C"
