// Batched factorization of the sketched Hessians (SA)^T SA + lam0_l I, one
// per lambda sub-interval (the matrix whose inverse is P_S, Section 4).
//
// Right-looking blocked Cholesky with 64 x 64 panels: the diagonal block is
// factored (and inverted) inside LDS by one workgroup per matrix, the panel
// below it is multiplied by the inverted block, and the trailing lower
// triangle is updated with the MFMA GEMM.  All nl matrices advance together,
// one launch per stage.  When the inverse factor L^-1 is wanted too (so that
// applying P_S = L^-T L^-1 to many vectors is two triangular matrix
// products), both are built together by halves (factor_inverse_batched).
#include <algorithm>
#include <cmath>
#include <utility>

#include "ops.hpp"

namespace ihs {

// H_l = G_{l / gper} + lam0_l I (lower triangle) for l < nl.
__global__ void build_shifted_kernel(const double* __restrict__ G, int64_t d,
                                     const double* __restrict__ lam0, int nl, int gper,
                                     double* H) {
  const int64_t per = d * d;
  const int64_t total = per * nl;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(t / per);
    const int64_t e = t % per;
    const int64_t r = e / d, c = e % d;
    const double* Gl = G + (int64_t)(l / gper) * per;
    H[t] = c > r ? 0.0 : Gl[e] + (r == c ? lam0[l] : 0.0);  // lower triangle only
  }
}

void launch_build_shifted(const double* G, int64_t d, const double* lam0_dev, int nl, double* H,
                          hipStream_t st, int gper) {
  int64_t blocks = cdiv(d * d * nl, 256);
  if (blocks > 16384) blocks = 16384;
  if (gper < 1) gper = nl;
  hipLaunchKernelGGL(build_shifted_kernel, dim3((unsigned)blocks), dim3(256), 0, st, G, d, lam0_dev,
                     nl, gper, H);
  IHS_CHECK_LAUNCH();
}

// Factor diagonal block p of every matrix, write L_pp back (upper part zeroed)
// and its inverse into dinv[l][p].  Thread (r, q) keeps row r, columns
// q, q + 4, ..., q + 60 of the block in registers; each column step publishes
// one column (factorization) or one row (inversion) through LDS and costs one
// barrier and at most four register updates (its 16-column panel); each
// panel's rank-16 update of the rest follows in one pass.  The steps are
// expanded at compile time so the register slots are addressed statically.
namespace {
constexpr int kS = kNB / 4;

// The 64 columns are taken in four panels of 16.  Inside a panel a column
// step updates only the panel's own columns; the columns right of the panel
// receive the panel's rank-16 update once, after its last step.

// factorization step j: owners publish column j; every row scales its entry
// into L[r][j] and updates its panel columns c in (j, r]
template <int J>
__device__ __forceinline__ void potrf_step(double (&a)[kS], double (*colbuf)[kNB], int r, int q,
                                           bool& bad) {
  constexpr int SEND = 4 * (J / 16) + 4;  // slots of the panel holding column J
  double* col = colbuf[J & 1];
  if (q == (J & 3)) col[r] = a[J >> 2];
  __syncthreads();
  double djj = col[J];
  if (!(djj > 0.0)) {
    bad = true;
    djj = 1.0;
  }
  // one division per step: entries of column J are scaled by 1 / sqrt(d_JJ)
  const double rpiv = 1.0 / sqrt(djj);
  const double lrj = r >= J ? col[r] * rpiv : 0.0;
  if (q == (J & 3)) a[J >> 2] = lrj;
#pragma unroll
  for (int s = J >> 2; s < SEND; ++s) {
    const int c = q + 4 * s;
    const double upd = lrj * (col[c] * rpiv);  // select, not branch: lanes differ in c
    a[s] -= (c > J && c <= r) ? upd : 0.0;
  }
}

// after panel P: a[r][c] -= sum_k L[r][16P+k] L[c][16P+k] for columns c right
// of the panel (the panel is published to lp first)
template <int P>
__device__ __forceinline__ void potrf_panel_update(double (&a)[kS], double (*lp)[17], int r,
                                                   int q) {
#pragma unroll
  for (int s = 4 * P; s < 4 * P + 4; ++s) lp[r][q + 4 * s - 16 * P] = a[s];
  __syncthreads();
  double lr[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) lr[k] = lp[r][k];
#pragma unroll
  for (int s = 4 * P + 4; s < kS; ++s) {
    const int c = q + 4 * s;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += lr[k] * lp[c][k];
    a[s] -= c <= r ? acc : 0.0;
  }
}

// inversion step i: row i of X = L^-1 becomes final and is published; rows
// below it inside the panel accumulate L[r][i] X[i]
template <int I>
__device__ __forceinline__ void trinv_step(double (&x)[kS], double (*rowbuf)[kNB],
                                           const double (*lf)[kNB + 1], int r, int q) {
  constexpr int PEND = 16 * (I / 16) + 16;  // first row after the panel
  double* row = rowbuf[I & 1];
  if (r == I) {
    const double rlii = 1.0 / lf[I][I];
#pragma unroll
    for (int s = 0; s <= (I >> 2); ++s) {
      const int c = q + 4 * s;
      x[s] = c <= I ? ((c == I ? 1.0 : 0.0) - x[s]) * rlii : 0.0;
      row[c] = x[s];
    }
  }
  __syncthreads();
  if (r > I && r < PEND) {
    const double lri = lf[r][I];
#pragma unroll
    for (int s = 0; s <= (I >> 2); ++s) {
      const int c = q + 4 * s;
      const double upd = lri * row[c];
      x[s] += c <= I ? upd : 0.0;
    }
  }
}

// after row panel P of X is final: rows below it accumulate
// sum_k L[r][16P+k] X[16P+k][c] for c <= 16P+15 (X rows published to xp)
template <int P>
__device__ __forceinline__ void trinv_panel_update(double (&x)[kS], double (*xp)[kNB + 1],
                                                   const double (*lf)[kNB + 1], int r, int q) {
  if (r >= 16 * P && r < 16 * P + 16) {
#pragma unroll
    for (int s = 0; s < 4 * P + 4; ++s) xp[r - 16 * P][q + 4 * s] = x[s];
  }
  __syncthreads();
  if (r >= 16 * P + 16) {
    double lr[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) lr[k] = lf[r][16 * P + k];
#pragma unroll
    for (int s = 0; s < 4 * P + 4; ++s) {
      const int c = q + 4 * s;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) acc += lr[k] * xp[k][c];
      x[s] += acc;
    }
  }
  __syncthreads();  // xp is rewritten by the next panel
}

template <int P, int... J>
__device__ __forceinline__ void potrf_panel(std::integer_sequence<int, J...>, double (&a)[kS],
                                            double (*colbuf)[kNB], double (*lp)[17], int r, int q,
                                            bool& bad) {
  (potrf_step<16 * P + J>(a, colbuf, r, q, bad), ...);
  if constexpr (P < 3) potrf_panel_update<P>(a, lp, r, q);
}

template <int P, int... I>
__device__ __forceinline__ void trinv_panel(std::integer_sequence<int, I...>, double (&x)[kS],
                                            double (*rowbuf)[kNB], double (*xp)[kNB + 1],
                                            const double (*lf)[kNB + 1], int r, int q) {
  (trinv_step<16 * P + I>(x, rowbuf, lf, r, q), ...);
  if constexpr (P < 3) trinv_panel_update<P>(x, xp, lf, r, q);
}
}  // namespace

__global__ __launch_bounds__(256) void potrf_diag_kernel(double* H, int64_t d, int p,
                                                         double* dinv, int nblk, int* status,
                                                         double* X) {
  constexpr int NB = kNB;
  static_assert(NB == 64, "register layout assumes 64 x 64 blocks and 256 threads");
  __shared__ double colbuf[2][NB];
  __shared__ double lf[NB][NB + 1];
  __shared__ double pbuf[NB * (NB + 1)];  // panel exchange (lp: 64 x 17, xp: 16 x 65)
  auto lp = reinterpret_cast<double (*)[17]>(pbuf);
  auto xp = reinterpret_cast<double (*)[NB + 1]>(pbuf);
  const int l = blockIdx.x;
  double* M = H + (int64_t)l * d * d;
  const int64_t o = (int64_t)p * NB;
  const int nb = (int)((d - o) < NB ? (d - o) : NB);
  const int tid = threadIdx.x;
  const int r = tid >> 2, q = tid & 3;
  double a[kS];
#pragma unroll
  for (int s = 0; s < kS; ++s) {
    const int c = q + 4 * s;
    a[s] = (c <= r) ? ((r < nb && c < nb) ? M[(o + r) * d + o + c] : (r == c ? 1.0 : 0.0)) : 0.0;
  }
  bool bad = false;
  const auto seq16 = std::make_integer_sequence<int, 16>{};
  potrf_panel<0>(seq16, a, colbuf, lp, r, q, bad);
  potrf_panel<1>(seq16, a, colbuf, lp, r, q, bad);
  potrf_panel<2>(seq16, a, colbuf, lp, r, q, bad);
  potrf_panel<3>(seq16, a, colbuf, lp, r, q, bad);
  if (bad) status[0] = 1;
#pragma unroll
  for (int s = 0; s < kS; ++s) {
    const int c = q + 4 * s;
    lf[r][c] = a[s];
    if (r < nb && c < nb) M[(o + r) * d + o + c] = a[s];
  }
  double x[kS];
#pragma unroll
  for (int s = 0; s < kS; ++s) x[s] = 0.0;
  __syncthreads();
  trinv_panel<0>(seq16, x, colbuf, xp, lf, r, q);
  trinv_panel<1>(seq16, x, colbuf, xp, lf, r, q);
  trinv_panel<2>(seq16, x, colbuf, xp, lf, r, q);
  trinv_panel<3>(seq16, x, colbuf, xp, lf, r, q);
  double* Di = dinv + ((int64_t)l * nblk + p) * NB * NB;
#pragma unroll
  for (int s = 0; s < kS; ++s) {
    const int c = q + 4 * s;
    Di[r * NB + c] = c <= r ? x[s] : 0.0;
  }
  if (X) {  // the inverse block in place on the diagonal of X (upper part zero)
    double* Xl = X + (int64_t)l * d * d;
#pragma unroll
    for (int s = 0; s < kS; ++s) {
      const int c = q + 4 * s;
      if (r < nb && c < nb) Xl[(o + r) * d + o + c] = c <= r ? x[s] : 0.0;
    }
  }
}

// The trailing updates compute whole GEMM tiles that touch the lower
// triangle, so entries right of the diagonal, within the widest tile's
// BM + BN (at most 288) columns, receive partial sums: the strict upper
// triangle is cleared within that band at the end.
constexpr int kUpperBand = 384;

__global__ void zero_upper_band_kernel(double* H, int64_t d, int nl) {
  const int64_t per = d * kUpperBand;
  const int64_t total = per * nl;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = t / per, e = t - l * per;
    const int64_t r = e / kUpperBand, c = r + 1 + (e - r * kUpperBand);
    if (c < d) H[l * d * d + r * d + c] = 0.0;
  }
}

// Two-level right-looking order: 64-column steps inside 256-column outer
// panels update only their own panel; the trailing matrix right of an outer
// panel is updated once per panel with K = 256, so it is read and written a
// quarter as often as with 64-column steps.
void cholesky_batched(double* H, int64_t d, int nl, double* dinv, int* status_dev,
                      hipStream_t st) {
  const int NB = kNB;
  const int64_t OB = 4 * (int64_t)kNB;
  const int nblk = (int)cdiv(d, NB);
  auto syrk_lower = [&](int64_t r0, int64_t c0, int64_t rows, int64_t cols, int64_t k0,
                        int64_t kk) {
    // H[r0:r0+rows, c0:c0+cols] -= H[r0:, k0:k0+kk] H[c0:, k0:k0+kk]^T  (tiles touching the lower part)
    Gemm tg;
    tg.M = rows;
    tg.N = cols;
    tg.K = kk;
    tg.A = H + r0 * d + k0;
    tg.lda = d;
    tg.strideA = d * d;
    tg.B = H + c0 * d + k0;
    tg.ldb = d;
    tg.strideB = d * d;
    tg.C = H + r0 * d + c0;
    tg.ldc = d;
    tg.strideC = d * d;
    tg.alpha = -1.0;
    tg.beta = 1.0;
    tg.batch = nl;
    tg.lower_only = 1;
    gemm(tg, DT::F64, false, DT::F64, true, st);
  };
  for (int64_t O = 0; O < d; O += OB) {
    const int64_t oe = (O + OB) < d ? (O + OB) : d;
    for (int64_t o = O; o < oe; o += NB) {
      const int p = (int)(o / NB);
      hipLaunchKernelGGL(potrf_diag_kernel, dim3(nl), dim3(256), 0, st, H, d, p, dinv, nblk,
                         status_dev, (double*)nullptr);
      IHS_CHECK_LAUNCH();
      const int64_t below = d - o - NB;
      if (below <= 0) break;
      // panel: H[o+NB:, o:o+NB] <- H[o+NB:, o:o+NB] * inv(L_pp)^T  (in place, one column tile)
      Gemm pg;
      pg.M = below;
      pg.N = NB;
      pg.K = NB;
      pg.A = H + (o + NB) * d + o;
      pg.lda = d;
      pg.strideA = d * d;
      pg.B = dinv + (int64_t)p * NB * NB;
      pg.ldb = NB;
      pg.strideB = (int64_t)nblk * NB * NB;
      pg.C = H + (o + NB) * d + o;
      pg.ldc = d;
      pg.strideC = d * d;
      pg.batch = nl;
      gemm(pg, DT::F64, false, DT::F64, true, st);
      // the rest of the outer panel
      const int64_t nc = oe - (o + NB);
      if (nc > 0) syrk_lower(o + NB, o + NB, below, nc, o, NB);
    }
    const int64_t rest = d - oe;
    if (rest > 0) syrk_lower(oe, oe, rest, rest, O, oe - O);
  }
  if (d > NB) {
    int64_t blocks = cdiv(d * kUpperBand * nl, 256);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(zero_upper_band_kernel, dim3((unsigned)blocks), dim3(256), 0, st, H, d, nl);
    IHS_CHECK_LAUNCH();
  }
}

// ------------------------------------------------ recursive factor + inverse
// Both factors of every H_l at once, by halves: for H = [H11 .; H21 H22],
//   L11, X11 = L11^-1           (the first half, recursively)
//   L21 = H21 X11^T             (X11 triangular: its zero K-slices skipped)
//   H22 <- H22 - L21 L21^T      (the Schur complement, lower tiles)
//   L22, X22 = L22^-1           (recursively)
//   X21 = -X22 (L21 X11)
// down to 64 x 64 diagonal blocks, which one workgroup per matrix factors
// and inverts in LDS.  The same flops as a right-looking factorization
// followed by a triangular inverse, but the large levels are single GEMMs
// with K = n / 2 (a right-looking order updates the trailing matrix with
// K = 256 slices, each output tile loaded and stored per slice).
namespace {
__global__ void copy_blocks_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                   int64_t d, int64_t rows, int64_t cols, int nl) {
  const int64_t per = rows * cols;
  const int64_t total = per * nl;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = t / per, e = t - l * per;
    const int64_t r = e / cols, c = e - r * cols;
    dst[l * d * d + r * d + c] = src[l * d * d + r * d + c];
  }
}

__global__ void zero_matrices_kernel(double* __restrict__ X, int64_t count) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x)
    X[t] = 0.0;
}

struct RecFactor {
  double* H;
  double* X;
  int64_t d;
  int nl;
  double* dinv;
  int nblk;
  int* status;
  double* work;  // n2 x n1 per matrix at the top split
  hipStream_t st;

  Gemm base(int64_t M, int64_t N, int64_t K) const {
    Gemm g;
    g.M = M;
    g.N = N;
    g.K = K;
    g.lda = d;
    g.ldb = d;
    g.ldc = d;
    g.strideA = d * d;
    g.strideB = d * d;
    g.strideC = d * d;
    g.batch = nl;
    return g;
  }

  int64_t work_doubles;  // capacity of work
  bool top_inverse = true;  // form X21 at the top split as well

  void run(int64_t o, int64_t n) {
    if (n <= kNB) {
      hipLaunchKernelGGL(potrf_diag_kernel, dim3(nl), dim3(256), 0, st, H, d, (int)(o / kNB), dinv,
                         nblk, status, X);
      IHS_CHECK_LAUNCH();
      return;
    }
    const int64_t n1 = cdiv(cdiv(n, 2), kNB) * kNB, n2 = n - n1;
    if (n2 * n1 * nl > work_doubles) fail(IHSBIN_EINVAL, "factor: work buffer too small");
    run(o, n1);
    double* H21 = H + (o + n1) * d + o;
    double* X21 = X + (o + n1) * d + o;
    const double* X11 = X + o * d + o;
    // L21 = H21 X11^T, first into X21's place (H21 is its input)
    Gemm g1 = base(n2, n1, n1);
    g1.A = H21;
    g1.B = X11;  // op(B) = X11^T: upper triangular
    g1.C = X21;
    g1.tri = 4;
    gemm(g1, DT::F64, false, DT::F64, true, st);
    int64_t blocks = cdiv(n2 * n1 * nl, 256);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(copy_blocks_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X21, H21, d,
                       n2, n1, nl);
    IHS_CHECK_LAUNCH();
    // H22 -= L21 L21^T (tiles touching the lower triangle)
    Gemm g2 = base(n2, n2, n1);
    g2.A = H21;
    g2.B = H21;
    g2.C = H + (o + n1) * d + o + n1;
    g2.alpha = -1.0;
    g2.beta = 1.0;
    g2.lower_only = 1;
    gemm(g2, DT::F64, false, DT::F64, true, st);
    run(o + n1, n2);
    // without the top split's X21, L^-1 is applied through its blocks
    // (X11, L21, X22): 3/4 of the inverse's flops are in this split
    if (o == 0 && n == d && !top_inverse) return;
    // T = L21 X11 (X11 lower triangular), then X21 = -X22 T (X22 lower)
    Gemm g3 = base(n2, n1, n1);
    g3.A = H21;
    g3.B = X11;
    g3.C = work;
    g3.ldc = n1;
    g3.strideC = n2 * n1;
    g3.tri = 3;
    gemm(g3, DT::F64, false, DT::F64, false, st);
    Gemm g4 = base(n2, n1, n2);
    g4.A = X + (o + n1) * d + o + n1;
    g4.B = work;
    g4.ldb = n1;
    g4.strideB = n2 * n1;
    g4.C = X21;
    g4.alpha = -1.0;
    g4.tri = 1;
    gemm(g4, DT::F64, false, DT::F64, false, st);
  }
};
}  // namespace

// largest n2 x n1 over every split of the recursion (a ragged top split can
// be smaller than the splits below it)
static int64_t largest_split(int64_t n) {
  if (n <= kNB) return 0;
  const int64_t n1 = cdiv(cdiv(n, 2), kNB) * kNB, n2 = n - n1;
  return std::max(n2 * n1, std::max(largest_split(n1), largest_split(n2)));
}

int64_t factor_inverse_work_doubles(int64_t d, int nl) {
  return std::max<int64_t>(1, largest_split(d) * nl);
}

int64_t factor_top_split(int64_t d) { return d <= kNB ? 0 : cdiv(cdiv(d, 2), kNB) * kNB; }

void factor_inverse_batched(double* H, double* X, int64_t d, int nl, double* dinv,
                            int* status_dev, double* work, hipStream_t st, bool full) {
  {
    int64_t blocks = cdiv(d * d * nl, 256);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(zero_matrices_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X,
                       d * d * nl);
    IHS_CHECK_LAUNCH();
  }
  RecFactor rf{H, X, d, nl, dinv, (int)cdiv(d, kNB), status_dev, work, st,
               factor_inverse_work_doubles(d, nl), full};
  rf.run(0, d);
  if (d > kNB) {
    int64_t blocks = cdiv(d * kUpperBand * nl, 256);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(zero_upper_band_kernel, dim3((unsigned)blocks), dim3(256), 0, st, H, d, nl);
    IHS_CHECK_LAUNCH();
  }
}

}  // namespace ihs
