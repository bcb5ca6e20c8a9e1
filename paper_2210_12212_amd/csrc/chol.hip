// Batched factorization of the sketched Hessians (SA)^T SA + lam0_l I, one
// per lambda sub-interval (the matrix whose inverse is P_S, Section 4).
//
// Right-looking blocked Cholesky with 64 x 64 panels: the diagonal block is
// factored (and inverted) inside LDS by one workgroup per matrix, the panel
// below it is multiplied by the inverted block, and the trailing lower
// triangle is updated with the MFMA GEMM.  All nl matrices advance together,
// one launch per stage.  The inverse factor L^-1 is then built row block by
// row block with the same GEMM, so that applying P_S = L^-T L^-1 to many
// vectors is two triangular matrix products.
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
                                                         double* dinv, int nblk, int* status) {
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
                         status_dev);
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
}

// X <- block diagonal of the 64 x 64 inverses dinv, zero elsewhere.
__global__ void init_inverse_kernel(double* X, int64_t d, int nl, const double* __restrict__ dinv,
                                    int nblk) {
  const int64_t per = d * d;
  const int64_t total = per * nl;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(t / per);
    const int64_t e = t % per;
    const int64_t r = e / d, c = e % d;
    const int64_t p = r / kNB;
    double v = 0.0;
    if (c / kNB == p && c <= r)
      v = dinv[((int64_t)l * nblk + p) * kNB * kNB + (r - p * kNB) * kNB + (c - p * kNB)];
    X[t] = v;
  }
}

// Doubling levels b = 64, 128, ...: diagonal blocks of size b already hold
// their inverses; neighbouring pairs (P, Q) are joined by
//   X_QP = -X_QQ (L_QP X_PP),
// two batched products per level (over pairs and matrices).
static int64_t level_pairs(int64_t d, int64_t b, int64_t& part_rows) {
  const int64_t full = d / (2 * b);
  const int64_t rem = d - full * 2 * b;
  part_rows = rem > b ? rem - b : 0;  // a last pair with a short second block
  return full;
}

int64_t tri_inverse_work_doubles(int64_t d, int nl) {
  int64_t mx = 0;
  for (int64_t b = kNB; b < d; b *= 2) {
    int64_t pr = 0;
    const int64_t full = level_pairs(d, b, pr);
    const int64_t need = full * b * b + pr * b;
    mx = need > mx ? need : mx;
  }
  return mx * nl;
}

void tri_inverse_batched(const double* Lf, int64_t d, int nl, const double* dinv, double* Linv,
                         double* work, hipStream_t st) {
  const int nblk = (int)cdiv(d, kNB);
  {
    int64_t blocks = cdiv(d * d * nl, 256);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(init_inverse_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Linv, d, nl,
                       dinv, nblk);
    IHS_CHECK_LAUNCH();
  }
  for (int64_t b = kNB; b < d; b *= 2) {
    int64_t pr = 0;
    const int64_t full = level_pairs(d, b, pr);
    // pairs start at diagonal offset o = 2 t b; P = [o, o + b), Q = [o + b, o + b + bq)
    auto join = [&](int64_t o, int64_t bq, int npairs, double* T, int64_t strideT) {
      // T = L_QP X_PP   (X_PP lower triangular)
      Gemm g1;
      g1.M = bq;
      g1.N = b;
      g1.K = b;
      g1.A = Lf + (o + b) * d + o;
      g1.lda = d;
      g1.strideA = d * d;
      g1.strideA2 = 2 * b * (d + 1);
      g1.B = Linv + o * d + o;
      g1.ldb = d;
      g1.strideB = d * d;
      g1.strideB2 = 2 * b * (d + 1);
      g1.C = T;
      g1.ldc = b;
      g1.strideC = strideT * npairs;
      g1.strideC2 = strideT;
      g1.batch = nl;
      g1.batch2 = npairs;
      g1.tri = 3;
      gemm(g1, DT::F64, false, DT::F64, false, st);
      // X_QP = -X_QQ T   (X_QQ lower triangular)
      Gemm g2;
      g2.M = bq;
      g2.N = b;
      g2.K = bq;
      g2.A = Linv + (o + b) * d + o + b;
      g2.lda = d;
      g2.strideA = d * d;
      g2.strideA2 = 2 * b * (d + 1);
      g2.B = T;
      g2.ldb = b;
      g2.strideB = strideT * npairs;
      g2.strideB2 = strideT;
      g2.C = Linv + (o + b) * d + o;
      g2.ldc = d;
      g2.strideC = d * d;
      g2.strideC2 = 2 * b * (d + 1);
      g2.alpha = -1.0;
      g2.batch = nl;
      g2.batch2 = npairs;
      g2.tri = 1;
      gemm(g2, DT::F64, false, DT::F64, false, st);
    };
    if (full > 0) join(0, b, (int)full, work, b * b);
    if (pr > 0) join(full * 2 * b, pr, 1, work, pr * b);
  }
}

}  // namespace ihs
