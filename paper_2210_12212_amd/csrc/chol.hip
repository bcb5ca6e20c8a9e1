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

__global__ void build_shifted_kernel(const double* __restrict__ G, int64_t d,
                                     const double* __restrict__ lam0, int nl, double* H) {
  const int64_t per = d * d;
  const int64_t total = per * nl;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(t / per);
    const int64_t e = t % per;
    const int64_t r = e / d, c = e % d;
    H[t] = c > r ? 0.0 : G[e] + (r == c ? lam0[l] : 0.0);  // lower triangle only
  }
}

void launch_build_shifted(const double* G, int64_t d, const double* lam0_dev, int nl, double* H,
                          hipStream_t st) {
  int64_t blocks = cdiv(d * d * nl, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(build_shifted_kernel, dim3((unsigned)blocks), dim3(256), 0, st, G, d, lam0_dev,
                     nl, H);
  IHS_CHECK_LAUNCH();
}

// Factor diagonal block p of every matrix, write L_pp back (upper part zeroed)
// and its inverse into dinv[l][p].  Thread (r, q) keeps row r, columns
// q, q + 4, ..., q + 60 of the block in registers; each column step publishes
// one column (factorization) or one row (inversion) through LDS, so a step
// costs one barrier and up to sixteen independent LDS reads.  The steps are
// expanded at compile time so the register slots are addressed statically.
namespace {
constexpr int kS = kNB / 4;

// factorization step j: owners publish column j; every row scales its entry
// into L[r][j] and updates its columns c in (j, r]
template <int J>
__device__ __forceinline__ void potrf_step(double (&a)[kS], double (*colbuf)[kNB], int r, int q,
                                           bool& bad) {
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
  for (int s = J >> 2; s < kS; ++s) {
    const int c = q + 4 * s;
    const double upd = lrj * (col[c] * rpiv);  // select, not branch: lanes differ in c
    a[s] -= (c > J && c <= r) ? upd : 0.0;
  }
}

// inversion step i: row i of X = L^-1 becomes final and is published; rows
// below accumulate L[r][i] X[i]
template <int I>
__device__ __forceinline__ void trinv_step(double (&x)[kS], double (*rowbuf)[kNB],
                                           const double (*lf)[kNB + 1], int r, int q) {
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
  if (r > I) {
    const double lri = lf[r][I];
#pragma unroll
    for (int s = 0; s <= (I >> 2); ++s) {
      const int c = q + 4 * s;
      const double upd = lri * row[c];
      x[s] += c <= I ? upd : 0.0;
    }
  }
}

template <int... J>
__device__ __forceinline__ void potrf_all(std::integer_sequence<int, J...>, double (&a)[kS],
                                          double (*colbuf)[kNB], int r, int q, bool& bad) {
  (potrf_step<J>(a, colbuf, r, q, bad), ...);
}

template <int... I>
__device__ __forceinline__ void trinv_all(std::integer_sequence<int, I...>, double (&x)[kS],
                                          double (*rowbuf)[kNB], const double (*lf)[kNB + 1],
                                          int r, int q) {
  (trinv_step<I>(x, rowbuf, lf, r, q), ...);
}
}  // namespace

__global__ __launch_bounds__(256) void potrf_diag_kernel(double* H, int64_t d, int p,
                                                         double* dinv, int nblk, int* status) {
  constexpr int NB = kNB;
  static_assert(NB == 64, "register layout assumes 64 x 64 blocks and 256 threads");
  __shared__ double colbuf[2][NB];
  __shared__ double lf[NB][NB + 1];
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
  potrf_all(std::make_integer_sequence<int, NB>{}, a, colbuf, r, q, bad);
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
  trinv_all(std::make_integer_sequence<int, NB>{}, x, colbuf, lf, r, q);
  double* Di = dinv + ((int64_t)l * nblk + p) * NB * NB;
#pragma unroll
  for (int s = 0; s < kS; ++s) {
    const int c = q + 4 * s;
    Di[r * NB + c] = c <= r ? x[s] : 0.0;
  }
}

void cholesky_batched(double* H, int64_t d, int nl, double* dinv, int* status_dev,
                      hipStream_t st) {
  const int NB = kNB;
  const int nblk = (int)cdiv(d, NB);
  for (int p = 0; p < nblk; ++p) {
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(nl), dim3(256), 0, st, H, d, p, dinv, nblk,
                       status_dev);
    IHS_CHECK_LAUNCH();
    const int64_t o = (int64_t)p * NB;
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
    // trailing lower triangle: H22 -= P P^T
    Gemm tg;
    tg.M = below;
    tg.N = below;
    tg.K = NB;
    tg.A = H + (o + NB) * d + o;
    tg.lda = d;
    tg.strideA = d * d;
    tg.B = H + (o + NB) * d + o;
    tg.ldb = d;
    tg.strideB = d * d;
    tg.C = H + (o + NB) * d + o + NB;
    tg.ldc = d;
    tg.strideC = d * d;
    tg.alpha = -1.0;
    tg.beta = 1.0;
    tg.batch = nl;
    tg.lower_only = 1;
    gemm(tg, DT::F64, false, DT::F64, true, st);
  }
}

__global__ void init_inverse_rows_kernel(double* X, int64_t d, int nl, int64_t r0, int64_t rows) {
  const int64_t per = rows * d;
  const int64_t total = per * nl;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(t / per);
    const int64_t e = t % per;
    const int64_t r = r0 + e / d, c = e % d;
    X[(int64_t)l * d * d + r * d + c] = (r == c) ? 1.0 : 0.0;
  }
}

void tri_inverse_batched(const double* Lf, int64_t d, int nl, const double* dinv, double* Linv,
                         hipStream_t st) {
  const int NB = kNB;
  const int nblk = (int)cdiv(d, NB);
  {
    int64_t blocks = cdiv(d * d * nl, 256);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(init_inverse_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Linv, d,
                       nl, (int64_t)0, d);
    IHS_CHECK_LAUNCH();
  }
  for (int I = 0; I < nblk; ++I) {
    const int64_t o = (int64_t)I * NB;
    const int64_t rows = (d - o) < NB ? (d - o) : NB;
    if (I > 0) {
      // X[I, 0:o] = -L[I, 0:o] X[0:o, 0:o]
      Gemm g;
      g.M = rows;
      g.N = o;
      g.K = o;
      g.A = Lf + o * d;
      g.lda = d;
      g.strideA = d * d;
      g.B = Linv;
      g.ldb = d;
      g.strideB = d * d;
      g.C = Linv + o * d;
      g.ldc = d;
      g.strideC = d * d;
      g.alpha = -1.0;
      g.beta = 0.0;
      g.batch = nl;
      g.tri = 3;  // X[0:o, 0:o] is lower triangular
      gemm(g, DT::F64, false, DT::F64, false, st);
    }
    // X[I, 0:o+rows] = inv(L_II) X[I, 0:o+rows]   (in place, one row tile)
    Gemm h;
    h.M = rows;
    h.N = o + rows;
    h.K = rows;
    h.A = dinv + (int64_t)I * NB * NB;
    h.lda = NB;
    h.strideA = (int64_t)nblk * NB * NB;
    h.B = Linv + o * d;
    h.ldb = d;
    h.strideB = d * d;
    h.C = Linv + o * d;
    h.ldc = d;
    h.strideC = d * d;
    h.batch = nl;
    gemm(h, DT::F64, false, DT::F64, false, st);
  }
}

}  // namespace ihs
