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

// Factor diagonal block p of every matrix in LDS, write L_pp back (upper part
// zeroed) and its inverse into dinv[l][p].  Both the factorization and the
// inversion are right-looking with one barrier per column: step j reads the
// pivot that step j-1 finished and updates everything to its right/below.
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* H, int64_t d, int p,
                                                         double* dinv, int nblk, int* status) {
  constexpr int NB = kNB;
  __shared__ double a[NB][NB + 1];   // trailing matrix during the factorization
  __shared__ double lf[NB][NB + 1];  // the factor L
  __shared__ double x[NB][NB + 1];   // accumulators, then L^-1
  const int l = blockIdx.x;
  double* M = H + (int64_t)l * d * d;
  const int64_t o = (int64_t)p * NB;
  const int nb = (int)((d - o) < NB ? (d - o) : NB);
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int r = e / NB, c = e % NB;
    a[r][c] = (r < nb && c < nb) ? M[(o + r) * d + o + c] : (r == c ? 1.0 : 0.0);
    lf[r][c] = 0.0;
    x[r][c] = 0.0;
  }
  // four threads per row: thread (ti, tq) owns row ti, columns tq, tq + 4, ...
  const int ti = tid >> 2, tq = tid & 3;
  // factorization: a[i][k] -= a[i][j] a[k][j] / a[j][j] for j < k <= i
  for (int j = 0; j < NB; ++j) {
    __syncthreads();
    double djj = a[j][j];
    if (!(djj > 0.0)) {
      if (tid == 0) status[0] = 1;
      djj = 1.0;
    }
    const double piv = sqrt(djj), inv = 1.0 / djj;
    if (tq == 0 && ti >= j) lf[ti][j] = (ti == j) ? piv : a[ti][j] / piv;
    if (ti > j) {
      const double f = a[ti][j] * inv;
      for (int k = j + 1 + tq; k <= ti; k += 4) a[ti][k] -= f * a[k][j];
    }
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int r = e / NB, c = e % NB;
    if (r < nb && c < nb) M[(o + r) * d + o + c] = lf[r][c];
  }
  // inversion of L: row i of X is (e_i - acc_i) / L_ii, and rows below
  // accumulate L[r][i] X[i][:]; row i is finalized one step later (no reader then)
  for (int i = 0; i < NB; ++i) {
    __syncthreads();
    if (i > 0) {
      const double lp = lf[i - 1][i - 1];
      for (int c = tid; c < i; c += blockDim.x) x[i - 1][c] = ((i - 1 == c ? 1.0 : 0.0) - x[i - 1][c]) / lp;
    }
    const double lii = lf[i][i];
    if (ti > i) {
      const double f = lf[ti][i] / lii;
      for (int c = tq; c <= i; c += 4) x[ti][c] += f * ((i == c ? 1.0 : 0.0) - x[i][c]);
    }
  }
  __syncthreads();
  for (int c = tid; c < NB; c += blockDim.x)
    x[NB - 1][c] = ((NB - 1 == c ? 1.0 : 0.0) - x[NB - 1][c]) / lf[NB - 1][NB - 1];
  __syncthreads();
  double* Di = dinv + ((int64_t)l * nblk + p) * NB * NB;
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int r = e / NB, c = e % NB;
    Di[e] = (c <= r) ? x[r][c] : 0.0;
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
