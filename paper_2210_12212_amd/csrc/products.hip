// Products with the data matrix A: W = A^T A U for a batch of w columns
// (every A^T A u_{i,j} of one basis step, Algorithm 2, across all intervals
// and right-hand sides at once) and C = A^T B.
//
// Dense A: Y = A U (n x w) with the MFMA GEMM, then W = A^T Y with split-K
// over n and a deterministic reduction; A is read in its stored type and
// widened to FP64 in the GEMM staging.  Columns are processed in chunks so
// the n x w intermediate stays within a fixed scratch budget.
// CSR A: row-parallel gather for A U; A^T Y gathers per column from the
// column-major copy of A (csc.hip) in fixed order, or, without that copy,
// scatters rows with FP64 atomics.
// Every pass adds its algorithmic bytes to ctx.bytes_moved: A read once per
// product, the n x w intermediate written and read once, U read and W
// written once.
#include "ops.hpp"

namespace ihs {

static constexpr size_t kYBudget = size_t(6) << 30;  // bytes for the n x w intermediate

// Tuned column tilings (autotune.py); see choose_tiles.
struct TunedTile {
  int64_t n, d;
  int32_t dtype, prec, nb, q, splits;
};
#include "tuned_tiles.inc"

// Column tiling and split-K count of the W = A^T Y product for a chunk of cw
// columns: forced (tuning calls), else the tuned table for this shape and
// width class, else the cost model of pick_col_tiles / pick_splits_cols.
static void choose_tiles(const MatView& A, bool f32, int64_t cw, const TileForce* force,
                         ColTiles& ct, int& splits) {
  const int64_t nb = cdiv(cw, 16);
  ct = pick_col_tiles(cw);
  splits = pick_splits_cols(A.d, ct, A.n, 1024);
  bool tuned = false;
  for (int i = 0; i < kNumTunedTiles && !(force && force->q > 0); ++i) {
    const TunedTile& e = kTunedTiles[i];
    if (e.n == A.n && e.d == A.d && e.dtype == A.dtype && e.prec == (f32 ? 1 : 0) && e.nb == nb &&
        e.q >= 1 && e.q <= kColTileMaxQ) {
      ct = ColTiles{(int)cdiv(nb, e.q), e.q};
      splits = e.splits > 0 ? e.splits : pick_splits_cols(A.d, ct, A.n, 1024);
      tuned = true;
      break;
    }
  }
  if (force && force->q > 0) {
    ct = ColTiles{(int)cdiv(nb, force->q), std::min(force->q, kColTileMaxQ)};
    if (!tuned) splits = pick_splits_cols(A.d, ct, A.n, 1024);
  }
  if (force && force->splits > 0) splits = force->splits;
  if (splits > 256) splits = 256;
}

// Y = A U (w > 32): one wave per row, lanes over columns of U.  The row's entries (64
// at a time) are loaded once, one per lane, and broadcast with shuffles, so
// the loop over entries issues only the loads of U's rows (four in flight);
// each output sums its entries in stored order.
template <typename T>
__global__ __launch_bounds__(256) void csr_spmm_kernel(const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const T* __restrict__ v, int64_t n,
                                                       const double* __restrict__ U, int64_t w,
                                                       int64_t ldu, double* __restrict__ Y,
                                                       int64_t ldy) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < n; i += nwaves) {
    const int32_t p0 = rp[i], p1 = rp[i + 1];
    for (int64_t c0 = 0; c0 < w; c0 += 64) {
      const int64_t c = c0 + lane;
      const bool live = c < w;
      double acc = 0.0;
      for (int32_t q0 = p0; q0 < p1; q0 += 64) {
        const int cnt = p1 - q0 < 64 ? p1 - q0 : 64;
        int32_t my_col = 0;
        double my_val = 0.0;
        if (lane < cnt) {
          my_col = ci[q0 + lane];
          my_val = (double)v[q0 + lane];
        }
        int t = 0;
        for (; t + 4 <= cnt; t += 4) {
          const int64_t k0 = __shfl(my_col, t), k1 = __shfl(my_col, t + 1),
                        k2 = __shfl(my_col, t + 2), k3 = __shfl(my_col, t + 3);
          const double a0 = __shfl(my_val, t), a1 = __shfl(my_val, t + 1),
                       a2 = __shfl(my_val, t + 2), a3 = __shfl(my_val, t + 3);
          if (live) {
            const double u0 = U[k0 * ldu + c], u1 = U[k1 * ldu + c], u2 = U[k2 * ldu + c],
                         u3 = U[k3 * ldu + c];
            acc += a0 * u0;
            acc += a1 * u1;
            acc += a2 * u2;
            acc += a3 * u3;
          }
        }
        for (; t < cnt; ++t) {
          const int64_t k = __shfl(my_col, t);
          const double a = __shfl(my_val, t);
          if (live) acc += a * U[k * ldu + c];
        }
      }
      if (live) Y[i * ldy + c] = acc;
    }
  }
}

// Y = A U for narrow U (w <= 32): 64 / G rows per wave, G = pow2ceil(w) lanes
// per row over its columns.  Each group loads its row's entries G at a time
// (one per lane) and broadcasts them with shuffles; eight loads of U's rows
// are in flight per lane, and each output sums its entries in stored order
// (the same sums as csr_spmm_kernel).
template <typename T>
__global__ __launch_bounds__(256) void csr_spmm_narrow_kernel(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, const T* __restrict__ v,
    int64_t n, const double* __restrict__ U, int64_t w, int64_t ldu, double* __restrict__ Y,
    int64_t ldy, int G) {
  constexpr int NB = 8;
  const int lane = threadIdx.x & 63;
  const int rows_per_wave = 64 / G;
  const int grp = lane / G, cl = lane - grp * G;
  const int64_t i = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * rows_per_wave + grp;
  const bool rlive = i < n;
  const bool live = rlive && cl < w;
  const int32_t p0 = rlive ? rp[i] : 0, p1 = rlive ? rp[i + 1] : 0;
  int len = p1 - p0;  // the longest row of the wave bounds its (uniform) loop
  for (int off = 1; off < 64; off <<= 1) len = max(len, __shfl_xor(len, off, 64));
  double acc = 0.0;
  for (int q = 0; q < len; q += G) {
    int32_t my_col = 0;
    double my_val = 0.0;
    if (p0 + q + cl < p1) {
      my_col = ci[p0 + q + cl];
      my_val = (double)v[p0 + q + cl];
    }
    const int cnt = p1 - p0 - q;  // this group's entries left (may be <= 0)
    for (int t0 = 0; t0 < G && t0 < len - q; t0 += NB) {
      double uv[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int t = t0 + u;
        const int64_t k = __shfl(my_col, grp * G + (t < G ? t : 0));
        uv[u] = (live && t < G && t < cnt) ? U[k * ldu + cl] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int t = t0 + u;
        const double a = __shfl(my_val, grp * G + (t < G ? t : 0));
        if (t < G && t < cnt) acc += a * uv[u];
      }
    }
  }
  if (live) Y[i * ldy + cl] = acc;
}

template <typename T>
__global__ void csr_spmm_t_kernel(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const T* __restrict__ v, int64_t n, const double* __restrict__ Y,
                                  int64_t w, int64_t ldy, double* W, int64_t ldw) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < n; i += nwaves) {
    const int32_t p0 = rp[i], p1 = rp[i + 1];
    for (int64_t c = lane; c < w; c += 64) {
      const double y = Y[i * ldy + c];
      if (y == 0.0) continue;
      for (int32_t p = p0; p < p1; ++p) atomicAdd(W + (int64_t)ci[p] * ldw + c, (double)v[p] * y);
    }
  }
}

void launch_csr_spmm(const MatView& A, const double* U, int64_t w, int64_t ldu, double* Y,
                     int64_t ldy, hipStream_t st) {
  if (w <= 0 || A.n <= 0) return;
  if (w <= 32) {
    int G = 1;
    while (G < w) G <<= 1;
    const int64_t waves = cdiv(A.n, 64 / G);
    const int64_t nblk = cdiv(waves, 4);
    if (nblk > INT32_MAX) fail(IHSBIN_EUNSUP, "CSR product: too many rows");
    if (A.dtype == IHSBIN_F32)
      hipLaunchKernelGGL(csr_spmm_narrow_kernel<float>, dim3((unsigned)nblk), dim3(256), 0, st,
                         A.row_ptr, A.col_idx, (const float*)A.vals, A.n, U, w, ldu, Y, ldy, G);
    else
      hipLaunchKernelGGL(csr_spmm_narrow_kernel<double>, dim3((unsigned)nblk), dim3(256), 0, st,
                         A.row_ptr, A.col_idx, (const double*)A.vals, A.n, U, w, ldu, Y, ldy, G);
    IHS_CHECK_LAUNCH();
    return;
  }
  int64_t blocks = cdiv(A.n * 64, 256);
  if (blocks > 65536) blocks = 65536;
  if (A.dtype == IHSBIN_F32)
    hipLaunchKernelGGL(csr_spmm_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, A.row_ptr,
                       A.col_idx, (const float*)A.vals, A.n, U, w, ldu, Y, ldy);
  else
    hipLaunchKernelGGL(csr_spmm_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, A.row_ptr,
                       A.col_idx, (const double*)A.vals, A.n, U, w, ldu, Y, ldy);
  IHS_CHECK_LAUNCH();
}

void launch_csr_spmm_t(const MatView& A, const double* Y, int64_t w, int64_t ldy, double* W,
                       int64_t ldw, hipStream_t st) {
  int64_t blocks = cdiv(A.n * 64, 256);
  if (blocks > 65536) blocks = 65536;
  if (A.dtype == IHSBIN_F32)
    hipLaunchKernelGGL(csr_spmm_t_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                       A.row_ptr, A.col_idx, (const float*)A.vals, A.n, Y, w, ldy, W, ldw);
  else
    hipLaunchKernelGGL(csr_spmm_t_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       A.row_ptr, A.col_idx, (const double*)A.vals, A.n, Y, w, ldy, W, ldw);
  IHS_CHECK_LAUNCH();
}

// UH[k][j] = U[cols[k]][j] (k < h, j < w), and the inverse scatter of WH.
__global__ void gather_rows_by_index_kernel(const double* __restrict__ U, int64_t ldu,
                                            const int32_t* __restrict__ cols, int64_t h,
                                            int64_t w, double* __restrict__ UH) {
  const int64_t total = h * w;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t / w, j = t - k * w;
    UH[t] = U[(int64_t)cols[k] * ldu + j];
  }
}

__global__ void scatter_rows_by_index_kernel(const double* __restrict__ WH,
                                             const int32_t* __restrict__ cols, int64_t h,
                                             int64_t w, double* __restrict__ W, int64_t ldw) {
  const int64_t total = h * w;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t / w, j = t - k * w;
    W[(int64_t)cols[k] * ldw + j] = WH[t];
  }
}

__global__ void zero_rows_kernel(double* W, int64_t rows, int64_t cols, int64_t ld) {
  const int64_t total = rows * cols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x)
    W[(t / cols) * ld + t % cols] = 0.0;
}

static void zero_block(double* W, int64_t rows, int64_t cols, int64_t ld, hipStream_t st) {
  int64_t blocks = cdiv(rows * cols, 256);
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) return;
  hipLaunchKernelGGL(zero_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, W, rows, cols, ld);
  IHS_CHECK_LAUNCH();
}

// D (n x d, FP64, contiguous) = the CSR matrix, one thread per row adding
// its entries in stored order (duplicates summed).
template <typename T>
__global__ void csr_densify_kernel(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                   const T* __restrict__ v, int64_t n, int64_t d,
                                   double* __restrict__ D) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double* row = D + i * d;
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) row[ci[p]] += (double)v[p];
  }
}

void launch_csr_densify(const MatView& A, double* D, hipStream_t st) {
  zero_block(D, A.n, A.d, A.d, st);
  int64_t blocks = cdiv(A.n, 256);
  if (blocks > 16384) blocks = 16384;
  if (A.dtype == IHSBIN_F32)
    hipLaunchKernelGGL(csr_densify_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                       A.row_ptr, A.col_idx, (const float*)A.vals, A.n, A.d, D);
  else
    hipLaunchKernelGGL(csr_densify_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       A.row_ptr, A.col_idx, (const double*)A.vals, A.n, A.d, D);
  IHS_CHECK_LAUNCH();
}

template <typename T>
__global__ void csr_atb_kernel(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               const T* __restrict__ v, int64_t n, const T* __restrict__ B,
                               int64_t K, int64_t ldb, double* C) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    for (int64_t c = 0; c < K; ++c) {
      const double bv = (double)B[i * ldb + c];
      for (int32_t p = rp[i]; p < rp[i + 1]; ++p) atomicAdd(C + (int64_t)ci[p] * K + c, (double)v[p] * bv);
    }
}

void launch_csr_atb(const MatView& A, const void* B, int64_t K, int64_t ldb, double* C,
                    hipStream_t st) {
  zero_block(C, A.d, K, K, st);
  int64_t blocks = cdiv(A.n, 256);
  if (blocks > 16384) blocks = 16384;
  if (A.dtype == IHSBIN_F32)
    hipLaunchKernelGGL(csr_atb_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, A.row_ptr,
                       A.col_idx, (const float*)A.vals, A.n, (const float*)B, K, ldb, C);
  else
    hipLaunchKernelGGL(csr_atb_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, A.row_ptr,
                       A.col_idx, (const double*)A.vals, A.n, (const double*)B, K, ldb, C);
  IHS_CHECK_LAUNCH();
}

// ------------------------------------------------ dual (n < d) helpers
// At = A^T (d x n row-major, ld n) through 32 x 32 LDS tiles.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ A, int64_t n,
                                                        int64_t d, int64_t lda, T* __restrict__ At) {
  __shared__ T tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;
    if (r < n && c < d) tile[k][tx] = A[r * lda + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (r < n && c < d) At[c * n + r] = tile[tx][k];
  }
}

void launch_transpose(const MatView& A, void* At, hipStream_t st) {
  if (A.format != IHSBIN_DENSE) fail(IHSBIN_EUNSUP, "transpose of a CSR matrix");
  const unsigned gy = (unsigned)cdiv(A.n, 32), gx = (unsigned)cdiv(A.d, 32);
  if (gy > 65535u) fail(IHSBIN_EUNSUP, "transpose: too many rows");
  if (A.dtype == IHSBIN_F32)
    hipLaunchKernelGGL(transpose_kernel<float>, dim3(gx, gy), dim3(256), 0, st,
                       (const float*)A.vals, A.n, A.d, A.ld, (float*)At);
  else
    hipLaunchKernelGGL(transpose_kernel<double>, dim3(gx, gy), dim3(256), 0, st,
                       (const double*)A.vals, A.n, A.d, A.ld, (double*)At);
  IHS_CHECK_LAUNCH();
}

// C (rows x K, FP64, contiguous) = B (rows x K, stride ldb, FP32 or FP64)
template <typename T>
__global__ void widen_rows_kernel(const T* __restrict__ B, int64_t rows, int64_t K, int64_t ldb,
                                  double* __restrict__ C) {
  const int64_t total = rows * K;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x)
    C[t] = (double)B[(t / K) * ldb + t % K];
}

void launch_widen_rows(const void* B, int dtype, int64_t rows, int64_t K, int64_t ldb, double* C,
                       hipStream_t st) {
  int64_t blocks = cdiv(rows * K, 256);
  if (blocks > 16384) blocks = 16384;
  if (dtype == IHSBIN_F32)
    hipLaunchKernelGGL(widen_rows_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const float*)B, rows, K, ldb, C);
  else
    hipLaunchKernelGGL(widen_rows_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const double*)B, rows, K, ldb, C);
  IHS_CHECK_LAUNCH();
}

// Z (rows x nb*K, row stride ldz) <- blocks blk[b] of a block array
// src[blk][rows][K]; and the inverse scatter into dst[blk][rows][K].
__global__ void gather_blocks_kernel(const double* __restrict__ src, const int32_t* __restrict__ blk,
                                     int nb, int64_t rows, int64_t K, double* __restrict__ Z,
                                     int64_t ldz) {
  const int64_t cols = (int64_t)nb * K, total = rows * cols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / cols, col = t % cols;
    const int64_t b = col / K, kk = col % K;
    Z[r * ldz + col] = src[((int64_t)blk[b] * rows + r) * K + kk];
  }
}

__global__ void scatter_blocks_kernel(const double* __restrict__ Z, int64_t ldz,
                                      const int32_t* __restrict__ blk, int nb, int64_t rows,
                                      int64_t K, double* __restrict__ dst) {
  const int64_t cols = (int64_t)nb * K, total = rows * cols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / cols, col = t % cols;
    const int64_t b = col / K, kk = col % K;
    dst[((int64_t)blk[b] * rows + r) * K + kk] = Z[r * ldz + col];
  }
}

void launch_gather_blocks(const double* src, const int32_t* blk, int nb, int64_t rows, int64_t K,
                          double* Z, int64_t ldz, hipStream_t st) {
  int64_t blocks = cdiv(rows * nb * K, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(gather_blocks_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, blk, nb,
                     rows, K, Z, ldz);
  IHS_CHECK_LAUNCH();
}

void launch_scatter_blocks(const double* Z, int64_t ldz, const int32_t* blk, int nb, int64_t rows,
                           int64_t K, double* dst, hipStream_t st) {
  int64_t blocks = cdiv(rows * nb * K, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(scatter_blocks_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Z, ldz, blk,
                     nb, rows, K, dst);
  IHS_CHECK_LAUNCH();
}

__global__ void copy_rect_kernel(const double* __restrict__ src, int64_t lds, int64_t rows,
                                 int64_t cols, double* __restrict__ dst, int64_t ldd) {
  const int64_t total = rows * cols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / cols, c = t - r * cols;
    dst[r * ldd + c] = src[r * lds + c];
  }
}

void launch_copy_rect(const double* src, int64_t lds, int64_t rows, int64_t cols, double* dst,
                      int64_t ldd, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return;
  int64_t blocks = cdiv(rows * cols, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(copy_rect_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, lds, rows,
                     cols, dst, ldd);
  IHS_CHECK_LAUNCH();
}

int64_t padded_width(int64_t w) {
  if (w <= 16) return 16;
  if (w <= 32) return 32;
  return cdiv(w, 64) * 64;
}

// Per-column powers of two that bring each column's largest entry into
// [1/2, 1): the basis vectors u_{i,j} grow like ||P_S||^j (their powers of
// tau (lam - lam0) shrink accordingly), far beyond the FP32 range for small
// lam0 and large j.  Scaling by a power of two is exact, so each column keeps
// its full FP32 relative precision; the product is linear per column and is
// scaled back exactly.  Two passes: the largest binary exponent of every
// column (64 columns by 256 rows per workgroup, combined with an integer
// atomic maximum, which does not depend on order), then scale[c] = 2^-e
// (1 for a zero column).
constexpr int kNoExp = -2147483647;

__global__ void col_exp_init_kernel(int* __restrict__ ex, int64_t w) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < w;
       c += (int64_t)gridDim.x * blockDim.x)
    ex[c] = kNoExp;
}

__global__ __launch_bounds__(256) void col_exp_max_kernel(const double* __restrict__ U, int64_t ldu,
                                                          int64_t d, int64_t w,
                                                          int* __restrict__ ex) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * 64 + lane;
  const int64_t r0 = (int64_t)blockIdx.y * 256;
  double mx = 0.0;
  if (c < w) {
    const int64_t r1 = r0 + 256 < d ? r0 + 256 : d;
    for (int64_t r = r0 + wave; r < r1; r += 4) mx = fmax(mx, fabs(U[r * ldu + c]));
  }
  red[wave][lane] = mx;
  __syncthreads();
  if (wave == 0 && c < w) {
    mx = fmax(fmax(red[0][lane], red[1][lane]), fmax(red[2][lane], red[3][lane]));
    if (mx > 0.0 && isfinite(mx)) {
      int e = 0;
      frexp(mx, &e);
      atomicMax(ex + c, e);
    }
  }
}

__global__ void col_scale_kernel(const int* __restrict__ ex, int64_t w, double* __restrict__ scale) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < w;
       c += (int64_t)gridDim.x * blockDim.x)
    scale[c] = ex[c] == kNoExp ? 1.0 : ldexp(1.0, -ex[c]);
}

// U32 (d x span, row stride span) = U columns [0, w) times scale, rounded to
// FP32, zero beyond w.
__global__ void round_cols_f32_kernel(const double* __restrict__ U, int64_t ldu, int64_t d,
                                      int64_t w, int64_t span, const double* __restrict__ scale,
                                      float* __restrict__ U32) {
  const int64_t total = d * span;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / span, c = t - r * span;
    U32[t] = c < w ? (float)(U[r * ldu + c] * scale[c]) : 0.0f;
  }
}

// W columns [0, w) divided by their scale (exact: powers of two).
__global__ void unscale_cols_kernel(double* __restrict__ W, int64_t ldw, int64_t d, int64_t w,
                                    const double* __restrict__ scale) {
  const int64_t total = d * w;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / w, c = t - r * w;
    W[r * ldw + c] /= scale[c];
  }
}

// The FP32 form of the pair: Y32 = A U32, W = A^T Y32 (split-K partials in FP64).
static void ata_f32(Ctx& ctx, const MatView& A, const double* U, int64_t w, int64_t ldu, double* W,
                    int64_t ldw, std::vector<hipEvent_t>* ev, const TileForce* force) {
  hipStream_t st = ctx.stream;
  auto mark = [&]() {
    if (!ev) return;
    hipEvent_t e;
    IHS_HIP(hipEventCreate(&e));
    IHS_HIP(hipEventRecord(e, st));
    ev->push_back(e);
  };
  int64_t wc = (int64_t)(kYBudget / (sizeof(float) * (size_t)A.n));
  if (wc >= 64) wc = (wc / 64) * 64;
  if (wc > w) wc = w;
  if (wc < 1) wc = 1;
  ColTiles ct_full;
  int sp_full = 1;
  choose_tiles(A, true, wc, force, ct_full, sp_full);
  const int64_t span_max = (int64_t)ct_full.c * 16 * ct_full.q;
  const int64_t ycap = std::max(padded_width(wc), span_max);
  float* Y = static_cast<float*>(ctx.ws_y.ensure(sizeof(float) * (size_t)A.n * (size_t)ycap));
  const size_t u32_bytes = ((sizeof(float) * (size_t)A.d * (size_t)ycap + 255) / 256) * 256;
  const size_t sc_bytes = ((sizeof(double) * (size_t)ycap + 255) / 256) * 256;
  char* f32_base = static_cast<char*>(
      ctx.ws_f32.ensure(u32_bytes + sc_bytes + sizeof(int) * (size_t)ycap));
  float* U32 = reinterpret_cast<float*>(f32_base);
  double* scale = reinterpret_cast<double*>(f32_base + u32_bytes);
  int* ex = reinterpret_cast<int*>(f32_base + u32_bytes + sc_bytes);
  for (int64_t c0 = 0; c0 < w; c0 += wc) {
    const int64_t cw = (w - c0) < wc ? (w - c0) : wc;
    ColTiles ct;
    int tuned_splits = 1;
    choose_tiles(A, true, cw, force, ct, tuned_splits);
    const int64_t span = std::min<int64_t>((int64_t)ct.c * 16 * ct.q, ycap);
    hipLaunchKernelGGL(col_exp_init_kernel, dim3((unsigned)cdiv(cw, 256)), dim3(256), 0, st, ex, cw);
    IHS_CHECK_LAUNCH();
    if (cdiv(A.d, 256) > 65535) fail(IHSBIN_EUNSUP, "FP32 products: d too large");
    hipLaunchKernelGGL(col_exp_max_kernel, dim3((unsigned)cdiv(cw, 64), (unsigned)cdiv(A.d, 256)),
                       dim3(256), 0, st, U + c0, ldu, A.d, cw, ex);
    IHS_CHECK_LAUNCH();
    hipLaunchKernelGGL(col_scale_kernel, dim3((unsigned)cdiv(cw, 256)), dim3(256), 0, st, ex, cw,
                       scale);
    IHS_CHECK_LAUNCH();
    int64_t blocks = cdiv(A.d * span, 256);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(round_cols_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, U + c0, ldu,
                       A.d, cw, span, scale, U32);
    IHS_CHECK_LAUNCH();
    mark();
    Gemm g1;
    g1.M = A.n;
    g1.N = cw;
    g1.K = A.d;
    g1.A = A.vals;
    g1.lda = A.ld;
    g1.B = U32;
    g1.ldb = span;
    g1.n_read = span;
    g1.C = reinterpret_cast<double*>(Y);
    g1.ldc = span;
    gemm_cols_f32(g1, false, true, ct, st);
    mark();
    // FP32 sums over at most 16384 rows each, FP64 across them
    const int splits =
        (int)std::min<int64_t>(256, std::max<int64_t>(tuned_splits, cdiv(A.n, 16384)));
    Gemm g2;
    g2.M = A.d;
    g2.N = cw;
    g2.K = A.n;
    g2.A = A.vals;
    g2.lda = A.ld;
    g2.B = Y;
    g2.ldb = span;
    g2.n_read = span;
    if (splits > 1) {
      double* part = static_cast<double*>(
          ctx.ws_part.ensure(sizeof(double) * (size_t)splits * (size_t)A.d * (size_t)cw));
      g2.C = part;
      g2.ldc = cw;
      g2.strideC = A.d * cw;
      g2.splits = splits;
      gemm_cols_f32(g2, true, false, ct, st);
      mark();
      reduce_splits(part, splits, 1, A.d, cw, cw, A.d * cw, W + c0, ldw, 0, 1.0, 0.0, st);
    } else {
      g2.C = W + c0;
      g2.ldc = ldw;
      gemm_cols_f32(g2, true, false, ct, st);
      mark();
    }
    int64_t ub = cdiv(A.d * cw, 256);
    if (ub > 16384) ub = 16384;
    hipLaunchKernelGGL(unscale_cols_kernel, dim3((unsigned)ub), dim3(256), 0, st, W + c0, ldw, A.d,
                       cw, scale);
    IHS_CHECK_LAUNCH();
  }
}

int64_t ata_apply(Ctx& ctx, const MatView& A, const double* U, int64_t w, int64_t ldu, double* W,
                  int64_t ldw, std::vector<hipEvent_t>* ev, int64_t wmax, bool f32,
                  const TileForce* force) {
  hipStream_t st = ctx.stream;
  if (w <= 0) return 0;
  const bool dense = A.format == IHSBIN_DENSE;
  if (f32 && dense && A.dtype == IHSBIN_F32) {
    int64_t wc = (int64_t)(kYBudget / (sizeof(float) * (size_t)A.n));
    if (wc >= 64) wc = (wc / 64) * 64;
    if (wc > w) wc = w;
    if (wc < 1) wc = 1;
    ctx.bytes_moved += 2.0 * matrix_bytes(A) * (double)cdiv(w, wc) +
                       (double)w * (8.0 * (double)A.n + 12.0 * (double)A.d);
    ata_f32(ctx, A, U, w, ldu, W, ldw, ev, force);
    return w;
  }
  // U holds `readable` columns (w unless the caller sized it wider): column
  // tiles may read past w up to there, so ragged widths avoid the checked path
  const int64_t readable = wmax > w && wmax <= ldu ? wmax : w;
  int64_t wc = (int64_t)(kYBudget / (sizeof(double) * (size_t)A.n));
  if (wc >= 64) wc = (wc / 64) * 64;
  if (wc > w) wc = w;
  if (wc < 1) wc = 1;
  const int64_t ycap = dense ? padded_width(wc) : wc;
  double* Y = static_cast<double*>(ctx.ws_y.ensure(sizeof(double) * (size_t)A.n * (size_t)ycap));
  const DT ta = A.dtype == IHSBIN_F32 ? DT::F32 : DT::F64;
  auto mark = [&]() {
    if (!ev) return;
    hipEvent_t e;
    IHS_HIP(hipEventCreate(&e));
    IHS_HIP(hipEventRecord(e, st));
    ev->push_back(e);
  };
  ctx.bytes_moved += 2.0 * matrix_bytes(A) * (double)cdiv(w, wc) +
                     8.0 * (double)w * (2.0 * (double)A.n + 2.0 * (double)A.d);
  for (int64_t c0 = 0; c0 < w; c0 += wc) {
    const int64_t cw = (w - c0) < wc ? (w - c0) : wc;
    ColTiles ct;
    int tuned_splits = 1;
    choose_tiles(A, false, cw, force, ct, tuned_splits);
    const int64_t span = (int64_t)ct.c * 16 * ct.q;  // columns the tiles cover
    int64_t nread = readable - c0;
    if (nread > span) nread = span;
    mark();
    if (dense) {
      Gemm g1;
      g1.M = A.n;
      g1.N = cw;
      g1.K = A.d;
      g1.A = A.vals;
      g1.lda = A.ld;
      g1.B = U + c0;
      g1.ldb = ldu;
      g1.n_read = nread;
      g1.C = Y;
      g1.ldc = ycap;
      gemm_cols(g1, ta, false, ct, st);
    } else if (A.ht && A.ht->h > 0) {
      // Y = A_tail U + AH U_head: the tail rows gathered, the head columns
      // one dense product added onto them
      const HeadTail& ht = *A.ht;
      launch_csr_spmm(ht.tail, U + c0, cw, ldu, Y, cw, st);
      double* UH = static_cast<double*>(ctx.ws_tmp.ensure(sizeof(double) * (size_t)(ht.h * cw)));
      {
        int64_t b = cdiv(ht.h * cw, 256);
        if (b > 16384) b = 16384;
        hipLaunchKernelGGL(gather_rows_by_index_kernel, dim3((unsigned)b), dim3(256), 0, st,
                           U + c0, ldu, ht.head_cols, ht.h, cw, UH);
        IHS_CHECK_LAUNCH();
      }
      Gemm gh;
      gh.M = A.n;
      gh.N = cw;
      gh.K = ht.h;
      gh.A = ht.AH;
      gh.lda = ht.ldh;
      gh.B = UH;
      gh.ldb = cw;
      gh.C = Y;
      gh.ldc = cw;
      gh.beta = 1.0;
      gemm(gh, ta, false, DT::F64, false, st);
    } else {
      launch_csr_spmm(A, U + c0, cw, ldu, Y, cw, st);
    }
    mark();
    if (dense) {
      // Y columns [cw, span) are never written; the W tiles read them (their
      // results land in columns >= cw, which are not stored)
      const int splits = tuned_splits;
      Gemm g2;
      g2.M = A.d;
      g2.N = cw;
      g2.K = A.n;
      g2.A = A.vals;
      g2.lda = A.ld;
      g2.B = Y;
      g2.ldb = ycap;
      g2.n_read = span <= ycap ? span : ycap;
      if (splits > 1) {
        double* part = static_cast<double*>(
            ctx.ws_part.ensure(sizeof(double) * (size_t)splits * (size_t)A.d * (size_t)cw));
        g2.C = part;
        g2.ldc = cw;
        g2.strideC = A.d * cw;
        g2.splits = splits;
        gemm_cols(g2, ta, true, ct, st);
        mark();  // the timed span is the product kernel itself
        reduce_splits(part, splits, 1, A.d, cw, cw, A.d * cw, W + c0, ldw, 0, 1.0, 0.0, st);
      } else {
        g2.C = W + c0;
        g2.ldc = ldw;
        gemm_cols(g2, ta, true, ct, st);
        mark();
      }
    } else {
      if (A.csc) {
        const bool split = A.ht && A.ht->h > 0;
        const HeadTail* ht = split ? A.ht : nullptr;
        const int64_t pd = std::max<int64_t>(1, csc_partial_doubles(*A.csc, cw));
        int hs = 1;
        if (split) hs = pick_splits(ht->h, cw, A.n, 1, 2048);
        const int64_t hd = split ? ht->h * cw * (1 + hs) : 0;  // WH and its split partials
        double* P = static_cast<double*>(ctx.ws_part.ensure(sizeof(double) * (size_t)(pd + hd)));
        launch_csc_atb(A, *A.csc, Y, false, cw, cw, P, W + c0, ldw, st, ht);
        if (split) {
          // W's head rows: AH^T Y, split over n, reduced in fixed order
          double* WH = P + pd;
          double* part = WH + ht->h * cw;
          Gemm gw;
          gw.M = ht->h;
          gw.N = cw;
          gw.K = A.n;
          gw.A = ht->AH;
          gw.lda = ht->ldh;
          gw.B = Y;
          gw.ldb = cw;
          gw.C = part;
          gw.ldc = cw;
          gw.strideC = ht->h * cw;
          gw.splits = hs;
          gemm(gw, ta, true, DT::F64, false, st);
          reduce_splits(part, hs, 1, ht->h, cw, cw, ht->h * cw, WH, cw, 0, 1.0, 0.0, st);
          int64_t b = cdiv(ht->h * cw, 256);
          if (b > 16384) b = 16384;
          hipLaunchKernelGGL(scatter_rows_by_index_kernel, dim3((unsigned)b), dim3(256), 0, st, WH,
                             ht->head_cols, ht->h, cw, W + c0, ldw);
          IHS_CHECK_LAUNCH();
        }
        mark();
        continue;
      }
      zero_block(W + c0, A.d, cw, ldw, st);
      launch_csr_spmm_t(A, Y, cw, cw, W + c0, ldw, st);
      mark();
    }
  }
  return w;
}

int64_t ata_batch_slack(int64_t per) {
  const ColTiles ct = pick_col_tiles(per);
  return (int64_t)ct.c * 16 * ct.q - per;
}

// Workspace of one batched product: the n x ycap intermediates of pc
// problems per launch, and the split-K partials of the widest launch.
struct BatchPlan {
  ColTiles ct;
  int64_t span, ycap, pc;
  size_t y_bytes, part_bytes;
};
static BatchPlan batch_plan(const MatView& A, int P, int64_t per) {
  BatchPlan b;
  b.ct = pick_col_tiles(per);
  b.span = (int64_t)b.ct.c * 16 * b.ct.q;
  b.ycap = std::max(padded_width(per), b.span);
  // problems per launch so that their n x ycap intermediates fit the budget
  b.pc = (int64_t)(kYBudget / (sizeof(double) * (size_t)A.n * (size_t)b.ycap));
  b.pc = std::max<int64_t>(1, std::min<int64_t>(b.pc, P));
  b.y_bytes = sizeof(double) * (size_t)b.pc * (size_t)A.n * (size_t)b.ycap;
  b.part_bytes = 0;
  for (int64_t p0 = 0; p0 < P; p0 += b.pc) {
    const int64_t nb = std::min<int64_t>(b.pc, P - p0);
    const int splits = pick_splits_cols(A.d, b.ct, A.n, std::max<int64_t>(1, 1024 / nb));
    if (splits > 1)
      b.part_bytes = std::max(b.part_bytes, sizeof(double) * (size_t)splits * (size_t)nb *
                                                (size_t)A.d * (size_t)per);
  }
  return b;
}

void ata_batch_reserve(Ctx& ctx, const MatView& A, int P, int64_t per) {
  const BatchPlan b = batch_plan(A, P, per);
  ctx.ws_y.ensure(b.y_bytes);
  if (b.part_bytes) ctx.ws_part.ensure(b.part_bytes);
}

void ata_apply_batch(Ctx& ctx, const MatView& A, int64_t strideA, int P, int groups, int64_t per,
                     const double* U, int64_t ldu, double* W, int64_t ldw) {
  hipStream_t st = ctx.stream;
  if (per <= 0 || P <= 0 || groups <= 0) return;
  if (A.format != IHSBIN_DENSE) fail(IHSBIN_EUNSUP, "batched products need dense matrices");
  const BatchPlan bp = batch_plan(A, P, per);
  const ColTiles ct = bp.ct;
  const int64_t span = bp.span;
  const int64_t ycap = bp.ycap;
  const int64_t pc = bp.pc;
  double* Y = static_cast<double*>(ctx.ws_y.ensure(bp.y_bytes));
  const DT ta = A.dtype == IHSBIN_F32 ? DT::F32 : DT::F64;
  const size_t es = A.dtype == IHSBIN_F32 ? 4 : 8;
  ctx.bytes_moved += (double)groups * (double)P *
                     (2.0 * matrix_bytes(A) + 8.0 * (double)per * (2.0 * (double)A.n + 2.0 * (double)A.d));
  for (int g = 0; g < groups; ++g) {
    for (int64_t p0 = 0; p0 < P; p0 += pc) {
      const int nb = (int)std::min<int64_t>(pc, P - p0);
      const int64_t col0 = (int64_t)g * P * per + p0 * per;
      const char* Ab = static_cast<const char*>(A.vals) + (size_t)p0 * (size_t)strideA * es;
      Gemm g1;
      g1.M = A.n;
      g1.N = per;
      g1.K = A.d;
      g1.A = Ab;
      g1.lda = A.ld;
      g1.strideA = strideA;
      g1.B = U + col0;
      g1.ldb = ldu;
      g1.strideB = per;
      g1.n_read = span;
      g1.C = Y;
      g1.ldc = ycap;
      g1.strideC = A.n * ycap;
      g1.batch = nb;
      gemm_cols(g1, ta, false, ct, st);
      const int splits = pick_splits_cols(A.d, ct, A.n, std::max<int64_t>(1, 1024 / nb));
      Gemm g2;
      g2.M = A.d;
      g2.N = per;
      g2.K = A.n;
      g2.A = Ab;
      g2.lda = A.ld;
      g2.strideA = strideA;
      g2.B = Y;
      g2.ldb = ycap;
      g2.strideB = A.n * ycap;
      g2.n_read = span;
      g2.batch = nb;
      if (splits > 1) {
        double* part = static_cast<double*>(ctx.ws_part.ensure(
            sizeof(double) * (size_t)splits * (size_t)nb * (size_t)A.d * (size_t)per));
        g2.C = part;
        g2.ldc = per;
        g2.strideC = A.d * per;
        g2.splits = splits;
        gemm_cols(g2, ta, true, ct, st);
        reduce_splits(part, splits, nb, A.d, per, per, A.d * per, W + col0, ldw, per, 1.0, 0.0, st);
      } else {
        g2.C = W + col0;
        g2.ldc = ldw;
        g2.strideC = per;
        gemm_cols(g2, ta, true, ct, st);
      }
    }
  }
}

void atb_apply_batch(Ctx& ctx, const MatView& A, int64_t strideA, int P, const void* B,
                     int64_t K, int64_t ldb, int64_t strideB, double* C) {
  if (A.format != IHSBIN_DENSE) fail(IHSBIN_EUNSUP, "batched products need dense matrices");
  hipStream_t st = ctx.stream;
  ctx.bytes_moved += (double)P * (matrix_bytes(A) + (double)A.n * (double)K *
                                                        (A.dtype == IHSBIN_F32 ? 4.0 : 8.0));
  const DT ta = A.dtype == IHSBIN_F32 ? DT::F32 : DT::F64;
  const int splits = pick_splits(A.d, K, A.n, P);
  Gemm g;
  g.M = A.d;
  g.N = K;
  g.K = A.n;
  g.A = A.vals;
  g.lda = A.ld;
  g.strideA = strideA;
  g.B = B;
  g.ldb = ldb;
  g.strideB = strideB;
  g.batch = P;
  if (splits > 1) {
    double* part = static_cast<double*>(
        ctx.ws_part.ensure(sizeof(double) * (size_t)splits * (size_t)P * (size_t)A.d * (size_t)K));
    g.C = part;
    g.ldc = K;
    g.strideC = A.d * K;
    g.splits = splits;
    gemm(g, ta, true, ta, false, st);
    reduce_splits(part, splits, P, A.d, K, K, A.d * K, C, K, A.d * K, 1.0, 0.0, st);
  } else {
    g.C = C;
    g.ldc = K;
    g.strideC = A.d * K;
    gemm(g, ta, true, ta, false, st);
  }
}

void atb_apply(Ctx& ctx, const MatView& A, const void* B, int64_t K, int64_t ldb, double* C) {
  hipStream_t st = ctx.stream;
  ctx.bytes_moved += matrix_bytes(A) + (double)A.n * (double)K * (A.dtype == IHSBIN_F32 ? 4.0 : 8.0) +
                     8.0 * (double)A.d * (double)K;
  if (A.format == IHSBIN_CSR && A.csc) {
    double* P = static_cast<double*>(
        ctx.ws_part.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, csc_partial_doubles(*A.csc, K))));
    launch_csc_atb(A, *A.csc, B, A.dtype == IHSBIN_F32, K, ldb, P, C, K, st);
    return;
  }
  if (A.format == IHSBIN_CSR) {
    launch_csr_atb(A, B, K, ldb, C, st);
    return;
  }
  const DT ta = A.dtype == IHSBIN_F32 ? DT::F32 : DT::F64;
  const int splits = pick_splits(A.d, K, A.n, 1);
  Gemm g;
  g.M = A.d;
  g.N = K;
  g.K = A.n;
  g.A = A.vals;
  g.lda = A.ld;
  g.B = B;
  g.ldb = ldb;
  if (splits > 1) {
    double* part = static_cast<double*>(
        ctx.ws_part.ensure(sizeof(double) * (size_t)splits * (size_t)A.d * (size_t)K));
    g.C = part;
    g.ldc = K;
    g.strideC = A.d * K;
    g.splits = splits;
    gemm(g, ta, true, ta, false, st);
    reduce_splits(part, splits, 1, A.d, K, K, A.d * K, C, K, 0, 1.0, 0.0, st);
  } else {
    g.C = C;
    g.ldc = K;
    gemm(g, ta, true, ta, false, st);
  }
}

}  // namespace ihs
