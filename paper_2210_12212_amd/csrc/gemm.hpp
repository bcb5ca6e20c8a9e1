// FP64 matrix products on the CDNA matrix cores (v_mfma_f64_16x16x4f64).
#pragma once

#include "common.hpp"

namespace ihs {

enum class DT { F32, F64 };

// C = alpha * op(A) op(B) + beta * C with op(A) M x K and op(B) K x N.
// transA: A is stored K x M row-major (else M x K).  transB: B is stored
// N x K row-major (else K x N).  All row-major with leading dimensions.
struct Gemm {
  int64_t M = 0, N = 0, K = 0;
  const void* A = nullptr;
  int64_t lda = 0, strideA = 0;
  const void* B = nullptr;
  int64_t ldb = 0, strideB = 0;
  double* C = nullptr;
  int64_t ldc = 0, strideC = 0;
  double alpha = 1.0, beta = 0.0;
  int batch = 1;         // independent problems (strides above)
  int batch2 = 1;        // second batch dimension (requires splits == 1): problem
                         // (b, b2) adds b2 * strideX2 to each operand
  int64_t strideA2 = 0, strideB2 = 0, strideC2 = 0;
  int splits = 1;        // split-K: partial sums of (b, s) go to C + (b*splits+s)*strideC
  int tri = 0;           // 1: op(A) lower triangular, 2: op(A) upper triangular,
                         // 3: op(B) lower triangular, 4: op(B) upper triangular
                         // (zero K-slices are skipped)
  int lower_only = 0;    // compute only C tiles touching the lower triangle
  const int32_t* amap = nullptr;  // optional device map: problem b uses A + amap[b]*strideA
  int small_tiles = 0;   // 1: 64 x 64 tiles even for large M (FP64 x FP64 products
                         // with large N, e.g. the sketched Gram, reuse L2 better)
  int vec_ok = 0;        // set by gemm(): operands allow aligned 16-byte vector loads
  // Columns of op(B) that may be read (0: N).  When n_read > N, memory for
  // op(B) columns [N, n_read) exists (its values are ignored): tiles that end
  // inside it still take the unchecked load path, and their 16-column blocks
  // past N skip the matrix-core work.  Output columns >= N are never written.
  int64_t n_read = 0;
};

void gemm(const Gemm& g, DT ta, bool transA, DT tb, bool transB, hipStream_t s);

// C[b] = alpha * sum_s part[b*splits + s] + beta * C[b]   (M x N blocks)
void reduce_splits(const double* part, int splits, int batch, int64_t M, int64_t N,
                   int64_t ldp, int64_t stride_part, double* C, int64_t ldc,
                   int64_t strideC, double alpha, double beta, hipStream_t s);

// Column tiling for products whose width N varies call to call (the A^T A
// products): c column tiles of 16 q columns each, q <= kColTileMaxQ, chosen
// to cover N with the fewest 16-column blocks.  The caller sets n_read so that
// op(B) holds c * 16 q readable columns.
constexpr int kColTileMaxQ = 7;
struct ColTiles {
  int c, q;
};
ColTiles pick_col_tiles(int64_t N);
// op(A) of type ta (FP32/FP64), B FP64 not transposed, C FP64.
void gemm_cols(const Gemm& g, DT ta, bool transA, const ColTiles& ct, hipStream_t s);
int pick_splits_cols(int64_t M, const ColTiles& ct, int64_t K, int64_t target);
// The same products on the FP32 matrix cores (v_mfma_f32_16x16x4f32): op(A)
// and B FP32; C FP32 when c_f32 (no split-K, beta = 0), else FP64 (split-K
// partials or a plain FP64 result of FP32 sums).  g.C is then a float*
// reinterpreted through the double* field.
void gemm_cols_f32(const Gemm& g, bool transA, bool c_f32, const ColTiles& ct, hipStream_t s);

// Split-K for a lower_only product with M = N = n on 64 x 64 tiles (small_tiles):
// roughly `target` workgroups over the lower tiles.
int pick_splits_lower(int64_t n, int64_t K, int64_t target);

// Choose split-K so that roughly `target` workgroups run.
int pick_splits(int64_t M, int64_t N, int64_t K, int batch, int64_t target = 2048);

}  // namespace ihs
