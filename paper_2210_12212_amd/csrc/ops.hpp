// Launch wrappers of the library's kernels (all enqueue on the given stream).
#pragma once

#include "common.hpp"
#include "gemm.hpp"

namespace ihs {

// ------------------------------------------------------------ sketches
// CountSketch / SJLT draws: idx[i*s + b], sign[i*s + b] for row i, block b.
void launch_draw_countsketch(uint64_t seed, int64_t n, int64_t m, int s, int32_t* idx,
                             int8_t* sign, hipStream_t st);
// idx[i] = i, sign[i] = +1 (row i to row i: the identity as a CountSketch)
void launch_identity_draws(int64_t n, int32_t* idx, int8_t* sign, hipStream_t st);
// SRHT draws: sign[i] for i < n, rows[k] in [0, npad) for k < m.
void launch_draw_srht(uint64_t seed, int64_t n, int64_t npad, int64_t m, int8_t* sign,
                      int32_t* rows, hipStream_t st);
// S (rows x n, FP64) holding Gaussian rows [r0, r0 + rows) of the m x n sketch.
void launch_gaussian_fill(uint64_t seed, int64_t m, int64_t r0, int64_t rows, int64_t n,
                          double* S, hipStream_t st);
// Y[i] = f * X[i] for i < count.
void launch_scale_copy(const double* X, int64_t count, double f, double* Y, hipStream_t st);
void launch_gaussian_fill_t(uint64_t seed, int64_t m, int64_t r0, int64_t rows, int64_t n,
                            double* St, hipStream_t st);
// SA = S A for CountSketch / SJLT (s blocks), deterministic (bucket-sorted
// sums); work: countsketch_work_bytes(A, m, s) bytes of device scratch.
int64_t countsketch_work_bytes(const MatView& A, int64_t m, int s);
void countsketch_apply(const MatView& A, uint64_t seed, int64_t m, int s, double* SA, void* work,
                       hipStream_t st);
// A sketch held as a CSR matrix (m x d; FP64 values, columns increasing
// within a row).
struct SparseRows {
  int32_t* row_ptr = nullptr;        // m + 1
  int32_t* col = nullptr;            // nnz
  double* val = nullptr;             // nnz
  int64_t m = 0, d = 0, nnz = 0;
};
// SA = S A for CountSketch / SJLT of a CSR matrix, kept sparse: the entries
// of SA are the runs of the bucket-sorted entries of A (the same sums as
// countsketch_apply).  work: countsketch_sparse_work_bytes; out:
// countsketch_sparse_out_bytes (holds sa's arrays).  Returns nnz(SA).
int64_t countsketch_sparse_work_bytes(const MatView& A, int64_t m, int s);
int64_t countsketch_sparse_out_bytes(const MatView& A, int64_t m, int s);
int64_t countsketch_apply_sparse(const MatView& A, uint64_t seed, int64_t m, int s, void* work,
                                 void* out, SparseRows& sa, hipStream_t st);
// Lower triangle and diagonal 64 x 64 tiles of G = (SA)^T SA (d x d, FP64)
// for a sparse SA with d <= kSparseGramMaxD: each column c of SA (from its
// column-major copy, chunked) accumulates row c of G in LDS, entry by entry
// in row order.  Scratch from ctx's pool; returns when G is written.
constexpr int64_t kSparseGramMaxD = 8192;
void sparse_gram(Ctx& ctx, const SparseRows& sa, double* G);
// Z (npad x d) = D A zero-padded, then the Walsh-Hadamard transform over rows.
// With SA given (and rstart, rk from build_row_sample), the last pass writes
// scale * row rows[k] of the transform to row k of SA for every k instead of
// storing its rows in Z (Z then holds an intermediate pass); returns whether
// it did (false: Z holds the whole transform, gather it).
bool launch_srht_transform(const MatView& A, const int8_t* sign, int64_t npad, double* Z,
                           hipStream_t st, const int32_t* rstart = nullptr,
                           const int32_t* rk = nullptr, double scale = 0.0,
                           double* SA = nullptr);
// The m sampled rows grouped by row: rk lists the positions k by rows[k]
// (stable), rstart (npad + 1) points into it.  work: row_sample_work_bytes.
int64_t row_sample_work_bytes(int64_t m, int64_t npad);
void build_row_sample(const int32_t* rows, int64_t m, int64_t npad, void* work,
                      const int32_t** rstart, const int32_t** rk, hipStream_t st);
// SA[k] = scale * Z[rows[k]].
void launch_gather_rows(const double* Z, int64_t d, const int32_t* rows, int64_t m, double scale,
                        double* SA, hipStream_t st);

// ------------------------------------------------------------ factorization
// H_l = G + lam0_l I for l < nl (d x d each).
void launch_build_shifted(const double* G, int64_t d, const double* lam0_dev, int nl, double* H,
                          hipStream_t st, int gper = 0);
// In-place blocked Cholesky of nl matrices (lower factor, upper zeroed);
// dinv receives the inverses of the diagonal blocks (nl x nblk x 64 x 64).
// status_dev (int) is set non-zero when a pivot is not positive.
void cholesky_batched(double* H, int64_t d, int nl, double* dinv, int* status_dev,
                      hipStream_t st);
// The factor and its inverse together, by halves (recursive: L and
// X = L^-1 of every H_l; H's upper triangle zeroed, X's upper triangle zero).  status_dev as cholesky_batched;
// work: factor_inverse_work_doubles(d, nl) doubles.
// full = false: the top split's lower-left block of X is not formed (it
// holds L21 instead); L^-1 is then [X11 0; -X22 L21 X11  X22] with
// n1 = factor_top_split(d), X11 = X[0:n1, 0:n1], X22 = X[n1:, n1:] and L21
// from H.
void factor_inverse_batched(double* H, double* X, int64_t d, int nl, double* dinv,
                            int* status_dev, double* work, hipStream_t st, bool full = true);
int64_t factor_inverse_work_doubles(int64_t d, int nl);
int64_t factor_top_split(int64_t d);
constexpr int kNB = 64;

// ------------------------------------------------------------ products with A
// W = A^T A U (d x w), FP64.  Uses ctx scratch for Y = A U and split-K partials.
// When wmax > w (and wmax <= ldu), columns [w, wmax) of U exist and may be read
// (their values are ignored): the dense GEMMs then run ragged widths on the
// unchecked load path.  padded_width(w) (16, 32 or a multiple of 64) bounds
// the columns read.  Only columns [0, w) of W are written; returns w.
// Sketched Gram on the BF16 matrix cores with three-term splits (FP32 sums of
// at most kMaxSplitRows rows, split partials part[s] (d x d FP64) to be added
// in FP64; every tile touching the lower triangle is written).  work:
// gram_bf16x3_work_bytes(m, d) bytes for the split terms.
constexpr int64_t kMaxSplitRows = 2048;
int gram_bf16x3_splits(int64_t m);
int64_t gram_bf16x3_work_bytes(int64_t m, int64_t d);
void gram_bf16x3(const double* X, int64_t m, int64_t d, int64_t ldx, void* work, double* part,
                 int splits, hipStream_t st);

// XS[p][c][k] (terms x d x mpad BF16, rows k >= m zero) = term p of the
// BF16 split x = x0 + x1 + x2 + ... of X[k][c] (each term the BF16 rounding of
// what the earlier ones leave; X: m x d, FP32 or FP64, row stride ldx);
// terms = 2 or 3.
void launch_split_transpose(const void* X, bool f32, int64_t m, int64_t d, int64_t ldx,
                            int64_t mpad, void* XS, int terms, hipStream_t st);
// Gaussian sketch on the BF16 matrix cores: SA = (1/sqrt(m)) G16 A where
// G16 = BF16(FP32(z)) of the same N(0,1) draws z as launch_gaussian_fill and
// A is split into two BF16 terms (what they leave is at most 2^-18 |a|).
// FP32 sums over at most kMaxSplitRows rows of A, then FP64.  work:
// sketch_bf16_work_bytes(m, n, d) bytes.
int64_t sketch_bf16_work_bytes(int64_t m, int64_t n, int64_t d);
// Rows [r_begin, m) only (earlier rows of SA are left alone).
void gaussian_sketch_bf16(const MatView& A, uint64_t seed, int64_t m, double* SA, void* work,
                          double* part, int64_t part_doubles, hipStream_t st,
                          int64_t r_begin = 0);
int64_t gaussian_sketch_bf16_part_doubles(int64_t m, int64_t n, int64_t d);
// Gaussian sketch on the FP8 matrix cores: SA = (1/sqrt(m)) S8 A~ where
// S8 = E4M3(FP32(z)) of the same draws and A~ is A in three e4m3 terms under a
// per-column power-of-two scale (about 12 bits relative to the column's
// largest entry).  Sums as in the BF16 form.  Rows [r_begin, m) only.
int64_t sketch_fp8_work_bytes(int64_t m, int64_t n, int64_t d);
int64_t gaussian_sketch_fp8_part_doubles(int64_t m, int64_t n, int64_t d);
void gaussian_sketch_fp8(const MatView& A, uint64_t seed, int64_t m, double* SA, void* work,
                         double* part, int64_t part_doubles, hipStream_t st,
                         int64_t r_begin = 0);

// Dual (n < d) helpers: At = A^T (d x n row-major, A's dtype; dense A only)
// and C = B widened to FP64 (rows x K contiguous).
void launch_transpose(const MatView& A, void* At, hipStream_t st);
// D (n x d FP64, contiguous) = the CSR matrix A (duplicates summed in order).
void launch_csr_densify(const MatView& A, double* D, hipStream_t st);
void launch_widen_rows(const void* B, int dtype, int64_t rows, int64_t K, int64_t ldb, double* C,
                       hipStream_t st);
// Z (rows x nb*K, row stride ldz) <- blocks blk[0..nb) of src[blocks][rows][K],
// and the scatter back into dst[blocks][rows][K].
void launch_gather_blocks(const double* src, const int32_t* blk, int nb, int64_t rows, int64_t K,
                          double* Z, int64_t ldz, hipStream_t st);
void launch_scatter_blocks(const double* Z, int64_t ldz, const int32_t* blk, int nb, int64_t rows,
                           int64_t K, double* dst, hipStream_t st);
int64_t padded_width(int64_t w);
// dst (rows x cols, row stride ldd) = src (row stride lds).
void launch_copy_rect(const double* src, int64_t lds, int64_t rows, int64_t cols, double* dst,
                      int64_t ldd, hipStream_t st);
// f32: products on the FP32 matrix cores (dense FP32 A only; each column of U
// scaled by a power of two into range and rounded to FP32, Y = A U kept in
// FP32, A^T Y summed in FP32 over at most 16384 rows and in FP64 across them,
// then scaled back).
// A forced tiling for tuning: q (16q-column tiles) and the split-K count of
// W = A^T Y (0: the library's choice).
struct TileForce {
  int q = 0, splits = 0;
};
int64_t ata_apply(Ctx& ctx, const MatView& A, const double* U, int64_t w, int64_t ldu, double* W,
                  int64_t ldw, std::vector<hipEvent_t>* ev, int64_t wmax = 0, bool f32 = false,
                  const TileForce* force = nullptr);
// Many problems of one shape (dense, problem p's matrix at A.vals + p *
// strideA elements): W = A_p^T A_p U for `groups` groups of P column blocks of
// `per` columns each (group g, problem p: columns (g P + p) per ...).  U must
// keep ata_batch_slack(per) readable columns after its last block.
int64_t ata_batch_slack(int64_t per);
// Grow the workspaces of ata_apply_batch to what `per` columns per problem need
// (so that calls captured into a graph allocate nothing).
void ata_batch_reserve(Ctx& ctx, const MatView& A, int P, int64_t per);
void ata_apply_batch(Ctx& ctx, const MatView& A, int64_t strideA, int P, int groups, int64_t per,
                     const double* U, int64_t ldu, double* W, int64_t ldw);
// C_p = A_p^T B_p for P problems (B_p at B + p * strideB elements), C: P blocks
// of d x K.
void atb_apply_batch(Ctx& ctx, const MatView& A, int64_t strideA, int P, const void* B,
                     int64_t K, int64_t ldb, int64_t strideB, double* C);
// C = A^T B (d x K), FP64, B in A's dtype (row stride ldb).
void atb_apply(Ctx& ctx, const MatView& A, const void* B, int64_t K, int64_t ldb, double* C);
// CSR kernels
void launch_csr_spmm(const MatView& A, const double* U, int64_t w, int64_t ldu, double* Y,
                     int64_t ldy, hipStream_t st);
void launch_csr_spmm_t(const MatView& A, const double* Y, int64_t w, int64_t ldy, double* W,
                       int64_t ldw, hipStream_t st);
void launch_csr_atb(const MatView& A, const void* B, int64_t K, int64_t ldb, double* C,
                    hipStream_t st);

// ------------------------------------------------ adaptive m (Algorithm 4)
// out[0..2] = (D.G, D.W, D.D) over count entries (W may be null: out[1] = 0);
// part: dots3_part_doubles() doubles of device scratch.  Fixed-order sums.
int dots3_part_doubles();
void launch_dots3(const double* D, const double* G, const double* W, int64_t count, double* part,
                  double* out, hipStream_t st);
// X -= tau D and Gr -= tau (W + lam D), elementwise over count entries.
void launch_alg4_step(double* X, double* Gr, const double* D, const double* W, int64_t count,
                      double tau, double lam, hipStream_t st);
// X = 0 and Gr = -C.
void launch_alg4_init(const double* C, double* X, double* Gr, int64_t count, hipStream_t st);

// ------------------------------------------------- CSR column-major copy
// Entries of every column by increasing row (a stable sort by column), cut
// into chunks of at most 1024 entries: chunks col_chunk[c] .. col_chunk[c+1]
// belong to column c, chunk_col[t] names the column of chunk t, and order
// lists the chunks by their first row (the order the gathers process them).
struct Csc {
  const int32_t* col_ptr = nullptr;    // d + 1
  const int32_t* col_chunk = nullptr;  // d + 1
  const int32_t* row = nullptr;        // nnz
  const void* val = nullptr;           // nnz, A's dtype
  const int32_t* chunk_col = nullptr;  // nchunks
  const int32_t* order = nullptr;      // nchunks
  int64_t nchunks = 0;
};
// The columns of a CSR matrix that hold at least n / 16 entries (at most
// 256 of them, increasing column order) kept as a dense n x h block AH (A's
// type, row stride ldh, zero where a row has no entry; duplicates summed in
// stored order), the other entries as a tail CSR matrix, and the column
// chunks of the tail columns in first-row order.  The products then run the
// head as dense GEMMs (one streaming pass over the n x w intermediate
// instead of one gather of its row per entry) and gather the tail.
struct HeadTail {
  int64_t h = 0, ldh = 0;
  const int32_t* head_cols = nullptr;  // h
  const int32_t* head_pos = nullptr;   // d: position in the head or -1
  const void* AH = nullptr;            // n x ldh
  MatView tail;                        // the tail entries (CSR, same n, d)
  const int32_t* torder = nullptr;     // tail chunks of the column-major copy
  int64_t tnchunks = 0;
};
// Builds `out` for A (CSR) and its column-major copy; device memory from
// `buf` (kept while used).  h = 0 (nothing allocated) when no column is
// dense enough.  Synchronizes the stream.
void build_head_tail(const MatView& A, const Csc& csc, PoolBuf& buf, HeadTail& out,
                     hipStream_t st);
int64_t csc_work_bytes(const MatView& A);
// Builds the copy inside `work` (csc_work_bytes(A) bytes, kept while used).
void build_csc(const MatView& A, void* work, Csc& out, hipStream_t st);
int64_t csc_partial_doubles(const Csc& csc, int64_t w);
// W (d x w, row stride ldw) = A^T Y for Y (n x w, row stride ldy, FP32 or
// FP64), gathered column by column; P: csc_partial_doubles(csc, w) doubles.
// ht: gather only the tail chunks and leave W's head rows untouched.
void launch_csc_atb(const MatView& A, const Csc& csc, const void* Y, bool y_f32, int64_t w,
                    int64_t ldy, double* P, double* W, int64_t ldw, hipStream_t st,
                    const HeadTail* ht = nullptr);

// ------------------------------------------------------------ basis kernels
struct StepParams;  // defined in basis.hip users
void launch_fill(double* p, int64_t count, double v, hipStream_t st);
void launch_zero_bytes(void* p, size_t bytes, hipStream_t st);

}  // namespace ihs
