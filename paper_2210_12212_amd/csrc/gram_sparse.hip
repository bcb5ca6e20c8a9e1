// Sketched Gram G = (SA)^T SA of a sparse sketch (CountSketch or SJLT of a
// CSR matrix, Section 4: such an SA keeps at most s nnz(A) entries).  The
// dense product would cost 2 m d^2 flop on mostly zero rows; here every entry
// (r, c) of SA adds its row r to row c of G:
//
//   G[c][c'] = sum over rows r holding column c of SA[r][c] SA[r][c'],
//
// which costs sum_r nnz(row r)^2 / 2 multiply-adds for the lower triangle.
// Row c of G is accumulated by one wave in LDS (c + 1 doubles), entry by
// entry in row order from the column-major copy of SA, so every sum has a
// fixed order.  A column with more than one chunk of entries (the column-
// major copy cuts columns into chunks of at most 1024) accumulates one
// partial row per chunk; the partials are added in chunk order afterwards.
// Within an entry, the lanes take the row's entries c' <= c (distinct
// columns, so no two lanes touch one LDS word); eight rows are loaded ahead.
// Output: the lower triangle and the full diagonal 64 x 64 tiles of G.
#include <algorithm>
#include <vector>

#include "ops.hpp"

namespace ihs {

namespace {
constexpr int kChunk = 1024;  // entries per chunk of the column-major copy
constexpr int kAhead = 8;     // rows of SA loaded ahead per wave

__global__ __launch_bounds__(64) void sparse_gram_kernel(
    const int32_t* __restrict__ col_ptr, const int32_t* __restrict__ col_chunk,
    const int32_t* __restrict__ chunk_col, const int32_t* __restrict__ crow,
    const double* __restrict__ cval, int64_t t_begin, int64_t t_end,
    const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, const double* __restrict__ v,
    int64_t d, const int64_t* __restrict__ poff, double* __restrict__ P, double* __restrict__ G) {
  extern __shared__ double acc[];
  const int lane = threadIdx.x;
  // the heaviest rows of G (large c) first: chunks in decreasing order
  const int64_t t = t_end - 1 - (int64_t)blockIdx.x;
  if (t < t_begin) return;
  const int c = chunk_col[t];
  const int32_t q0 = col_ptr[c] + (int32_t)(t - col_chunk[c]) * kChunk;
  const int32_t q1 = min(q0 + kChunk, col_ptr[c + 1]);
  for (int k = lane; k <= c; k += 64) acc[k] = 0.0;
  __syncthreads();
  for (int32_t b0 = q0; b0 < q1; b0 += 64) {
    const int cnt = q1 - b0 < 64 ? q1 - b0 : 64;
    int32_t my_s = 0, my_len = 0;
    double my_f = 0.0;
    if (lane < cnt) {
      const int32_t r = crow[b0 + lane];
      my_f = cval[b0 + lane];
      my_s = rp[r];
      my_len = rp[r + 1] - my_s;
    }
    for (int u0 = 0; u0 < cnt; u0 += kAhead) {
      int32_t cc[kAhead];
      double vv[kAhead];
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int e = (u0 + u) & 63;
        const int32_t s = __shfl(my_s, e), len = __shfl(my_len, e);
        const bool ok = u0 + u < cnt && lane < len;
        cc[u] = ok ? ci[s + lane] : INT32_MAX;
        vv[u] = ok ? v[s + lane] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int e = (u0 + u) & 63;
        const double f = __shfl(my_f, e);
        const int32_t s = __shfl(my_s, e), len = __shfl(my_len, e);
        if (cc[u] <= c) acc[cc[u]] += f * vv[u];
        // entries of a row beyond its first 64 (the row is finished before
        // the next entry's row starts)
        if (u0 + u < cnt)
          for (int k = 64 + lane; k < len; k += 64) {
            const int32_t col = ci[s + k];
            if (col <= c) acc[col] += f * v[s + k];
          }
      }
    }
  }
  __syncthreads();
  const int64_t off = poff[t];
  if (off >= 0) {
    for (int k = lane; k <= c; k += 64) P[off + k] = acc[k];
  } else {
    const int tile0 = c & ~63;
    for (int k = lane; k <= c; k += 64) {
      G[(int64_t)c * d + k] = acc[k];
      if (k >= tile0 && k < c) G[(int64_t)k * d + c] = acc[k];
    }
  }
}

// Rows c of G for the columns with several chunks: the chunk partials added
// in chunk order (and mirrored inside the diagonal tile).
__global__ __launch_bounds__(256) void sparse_gram_reduce_kernel(
    const int32_t* __restrict__ multi, const int32_t* __restrict__ col_chunk,
    const int64_t* __restrict__ poff, const double* __restrict__ P, int64_t d,
    double* __restrict__ G) {
  const int c = multi[blockIdx.y];
  const int tile0 = c & ~63;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= c;
       k += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int32_t t = col_chunk[c]; t < col_chunk[c + 1]; ++t) s += P[poff[t] + k];
    G[(int64_t)c * d + k] = s;
    if (k >= tile0 && k < c) G[k * d + c] = s;
  }
}

// Columns of SA without entries: row c of G (lower triangle) is zero, and so
// is column c inside its diagonal tile; no chunk writes them.
__global__ __launch_bounds__(256) void zero_empty_rows_kernel(const int32_t* __restrict__ col_ptr,
                                                              int64_t d, double* __restrict__ G) {
  for (int64_t c = blockIdx.x; c < d; c += gridDim.x) {
    if (col_ptr[c + 1] > col_ptr[c]) continue;
    const int64_t tile0 = c & ~int64_t(63);
    for (int64_t k = threadIdx.x; k <= c; k += blockDim.x) {
      G[c * d + k] = 0.0;
      if (k >= tile0 && k < c) G[k * d + c] = 0.0;
    }
  }
}
}  // namespace

void sparse_gram(Ctx& ctx, const SparseRows& sa, double* G) {
  hipStream_t st = ctx.stream;
  const int64_t d = sa.d;
  if (d > kSparseGramMaxD) fail(IHSBIN_EUNSUP, "sparse Gram: d too large");
  MatView view;
  view.format = IHSBIN_CSR;
  view.dtype = IHSBIN_F64;
  view.n = sa.m;
  view.d = d;
  view.ld = d;
  view.nnz = sa.nnz;
  view.vals = sa.val;
  view.row_ptr = sa.row_ptr;
  view.col_idx = sa.col;
  PoolBuf cb(ctx.pool), pb(ctx.pool), ob(ctx.pool), mb(ctx.pool);
  Csc csc;
  build_csc(view, cb.ensure((size_t)csc_work_bytes(view)), csc, st);  // synchronizes
  const int64_t nch = csc.nchunks;
  // partial rows for the columns with several chunks (host plan)
  std::vector<int32_t> col_chunk(d + 1);
  IHS_HIP(hipMemcpyAsync(col_chunk.data(), csc.col_chunk, sizeof(int32_t) * (size_t)(d + 1),
                         hipMemcpyDeviceToHost, st));
  IHS_HIP(hipStreamSynchronize(st));
  std::vector<int64_t> poff(std::max<int64_t>(nch, 1), -1);
  std::vector<int32_t> multi;
  int64_t total = 0;
  for (int64_t c = 0; c < d; ++c) {
    if (col_chunk[c + 1] - col_chunk[c] < 2) continue;
    multi.push_back((int32_t)c);
    for (int32_t t = col_chunk[c]; t < col_chunk[c + 1]; ++t) {
      poff[t] = total;
      total += c + 1;
    }
  }
  int64_t* poff_d = static_cast<int64_t*>(ob.ensure(sizeof(int64_t) * poff.size()));
  IHS_HIP(hipMemcpyAsync(poff_d, poff.data(), sizeof(int64_t) * poff.size(), hipMemcpyHostToDevice,
                         st));
  double* P = static_cast<double*>(pb.ensure(sizeof(double) * (size_t)std::max<int64_t>(total, 1)));
  int32_t* multi_d = nullptr;
  if (!multi.empty()) {
    multi_d = static_cast<int32_t*>(mb.ensure(sizeof(int32_t) * multi.size()));
    IHS_HIP(hipMemcpyAsync(multi_d, multi.data(), sizeof(int32_t) * multi.size(),
                           hipMemcpyHostToDevice, st));
  }
  // column ranges [lo, hi) by LDS need: c < 1024 (8 KB), then doubling
  for (int64_t lo = 0; lo < d;) {
    const int64_t hi = std::min<int64_t>(d, lo == 0 ? 1024 : 2 * lo);
    const int64_t t0 = col_chunk[lo], t1 = col_chunk[hi];
    if (t1 > t0) {
      const size_t lds = sizeof(double) * (size_t)hi;
      hipLaunchKernelGGL(sparse_gram_kernel, dim3((unsigned)(t1 - t0)), dim3(64), lds, st,
                         csc.col_ptr, csc.col_chunk, csc.chunk_col, csc.row,
                         static_cast<const double*>(csc.val), t0, t1, sa.row_ptr, sa.col, sa.val,
                         d, poff_d, P, G);
      IHS_CHECK_LAUNCH();
    }
    lo = hi;
  }
  if (!multi.empty()) {
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(d, 256), 32);
    hipLaunchKernelGGL(sparse_gram_reduce_kernel, dim3(gx, (unsigned)multi.size()), dim3(256), 0,
                       st, multi_d, csc.col_chunk, poff_d, P, d, G);
    IHS_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(zero_empty_rows_kernel, dim3((unsigned)std::min<int64_t>(d, 16384)),
                     dim3(256), 0, st, csc.col_ptr, d, G);
  IHS_CHECK_LAUNCH();
  // the buffers go back to the pool after the stream has used them
  IHS_HIP(hipStreamSynchronize(st));
}

}  // namespace ihs
