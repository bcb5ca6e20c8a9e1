// Sketch generation and application (Section 4: Gaussian, CountSketch, SJLT,
// SRHT).  Integer draws follow the SplitMix64 counter specification; the
// SRHT transform runs as LDS-resident Walsh-Hadamard passes over digits of
// the row index.
#include <cmath>

#include <hipcub/hipcub.hpp>

#include "ops.hpp"

namespace ihs {

__global__ void draw_countsketch_kernel(uint64_t key, int64_t n, int64_t m, int s, int32_t* idx,
                                        int8_t* sign) {
  const int64_t total = n * s;
  const uint32_t mb = (uint32_t)(m / s);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t x = sm_draw(key, (uint64_t)t);  // t = i*s + b
    const int b = (int)(t % s);
    idx[t] = (int32_t)((uint32_t)b * mb + sm_range(x, mb));
    sign[t] = (x & 1ull) ? (int8_t)-1 : (int8_t)1;
  }
}

__global__ void identity_draws_kernel(int64_t n, int32_t* __restrict__ idx,
                                      int8_t* __restrict__ sign) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    idx[i] = (int32_t)i;
    sign[i] = 1;
  }
}

void launch_identity_draws(int64_t n, int32_t* idx, int8_t* sign, hipStream_t st) {
  int64_t blocks = cdiv(n, 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(identity_draws_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n, idx, sign);
  IHS_CHECK_LAUNCH();
}

void launch_draw_countsketch(uint64_t seed, int64_t n, int64_t m, int s, int32_t* idx,
                             int8_t* sign, hipStream_t st) {
  int64_t blocks = cdiv(n * s, 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(draw_countsketch_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     stream_key(seed, 0), n, m, s, idx, sign);
  IHS_CHECK_LAUNCH();
}

__global__ void draw_srht_kernel(uint64_t k1, uint64_t k2, int64_t n, int64_t npad, int64_t m,
                                 int8_t* sign, int32_t* rows) {
  const int64_t total = n > m ? n : m;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    if (t < n) sign[t] = (sm_draw(k1, (uint64_t)t) & 1ull) ? (int8_t)-1 : (int8_t)1;
    if (t < m) rows[t] = (int32_t)sm_range(sm_draw(k2, (uint64_t)t), (uint32_t)npad);
  }
}

void launch_draw_srht(uint64_t seed, int64_t n, int64_t npad, int64_t m, int8_t* sign,
                      int32_t* rows, hipStream_t st) {
  int64_t blocks = cdiv(n > m ? n : m, 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(draw_srht_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     stream_key(seed, 1), stream_key(seed, 2), n, npad, m, sign, rows);
  IHS_CHECK_LAUNCH();
}

// S (rows x n, row-major) = scale z for sketch rows r0 .. r0 + rows - 1:
// entry q = r n + i of the stream by its Box-Muller pair (q / 2).  One thread
// per pair slot: slot t holds chunk entries j = j0 + 2t and j + 1, j0 = -1
// when the chunk starts on an odd entry (that half belongs to the previous
// chunk and is not written).
__global__ void gaussian_fill_kernel(uint64_t key, int64_t r0, int64_t rows, int64_t n,
                                     double scale, double* S) {
  const int64_t total = rows * n, j0 = -((r0 * n) & 1);
  const int64_t slots = (total - j0 + 1) / 2;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < slots;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = j0 + 2 * t;
    const uint64_t p = (uint64_t)(r0 * n + j) >> 1;
    double zc, zs;
    box_muller64(sm_draw(key, 2ull * p), sm_draw(key, 2ull * p + 1ull), zc, zs);
    if (j >= 0) S[j] = scale * zc;
    if (j + 1 < total) S[j + 1] = scale * zs;
  }
}

void launch_gaussian_fill(uint64_t seed, int64_t m, int64_t r0, int64_t rows, int64_t n,
                          double* S, hipStream_t st) {
  int64_t blocks = cdiv(rows * n / 2 + 1, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(gaussian_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     stream_key(seed, 3), r0, rows, n, 1.0 / std::sqrt((double)m), S);
  IHS_CHECK_LAUNCH();
}

__global__ void scale_copy_kernel(const double* __restrict__ X, int64_t count, double f,
                                  double* __restrict__ Y) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x)
    Y[t] = f * X[t];
}

void launch_scale_copy(const double* X, int64_t count, double f, double* Y, hipStream_t st) {
  if (count <= 0) return;
  int64_t blocks = cdiv(count, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(scale_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, count, f, Y);
  IHS_CHECK_LAUNCH();
}

// The same draws transposed: St[i][r - r0] = S[r][i] for r0 <= r < r0 + rows
// (row stride `rows`), the layout a product A^T St gathers from.
__global__ void gaussian_fill_t_kernel(uint64_t key, int64_t r0, int64_t rows, int64_t n,
                                       double scale, double* St) {
  const int64_t total = rows * n, j0 = -((r0 * n) & 1);
  const int64_t slots = (total - j0 + 1) / 2;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < slots;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = j0 + 2 * t;
    const uint64_t p = (uint64_t)(r0 * n + j) >> 1;
    double z[2];
    box_muller64(sm_draw(key, 2ull * p), sm_draw(key, 2ull * p + 1ull), z[0], z[1]);
    for (int h = 0; h < 2; ++h) {
      const int64_t e = j + h;
      if (e < 0 || e >= total) continue;
      const int64_t r = e / n, i = e - r * n;
      St[i * rows + r] = scale * z[h];
    }
  }
}

void launch_gaussian_fill_t(uint64_t seed, int64_t m, int64_t r0, int64_t rows, int64_t n,
                            double* St, hipStream_t st) {
  int64_t blocks = cdiv(rows * n / 2 + 1, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(gaussian_fill_t_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     stream_key(seed, 3), r0, rows, n, 1.0 / std::sqrt((double)m), St);
  IHS_CHECK_LAUNCH();
}

// ----------------------------------------------------------- CountSketch
// One workgroup per row of A: row i is added, with its sign, to row idx of SA.
// Deterministic: the draws are sorted by bucket (a stable radix sort, so the
// rows of a bucket keep increasing order), and each output entry is summed
// in that order by one thread.
//  Dense A: bucket b of SA is the signed sum of the rows drawn into b, one
//  workgroup per bucket, threads over columns.
//  CSR A: every entry (row i, column c) of every block bb has the key
//  idx[i*s+bb] * d + c; after the stable sort, each run of equal keys is one
//  entry of SA, summed in row order (duplicates in their stored order).
namespace {

__global__ void iota_kernel(int32_t* __restrict__ v, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = (int32_t)i;
}

// ptr[b] = first sorted position whose key is >= b (b = 0..m)
__global__ void bucket_ptr_kernel(const int32_t* __restrict__ keys, int64_t count, int64_t m,
                                  int32_t* __restrict__ ptr) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= m;
       b += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = count;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < b) lo = mid + 1;
      else hi = mid;
    }
    ptr[b] = (int32_t)lo;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void countsketch_gather_dense_kernel(
    const T* __restrict__ A, int64_t d, int64_t ld, const int32_t* __restrict__ ptr,
    const int32_t* __restrict__ perm, const int8_t* __restrict__ sign, int s, double scale,
    int64_t m, double* __restrict__ SA) {
  for (int64_t b = blockIdx.x; b < m; b += gridDim.x) {
    const int32_t q0 = ptr[b], q1 = ptr[b + 1];
    for (int64_t c = threadIdx.x; c < d; c += blockDim.x) {
      double acc = 0.0;
      for (int32_t q = q0; q < q1; ++q) {
        const int32_t t = perm[q];
        acc += scale * (double)sign[t] * (double)A[(int64_t)(t / s) * ld + c];
      }
      SA[b * d + c] = acc;
    }
  }
}

__global__ void entry_keys_kernel(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  int64_t n, int64_t d, const int32_t* __restrict__ idx, int s,
                                  uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p0 = rp[i], p1 = rp[i + 1];
    for (int b = 0; b < s; ++b) {
      const uint64_t base = (uint64_t)idx[i * s + b] * (uint64_t)d;
      for (int32_t p = p0; p < p1; ++p) {
        const int64_t e = (int64_t)p * s + b;
        keys[e] = base + (uint64_t)ci[p];
        vals[e] = (int32_t)e;
      }
    }
  }
}

__global__ void row_of_entry_kernel(const int32_t* __restrict__ rp, int64_t n,
                                    int32_t* __restrict__ row) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) row[p] = (int32_t)i;
}

template <typename T>
__global__ void countsketch_runs_kernel(const uint64_t* __restrict__ keys,
                                        const int32_t* __restrict__ perm, int64_t count,
                                        const T* __restrict__ v, const int32_t* __restrict__ row_of,
                                        const int8_t* __restrict__ sign, int s, double scale,
                                        double* __restrict__ SA) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count;
       q += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[q];
    if (q > 0 && keys[q - 1] == k) continue;  // not the start of a run
    double acc = 0.0;
    for (int64_t r = q; r < count && keys[r] == k; ++r) {
      const int32_t e = perm[r];
      const int32_t p = e / s, b = e - p * s;
      acc += scale * (double)sign[(int64_t)row_of[p] * s + b] * (double)v[p];
    }
    SA[k] = acc;
  }
}

// flag[q] = 1 where a run of equal keys starts
__global__ void run_start_kernel(const uint64_t* __restrict__ keys, int64_t count,
                                 int32_t* __restrict__ flag) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count;
       q += (int64_t)gridDim.x * blockDim.x)
    flag[q] = (q == 0 || keys[q - 1] != keys[q]) ? 1 : 0;
}

// The runs as a CSR matrix: run j (j = run_idx[q] at its first position q)
// holds the column key % d and the signed sum of its entries in row order
// (the same sums as countsketch_runs_kernel); rkey[j] = its key.
template <typename T>
__global__ void countsketch_runs_csr_kernel(const uint64_t* __restrict__ keys,
                                            const int32_t* __restrict__ perm,
                                            const int32_t* __restrict__ run_idx, int64_t count,
                                            const T* __restrict__ v,
                                            const int32_t* __restrict__ row_of,
                                            const int8_t* __restrict__ sign, int s, double scale,
                                            int64_t d, uint64_t* __restrict__ rkey,
                                            int32_t* __restrict__ col, double* __restrict__ val) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count;
       q += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[q];
    if (q > 0 && keys[q - 1] == k) continue;  // not the start of a run
    double acc = 0.0;
    for (int64_t r = q; r < count && keys[r] == k; ++r) {
      const int32_t e = perm[r];
      const int32_t p = e / s, b = e - p * s;
      acc += scale * (double)sign[(int64_t)row_of[p] * s + b] * (double)v[p];
    }
    const int32_t j = run_idx[q];
    rkey[j] = k;
    col[j] = (int32_t)(k % (uint64_t)d);
    val[j] = acc;
  }
}

// row_ptr[b] = first run whose key is >= b d (b = 0..m)
__global__ void run_row_ptr_kernel(const uint64_t* __restrict__ rkey, int64_t nrun, int64_t m,
                                   int64_t d, int32_t* __restrict__ row_ptr) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= m;
       b += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = (uint64_t)b * (uint64_t)d;
    int64_t lo = 0, hi = nrun;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (rkey[mid] < key) lo = mid + 1;
      else hi = mid;
    }
    row_ptr[b] = (int32_t)lo;
  }
}

__global__ void zero_kernel(double* __restrict__ p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

unsigned blocks_for(int64_t count, int64_t cap = 16384) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(count, 256), cap));
}

int bits_for(uint64_t maxval) {
  int b = 1;
  while (b < 64 && (uint64_t(1) << b) <= maxval) ++b;
  return b;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

int64_t countsketch_work_bytes(const MatView& A, int64_t m, int s) {
  const int64_t ns = A.n * s;
  size_t tmp = 0;
  if (A.format == IHSBIN_DENSE) {
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const int32_t*)nullptr,
                                             (int32_t*)nullptr, (const int32_t*)nullptr,
                                             (int32_t*)nullptr, (int)ns, 0, 32);
    // draws (5 ns), sorted keys, iota, perm (4 ns each), bucket pointers
    return (int64_t)(align256(5 * ns) + 3 * align256(4 * ns) + align256(4 * (m + 1)) +
                     align256(tmp) + 256);
  }
  const int64_t es = A.nnz * s;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const uint64_t*)nullptr,
                                           (uint64_t*)nullptr, (const int32_t*)nullptr,
                                           (int32_t*)nullptr, (int)es, 0, 64);
  // draws, keys in/out (8 es each), values in/out (4 es each), row of entry
  return (int64_t)(align256(5 * ns) + 2 * align256(8 * es) + 2 * align256(4 * es) +
                   align256(4 * A.nnz) + align256(tmp) + 256);
}

void countsketch_apply(const MatView& A, uint64_t seed, int64_t m, int s, double* SA, void* work,
                       hipStream_t st) {
  const double scale = 1.0 / std::sqrt((double)s);
  const int64_t ns = A.n * s;
  if (ns >= INT32_MAX) fail(IHSBIN_EUNSUP, "CountSketch: too many rows");
  char* p = static_cast<char*>(work);
  auto take = [&](size_t bytes) {
    char* r = p;
    p += align256(bytes);
    return r;
  };
  int32_t* idx = reinterpret_cast<int32_t*>(take(4 * ns));
  int8_t* sg = reinterpret_cast<int8_t*>(take(ns));
  launch_draw_countsketch(seed, A.n, m, s, idx, sg, st);
  if (A.format == IHSBIN_DENSE) {
    int32_t* keys = reinterpret_cast<int32_t*>(take(4 * ns));
    int32_t* iota = reinterpret_cast<int32_t*>(take(4 * ns));
    int32_t* perm = reinterpret_cast<int32_t*>(take(4 * ns));
    int32_t* ptr = reinterpret_cast<int32_t*>(take(4 * (m + 1)));
    const int end_bit = bits_for((uint64_t)m);
    size_t tmp = 0;
    IHS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, idx, keys, iota, perm, (int)ns, 0,
                                               end_bit, st));
    void* tw = take(tmp);
    hipLaunchKernelGGL(iota_kernel, dim3(blocks_for(ns)), dim3(256), 0, st, iota, ns);
    IHS_CHECK_LAUNCH();
    IHS_HIP(hipcub::DeviceRadixSort::SortPairs(tw, tmp, idx, keys, iota, perm, (int)ns, 0, end_bit,
                                               st));
    hipLaunchKernelGGL(bucket_ptr_kernel, dim3(blocks_for(m + 1)), dim3(256), 0, st, keys, ns, m,
                       ptr);
    IHS_CHECK_LAUNCH();
    const unsigned g = (unsigned)std::min<int64_t>(m, 65536);
    if (A.dtype == IHSBIN_F32)
      hipLaunchKernelGGL(countsketch_gather_dense_kernel<float>, dim3(g), dim3(256), 0, st,
                         (const float*)A.vals, A.d, A.ld, ptr, perm, sg, s, scale, m, SA);
    else
      hipLaunchKernelGGL(countsketch_gather_dense_kernel<double>, dim3(g), dim3(256), 0, st,
                         (const double*)A.vals, A.d, A.ld, ptr, perm, sg, s, scale, m, SA);
    IHS_CHECK_LAUNCH();
    return;
  }
  const int64_t es = A.nnz * s;
  if (es >= INT32_MAX) fail(IHSBIN_EUNSUP, "CountSketch: too many entries");
  uint64_t* kin = reinterpret_cast<uint64_t*>(take(8 * es));
  uint64_t* kout = reinterpret_cast<uint64_t*>(take(8 * es));
  int32_t* vin = reinterpret_cast<int32_t*>(take(4 * es));
  int32_t* vout = reinterpret_cast<int32_t*>(take(4 * es));
  int32_t* row_of = reinterpret_cast<int32_t*>(take(4 * A.nnz));
  const int end_bit = bits_for((uint64_t)m * (uint64_t)A.d);
  size_t tmp = 0;
  IHS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, kin, kout, vin, vout, (int)es, 0, end_bit,
                                             st));
  void* tw = take(tmp);
  hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(m * A.d)), dim3(256), 0, st, SA, m * A.d);
  IHS_CHECK_LAUNCH();
  if (es == 0) return;
  hipLaunchKernelGGL(entry_keys_kernel, dim3(blocks_for(A.n)), dim3(256), 0, st, A.row_ptr,
                     A.col_idx, A.n, A.d, idx, s, kin, vin);
  IHS_CHECK_LAUNCH();
  hipLaunchKernelGGL(row_of_entry_kernel, dim3(blocks_for(A.n)), dim3(256), 0, st, A.row_ptr, A.n,
                     row_of);
  IHS_CHECK_LAUNCH();
  IHS_HIP(hipcub::DeviceRadixSort::SortPairs(tw, tmp, kin, kout, vin, vout, (int)es, 0, end_bit, st));
  if (A.dtype == IHSBIN_F32)
    hipLaunchKernelGGL(countsketch_runs_kernel<float>, dim3(blocks_for(es)), dim3(256), 0, st, kout,
                       vout, es, (const float*)A.vals, row_of, sg, s, scale, SA);
  else
    hipLaunchKernelGGL(countsketch_runs_kernel<double>, dim3(blocks_for(es)), dim3(256), 0, st, kout,
                       vout, es, (const double*)A.vals, row_of, sg, s, scale, SA);
  IHS_CHECK_LAUNCH();
}

int64_t countsketch_sparse_work_bytes(const MatView& A, int64_t m, int s) {
  const int64_t es = A.nnz * s;
  size_t scan = 0;
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan, (const int32_t*)nullptr, (int32_t*)nullptr,
                                         (int)std::max<int64_t>(es, 1));
  // the sort's arrays, then the run index (4 es) and its scan scratch
  return countsketch_work_bytes(A, m, s) + (int64_t)(align256(4 * es) + align256(scan) + 256);
}

int64_t countsketch_sparse_out_bytes(const MatView& A, int64_t m, int s) {
  const int64_t es = A.nnz * s;
  return (int64_t)(align256(4 * (m + 1)) + align256(4 * std::max<int64_t>(es, 1)) +
                   align256(8 * std::max<int64_t>(es, 1)) + 256);
}

int64_t countsketch_apply_sparse(const MatView& A, uint64_t seed, int64_t m, int s, void* work,
                                 void* out, SparseRows& sa, hipStream_t st) {
  if (A.format != IHSBIN_CSR) fail(IHSBIN_EINVAL, "sparse CountSketch of a dense matrix");
  const double scale = 1.0 / std::sqrt((double)s);
  const int64_t ns = A.n * s, es = A.nnz * s;
  if (ns >= INT32_MAX || es >= INT32_MAX) fail(IHSBIN_EUNSUP, "CountSketch: too many entries");
  char* p = static_cast<char*>(work);
  auto take = [&](size_t bytes) {
    char* r = p;
    p += align256(bytes);
    return r;
  };
  char* o = static_cast<char*>(out);
  sa.row_ptr = reinterpret_cast<int32_t*>(o);
  o += align256(4 * (m + 1));
  sa.col = reinterpret_cast<int32_t*>(o);
  o += align256(4 * std::max<int64_t>(es, 1));
  sa.val = reinterpret_cast<double*>(o);
  sa.m = m;
  sa.d = A.d;
  int32_t* idx = reinterpret_cast<int32_t*>(take(4 * ns));
  int8_t* sg = reinterpret_cast<int8_t*>(take(ns));
  launch_draw_countsketch(seed, A.n, m, s, idx, sg, st);
  uint64_t* kin = reinterpret_cast<uint64_t*>(take(8 * es));
  uint64_t* kout = reinterpret_cast<uint64_t*>(take(8 * es));
  int32_t* vin = reinterpret_cast<int32_t*>(take(4 * es));
  int32_t* vout = reinterpret_cast<int32_t*>(take(4 * es));
  int32_t* row_of = reinterpret_cast<int32_t*>(take(4 * A.nnz));
  const int end_bit = bits_for((uint64_t)m * (uint64_t)A.d);
  size_t tmp = 0;
  IHS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, kin, kout, vin, vout, (int)es, 0, end_bit,
                                             st));
  void* tw = take(tmp);
  int32_t* run_idx = reinterpret_cast<int32_t*>(take(4 * es));
  size_t scan = 0;
  IHS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan, vin, run_idx,
                                           (int)std::max<int64_t>(es, 1), st));
  void* sw = take(scan);
  if (es == 0) {
    hipLaunchKernelGGL(run_row_ptr_kernel, dim3(blocks_for(m + 1)), dim3(256), 0, st,
                       (const uint64_t*)kin, (int64_t)0, m, A.d, sa.row_ptr);
    IHS_CHECK_LAUNCH();
    sa.nnz = 0;
    return 0;
  }
  hipLaunchKernelGGL(entry_keys_kernel, dim3(blocks_for(A.n)), dim3(256), 0, st, A.row_ptr,
                     A.col_idx, A.n, A.d, idx, s, kin, vin);
  IHS_CHECK_LAUNCH();
  hipLaunchKernelGGL(row_of_entry_kernel, dim3(blocks_for(A.n)), dim3(256), 0, st, A.row_ptr, A.n,
                     row_of);
  IHS_CHECK_LAUNCH();
  IHS_HIP(hipcub::DeviceRadixSort::SortPairs(tw, tmp, kin, kout, vin, vout, (int)es, 0, end_bit, st));
  // vin is free after the sort: it holds the run-start flags
  hipLaunchKernelGGL(run_start_kernel, dim3(blocks_for(es)), dim3(256), 0, st, kout, es, vin);
  IHS_CHECK_LAUNCH();
  IHS_HIP(hipcub::DeviceScan::ExclusiveSum(sw, scan, vin, run_idx, (int)es, st));
  int32_t last[2] = {0, 0};
  IHS_HIP(hipMemcpyAsync(&last[0], run_idx + es - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  IHS_HIP(hipMemcpyAsync(&last[1], vin + es - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  // kin is free too: it receives the key of every run
  if (A.dtype == IHSBIN_F32)
    hipLaunchKernelGGL(countsketch_runs_csr_kernel<float>, dim3(blocks_for(es)), dim3(256), 0, st,
                       kout, vout, run_idx, es, (const float*)A.vals, row_of, sg, s, scale, A.d,
                       kin, sa.col, sa.val);
  else
    hipLaunchKernelGGL(countsketch_runs_csr_kernel<double>, dim3(blocks_for(es)), dim3(256), 0, st,
                       kout, vout, run_idx, es, (const double*)A.vals, row_of, sg, s, scale, A.d,
                       kin, sa.col, sa.val);
  IHS_CHECK_LAUNCH();
  IHS_HIP(hipStreamSynchronize(st));
  const int64_t nrun = (int64_t)last[0] + last[1];
  hipLaunchKernelGGL(run_row_ptr_kernel, dim3(blocks_for(m + 1)), dim3(256), 0, st,
                     (const uint64_t*)kin, nrun, m, A.d, sa.row_ptr);
  IHS_CHECK_LAUNCH();
  sa.nnz = nrun;
  return nrun;
}

// ----------------------------------------------------------------- SRHT
// Rows are indexed i = (h * len + t) * stride + l; one pass transforms over t
// for every (h, l) and a tile of CT columns, holding len x CT values in LDS.
constexpr int kFwhtCT = 8;
constexpr int kFwhtMaxLen = 512;

// load == 1: the source is A (rows < n, times sign), zero rows beyond n.
template <typename T, bool LOAD>
__global__ __launch_bounds__(256) void fwht_pass_kernel(const T* __restrict__ A, int64_t n,
                                                        int64_t ld, const int8_t* __restrict__ sign,
                                                        double* Z, int64_t npad, int64_t d,
                                                        int64_t stride, int len) {
  __shared__ double buf[kFwhtMaxLen][kFwhtCT + 1];
  const int64_t groups = npad / ((int64_t)len * stride);
  const int64_t ctiles = (d + kFwhtCT - 1) / kFwhtCT;
  const int64_t total = groups * stride * ctiles;
  for (int64_t job = blockIdx.x; job < total; job += gridDim.x) {
    const int64_t ct = job % ctiles;
    const int64_t hl = job / ctiles;
    const int64_t l = hl % stride, h = hl / stride;
    const int64_t c0 = ct * kFwhtCT;
    __syncthreads();
    for (int e = threadIdx.x; e < len * kFwhtCT; e += blockDim.x) {
      const int t = e / kFwhtCT, c = e % kFwhtCT;
      const int64_t row = (h * len + t) * stride + l;
      const int64_t col = c0 + c;
      double v = 0.0;
      if (col < d) {
        if (LOAD) {
          if (row < n) v = (double)sign[row] * (double)A[row * ld + col];
        } else {
          v = Z[row * d + col];
        }
      }
      buf[t][c] = v;
    }
    __syncthreads();
    for (int hlen = 1; hlen < len; hlen <<= 1) {
      for (int e = threadIdx.x; e < (len / 2) * kFwhtCT; e += blockDim.x) {
        const int p = e / kFwhtCT, c = e % kFwhtCT;
        const int blk = p / hlen, off = p % hlen;
        const int i0 = blk * 2 * hlen + off, i1 = i0 + hlen;
        const double a = buf[i0][c], b = buf[i1][c];
        buf[i0][c] = a + b;
        buf[i1][c] = a - b;
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < len * kFwhtCT; e += blockDim.x) {
      const int t = e / kFwhtCT, c = e % kFwhtCT;
      const int64_t row = (h * len + t) * stride + l;
      const int64_t col = c0 + c;
      if (col < d) Z[row * d + col] = buf[t][c];
    }
  }
}

// Register-blocked pass for len = 16 V (16 <= len <= 512) over a tile of 16
// columns: thread (c, g) first holds rows g + 16 k (k < V) of column c and
// transforms over k in registers; one LDS exchange regroups the rows as
// 16 kk + j (j < 16) and the transform over j finishes in registers.  The
// Walsh-Hadamard matrix factorizes over the two bit groups of the row index,
// so the two half-transforms compose to the full one.  Rows of 16 doubles
// (128 bytes) are read and written per thread group.
constexpr int kFwhtRC = 16;

// With `sample` (the last pass of a sampled transform) a finished row r is
// not stored in Z but written, times scale, to every row k of SA with
// rows[k] = r (sample->rk[sample->rstart[r] .. sample->rstart[r + 1]]).
struct RowSample {
  const int32_t* rstart;  // npad + 1
  const int32_t* rk;      // m: sample positions ordered by their row
  double scale;
  double* SA;
};

template <typename T, bool LOAD, int V>
__global__ __launch_bounds__(256) void fwht_reg_kernel(const T* __restrict__ A, int64_t n,
                                                       int64_t ld, const int8_t* __restrict__ sign,
                                                       double* Z, int64_t npad, int64_t d,
                                                       int64_t stride, RowSample sample) {
  constexpr int LEN = 16 * V;
  constexpr int PER = V >= 16 ? V / 16 : 1;  // row sets of 16 per thread in phase 2
  __shared__ double buf[LEN][kFwhtRC + 1];
  const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int64_t groups = npad / ((int64_t)LEN * stride);
  const int64_t ctiles = (d + kFwhtRC - 1) / kFwhtRC;
  const int64_t total = groups * stride * ctiles;
  for (int64_t job = blockIdx.x; job < total; job += gridDim.x) {
    const int64_t ct = job % ctiles;
    const int64_t hl = job / ctiles;
    const int64_t l = hl % stride, h = hl / stride;
    const int64_t col = ct * kFwhtRC + c;
    const bool cok = col < d;
    auto row_of = [&](int t) { return (h * LEN + t) * stride + l; };
    double v[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const int64_t row = row_of(g + 16 * k);
      double x = 0.0;
      if (cok) {
        if (LOAD) {
          if (row < n) x = (double)sign[row] * (double)A[row * ld + col];
        } else {
          x = Z[row * d + col];
        }
      }
      v[k] = x;
    }
#pragma unroll
    for (int hh = 1; hh < V; hh <<= 1)
#pragma unroll
      for (int k = 0; k < V; ++k)
        if ((k & hh) == 0) {
          const double a = v[k], b = v[k + hh];
          v[k] = a + b;
          v[k + hh] = a - b;
        }
    __syncthreads();  // the previous job's phase-2 reads are done
#pragma unroll
    for (int k = 0; k < V; ++k) buf[g + 16 * k][c] = v[k];
    __syncthreads();
    if (V >= 16 || g < V) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int kk = V >= 16 ? g * PER + q : g;
        double w[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) w[j] = buf[16 * kk + j][c];
#pragma unroll
        for (int hh = 1; hh < 16; hh <<= 1)
#pragma unroll
          for (int j = 0; j < 16; ++j)
            if ((j & hh) == 0) {
              const double a = w[j], b = w[j + hh];
              w[j] = a + b;
              w[j + hh] = a - b;
            }
        if (cok) {
          if (!sample.SA) {
#pragma unroll
            for (int j = 0; j < 16; ++j) Z[row_of(16 * kk + j) * d + col] = w[j];
          } else {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
              const int64_t row = row_of(16 * kk + j);
              for (int32_t q = sample.rstart[row]; q < sample.rstart[row + 1]; ++q)
                sample.SA[(int64_t)sample.rk[q] * d + col] = sample.scale * w[j];
            }
          }
        }
      }
    }
  }
}

template <typename T, bool LOAD>
static void launch_fwht_reg(int dg, unsigned blocks, hipStream_t st, const T* A, int64_t n,
                            int64_t ld, const int8_t* sign, double* Z, int64_t npad, int64_t d,
                            int64_t stride, const RowSample& sample) {
  switch (dg) {
#define IHS_FWHT_CASE(DG, V)                                                                   \
  case DG:                                                                                     \
    hipLaunchKernelGGL((fwht_reg_kernel<T, LOAD, V>), dim3(blocks), dim3(256), 0, st, A, n, ld, \
                       sign, Z, npad, d, stride, sample);                                      \
    break;
    IHS_FWHT_CASE(4, 1)
    IHS_FWHT_CASE(5, 2)
    IHS_FWHT_CASE(6, 4)
    IHS_FWHT_CASE(7, 8)
    IHS_FWHT_CASE(8, 16)
    IHS_FWHT_CASE(9, 32)
#undef IHS_FWHT_CASE
    default:
      fail(IHSBIN_EINVAL, "fwht: digit out of range");
  }
}

// CSR rows are scattered into the (zeroed) Z with their signs first.
template <typename T>
__global__ void csr_signed_scatter_kernel(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                          const T* __restrict__ v, int64_t n, int64_t d,
                                          const int8_t* __restrict__ sign, double* Z) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double sg = (double)sign[i];
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) Z[i * d + ci[p]] += sg * (double)v[p];
  }
}

bool launch_srht_transform(const MatView& A, const int8_t* sign, int64_t npad, double* Z,
                           hipStream_t st, const int32_t* rstart, const int32_t* rk,
                           double scale, double* SA) {
  const RowSample none{nullptr, nullptr, 0.0, nullptr};
  bool fused = false;
  int p = 0;
  while ((int64_t(1) << p) < npad) ++p;
  // digits of at most 9 bits, lowest first
  std::vector<int> digits;
  for (int left = p; left > 0;) {
    int take = left > 9 ? 9 : left;
    if (left > 9 && left < 18) take = left / 2;  // the reading pass takes the smaller digit
    digits.push_back(take);
    left -= take;
  }
  if (digits.empty()) digits.push_back(0);
  int64_t stride = 1;
  const int64_t ctiles = cdiv(A.d, kFwhtCT);
  bool first = true;
  if (A.format == IHSBIN_CSR) {
    IHS_HIP(hipMemsetAsync(Z, 0, (size_t)npad * A.d * sizeof(double), st));
    int64_t blocks = cdiv(A.n, 256);
    if (blocks > 16384) blocks = 16384;
    if (A.dtype == IHSBIN_F32)
      hipLaunchKernelGGL(csr_signed_scatter_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                         A.row_ptr, A.col_idx, (const float*)A.vals, A.n, A.d, sign, Z);
    else
      hipLaunchKernelGGL(csr_signed_scatter_kernel<double>, dim3((unsigned)blocks), dim3(256), 0,
                         st, A.row_ptr, A.col_idx, (const double*)A.vals, A.n, A.d, sign, Z);
    IHS_CHECK_LAUNCH();
    first = false;
  }
  for (size_t di = 0; di < digits.size(); ++di) {
    const int dg = digits[di];
    const int len = 1 << dg;
    if (dg >= 4) {
      const int64_t rjobs = (npad / ((int64_t)len * stride)) * stride * cdiv(A.d, kFwhtRC);
      const unsigned rblocks = (unsigned)(rjobs < 32768 ? rjobs : 32768);
      // the last pass writes the sampled rows straight into SA
      const bool last = di + 1 == digits.size() && SA != nullptr;
      const RowSample rs = last ? RowSample{rstart, rk, scale, SA} : none;
      fused = fused || last;
      if (first && A.format == IHSBIN_DENSE) {
        if (A.dtype == IHSBIN_F32)
          launch_fwht_reg<float, true>(dg, rblocks, st, (const float*)A.vals, A.n, A.ld, sign, Z,
                                       npad, A.d, stride, rs);
        else
          launch_fwht_reg<double, true>(dg, rblocks, st, (const double*)A.vals, A.n, A.ld, sign,
                                        Z, npad, A.d, stride, rs);
      } else {
        launch_fwht_reg<double, false>(dg, rblocks, st, (const double*)nullptr, A.n, A.ld, sign, Z,
                                       npad, A.d, stride, rs);
      }
      IHS_CHECK_LAUNCH();
      first = false;
      stride *= len;
      continue;
    }
    const int64_t jobs = (npad / ((int64_t)len * stride)) * stride * ctiles;
    const unsigned blocks = (unsigned)(jobs < 65536 ? jobs : 65536);
    if (first && A.format == IHSBIN_DENSE) {
      if (A.dtype == IHSBIN_F32)
        hipLaunchKernelGGL((fwht_pass_kernel<float, true>), dim3(blocks), dim3(256), 0, st,
                           (const float*)A.vals, A.n, A.ld, sign, Z, npad, A.d, stride, len);
      else
        hipLaunchKernelGGL((fwht_pass_kernel<double, true>), dim3(blocks), dim3(256), 0, st,
                           (const double*)A.vals, A.n, A.ld, sign, Z, npad, A.d, stride, len);
    } else {
      hipLaunchKernelGGL((fwht_pass_kernel<double, false>), dim3(blocks), dim3(256), 0, st,
                         (const double*)nullptr, A.n, A.ld, sign, Z, npad, A.d, stride, len);
    }
    IHS_CHECK_LAUNCH();
    first = false;
    stride *= len;
  }
  return fused;
}

// rk = the sample positions k ordered by rows[k] (stable), rstart[r] = the
// first of them whose row is >= r (r = 0..npad)
__global__ void row_start_kernel(const int32_t* __restrict__ sorted_rows, int64_t m, int64_t npad,
                                 int32_t* __restrict__ rstart) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= npad;
       r += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (sorted_rows[mid] < r) lo = mid + 1;
      else hi = mid;
    }
    rstart[r] = (int32_t)lo;
  }
}

int64_t row_sample_work_bytes(int64_t m, int64_t npad) {
  size_t tmp = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const int32_t*)nullptr, (int32_t*)nullptr,
                                           (const int32_t*)nullptr, (int32_t*)nullptr, (int)m, 0,
                                           32);
  return (int64_t)(4 * align256(4 * (size_t)m) + align256(4 * (size_t)(npad + 1)) + align256(tmp) +
                   256);
}

void build_row_sample(const int32_t* rows, int64_t m, int64_t npad, void* work,
                      const int32_t** rstart, const int32_t** rk, hipStream_t st) {
  if (m >= INT32_MAX || npad >= INT32_MAX) fail(IHSBIN_EUNSUP, "SRHT sample too large");
  char* p = static_cast<char*>(work);
  auto take = [&](size_t b) {
    char* r = p;
    p += align256(b);
    return r;
  };
  int32_t* keys = reinterpret_cast<int32_t*>(take(4 * (size_t)m));
  int32_t* iota = reinterpret_cast<int32_t*>(take(4 * (size_t)m));
  int32_t* sk = reinterpret_cast<int32_t*>(take(4 * (size_t)m));
  int32_t* sv = reinterpret_cast<int32_t*>(take(4 * (size_t)m));
  int32_t* rs = reinterpret_cast<int32_t*>(take(4 * (size_t)(npad + 1)));
  int end_bit = 1;
  while ((int64_t(1) << end_bit) < npad) ++end_bit;
  size_t tmp = 0;
  IHS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, keys, sk, iota, sv, (int)m, 0, end_bit,
                                             st));
  void* tw = take(tmp);
  IHS_HIP(hipMemcpyAsync(keys, rows, 4 * (size_t)m, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(iota_kernel, dim3(blocks_for(m)), dim3(256), 0, st, iota, m);
  IHS_CHECK_LAUNCH();
  IHS_HIP(hipcub::DeviceRadixSort::SortPairs(tw, tmp, keys, sk, iota, sv, (int)m, 0, end_bit, st));
  hipLaunchKernelGGL(row_start_kernel, dim3(blocks_for(npad + 1)), dim3(256), 0, st, sk, m, npad,
                     rs);
  IHS_CHECK_LAUNCH();
  *rstart = rs;
  *rk = sv;
}

__global__ void gather_rows_kernel(const double* __restrict__ Z, int64_t d,
                                   const int32_t* __restrict__ rows, int64_t m, double scale,
                                   double* __restrict__ SA) {
  const int64_t total = m * d;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t / d, c = t % d;
    SA[t] = scale * Z[(int64_t)rows[k] * d + c];
  }
}

void launch_gather_rows(const double* Z, int64_t d, const int32_t* rows, int64_t m, double scale,
                        double* SA, hipStream_t st) {
  int64_t blocks = cdiv(m * d, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Z, d, rows, m,
                     scale, SA);
  IHS_CHECK_LAUNCH();
}

}  // namespace ihs
