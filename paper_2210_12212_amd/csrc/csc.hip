// Column-major copy of a CSR matrix and the transposed product W = A^T Y
// gathered from it (no atomics, fixed summation order).
//
// The copy is a stable sort of the entries by column (LSD radix sort of the
// column indices with the entry positions as values), so every column lists
// its entries by increasing row: the result is the same bits on every run.
// Columns are cut into chunks of at most kCscChunk entries so that a heavy
// column (a skewed column distribution puts most rows into a few columns)
// is summed by many waves; a second pass adds the chunk partials of every
// column in chunk order.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "ops.hpp"

namespace ihs {

namespace {
constexpr int kCscChunk = 1024;

__global__ void row_of_entry_kernel(const int32_t* __restrict__ rp, int64_t n,
                                    int32_t* __restrict__ row) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) row[p] = (int32_t)i;
}

__global__ void iota_kernel(int32_t* __restrict__ v, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = (int32_t)i;
}

// col_ptr[c] = first sorted position whose column is >= c (c = 0..d)
__global__ void col_ptr_kernel(const int32_t* __restrict__ keys, int64_t nnz, int64_t d,
                               int32_t* __restrict__ col_ptr) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= d;
       c += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < c) lo = mid + 1;
      else hi = mid;
    }
    col_ptr[c] = (int32_t)lo;
  }
}

template <typename T>
__global__ void permute_kernel(const int32_t* __restrict__ perm, const int32_t* __restrict__ row_of,
                               const T* __restrict__ v, int64_t nnz, int32_t* __restrict__ row,
                               T* __restrict__ val) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = perm[q];
    row[q] = row_of[p];
    val[q] = v[p];
  }
}

__global__ void chunk_count_kernel(const int32_t* __restrict__ col_ptr, int64_t d,
                                   int32_t* __restrict__ cnt) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < d;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t len = col_ptr[c + 1] - col_ptr[c];
    cnt[c] = (len + kCscChunk - 1) / kCscChunk;
  }
}

__global__ void chunk_table_kernel(const int32_t* __restrict__ col_chunk, int64_t d,
                                   int32_t* __restrict__ chunk_col) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < d;
       c += (int64_t)gridDim.x * blockDim.x)
    for (int32_t t = col_chunk[c]; t < col_chunk[c + 1]; ++t) chunk_col[t] = (int32_t)c;
}

// key[t] = first row of chunk t, idx[t] = t
__global__ void chunk_first_row_kernel(const int32_t* __restrict__ col_ptr,
                                       const int32_t* __restrict__ col_chunk,
                                       const int32_t* __restrict__ chunk_col,
                                       const int32_t* __restrict__ row, int64_t nch,
                                       int32_t* __restrict__ key, int32_t* __restrict__ idx) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nch;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int c = chunk_col[t];
    key[t] = row[col_ptr[c] + (int32_t)(t - col_chunk[c]) * kCscChunk];
    idx[t] = (int32_t)t;
  }
}

unsigned grid_for(int64_t count) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(count, 256), 16384));
}

int pow2ceil(int64_t w) {
  int g = 1;
  while (g < w && g < 64) g <<= 1;
  return g;
}
}  // namespace

int64_t csc_work_bytes(const MatView& A) {
  const int64_t nnz = A.nnz, d = A.d;
  const int64_t es = A.dtype == IHSBIN_F32 ? 4 : 8;
  size_t sort_tmp = 0, scan_tmp = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sort_tmp, (const int32_t*)nullptr,
                                           (int32_t*)nullptr, (const int32_t*)nullptr,
                                           (int32_t*)nullptr, (int)nnz, 0, 32);
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan_tmp, (const int32_t*)nullptr,
                                         (int32_t*)nullptr, (int)(d + 1));
  size_t order_tmp = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, order_tmp, (const int32_t*)nullptr,
                                           (int32_t*)nullptr, (const int32_t*)nullptr,
                                           (int32_t*)nullptr, (int)std::max<int64_t>(nnz, 1), 0, 32);
  // kept: col_ptr, col_chunk (d+1 each), row, val (nnz), chunk_col and order
  // (<= nnz/chunk + d each)
  // transient: row_of, keys_out, perm in/out (nnz each), counts, sort/scan scratch
  const int64_t kept = 4 * 2 * (d + 1) + (4 + es) * nnz + 2 * 4 * (nnz / kCscChunk + d + 1);
  const int64_t transient =
      4 * 4 * nnz + 4 * (d + 1) + (int64_t)std::max(std::max(sort_tmp, scan_tmp), order_tmp);
  return kept + transient + 16 * 256;
}

void build_csc(const MatView& A, void* work, Csc& out, hipStream_t st) {
  if (A.format != IHSBIN_CSR) fail(IHSBIN_EINVAL, "CSC copy of a dense matrix");
  const int64_t nnz = A.nnz, d = A.d, n = A.n;
  if (nnz >= INT32_MAX || d >= INT32_MAX) fail(IHSBIN_EUNSUP, "CSC copy: too many entries");
  const int64_t es = A.dtype == IHSBIN_F32 ? 4 : 8;
  char* p = static_cast<char*>(work);
  auto take = [&](int64_t bytes) {
    char* r = p;
    p += (bytes + 255) / 256 * 256;
    return r;
  };
  int32_t* col_ptr = reinterpret_cast<int32_t*>(take(4 * (d + 1)));
  int32_t* col_chunk = reinterpret_cast<int32_t*>(take(4 * (d + 1)));
  int32_t* row = reinterpret_cast<int32_t*>(take(4 * nnz));
  void* val = take(es * nnz);
  int32_t* chunk_col = reinterpret_cast<int32_t*>(take(4 * (nnz / kCscChunk + d + 1)));
  int32_t* order = reinterpret_cast<int32_t*>(take(4 * (nnz / kCscChunk + d + 1)));
  int32_t* row_of = reinterpret_cast<int32_t*>(take(4 * nnz));
  int32_t* keys_out = reinterpret_cast<int32_t*>(take(4 * nnz));
  int32_t* perm_in = reinterpret_cast<int32_t*>(take(4 * nnz));
  int32_t* perm_out = reinterpret_cast<int32_t*>(take(4 * nnz));
  int32_t* cnt = reinterpret_cast<int32_t*>(take(4 * (d + 1)));
  int end_bit = 1;
  while ((int64_t(1) << end_bit) < d) ++end_bit;
  size_t sort_tmp = 0, scan_tmp = 0, order_tmp = 0;
  IHS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_tmp, A.col_idx, keys_out, perm_in,
                                             perm_out, (int)nnz, 0, end_bit, st));
  IHS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_tmp, cnt, col_chunk, (int)(d + 1), st));
  IHS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, order_tmp, keys_out, perm_in, perm_out,
                                             order, (int)std::max<int64_t>(nnz, 1), 0, 32, st));
  const size_t tmp_bytes = std::max(std::max(sort_tmp, scan_tmp), order_tmp);
  void* tmp = take((int64_t)tmp_bytes);

  hipLaunchKernelGGL(row_of_entry_kernel, dim3(grid_for(n)), dim3(256), 0, st, A.row_ptr, n, row_of);
  IHS_CHECK_LAUNCH();
  hipLaunchKernelGGL(iota_kernel, dim3(grid_for(nnz)), dim3(256), 0, st, perm_in, nnz);
  IHS_CHECK_LAUNCH();
  size_t bytes = sort_tmp;
  IHS_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, bytes, A.col_idx, keys_out, perm_in, perm_out,
                                             (int)nnz, 0, end_bit, st));
  hipLaunchKernelGGL(col_ptr_kernel, dim3(grid_for(d + 1)), dim3(256), 0, st, keys_out, nnz, d,
                     col_ptr);
  IHS_CHECK_LAUNCH();
  if (A.dtype == IHSBIN_F32)
    hipLaunchKernelGGL(permute_kernel<float>, dim3(grid_for(nnz)), dim3(256), 0, st, perm_out,
                       row_of, static_cast<const float*>(A.vals), nnz, row, static_cast<float*>(val));
  else
    hipLaunchKernelGGL(permute_kernel<double>, dim3(grid_for(nnz)), dim3(256), 0, st, perm_out,
                       row_of, static_cast<const double*>(A.vals), nnz, row,
                       static_cast<double*>(val));
  IHS_CHECK_LAUNCH();
  hipLaunchKernelGGL(chunk_count_kernel, dim3(grid_for(d)), dim3(256), 0, st, col_ptr, d, cnt);
  IHS_CHECK_LAUNCH();
  IHS_HIP(hipMemsetAsync(cnt + d, 0, sizeof(int32_t), st));
  bytes = scan_tmp;
  IHS_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, bytes, cnt, col_chunk, (int)(d + 1), st));
  hipLaunchKernelGGL(chunk_table_kernel, dim3(grid_for(d)), dim3(256), 0, st, col_chunk, d,
                     chunk_col);
  IHS_CHECK_LAUNCH();
  int32_t nch = 0;
  IHS_HIP(hipMemcpyAsync(&nch, col_chunk + d, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  IHS_HIP(hipStreamSynchronize(st));
  // processing order of the chunks: by their first row (stable, so ties keep
  // chunk order).  Chunks that start near each other read nearby rows of the
  // gathered matrix while they run together; every chunk still writes its
  // own partial, so the order does not change any result.  The nnz-sized
  // transient arrays hold the keys (nch <= nnz: every chunk has an entry).
  if (nch > 0) {
    int nbits = 1;
    while ((int64_t(1) << nbits) < n) ++nbits;
    hipLaunchKernelGGL(chunk_first_row_kernel, dim3(grid_for(nch)), dim3(256), 0, st, col_ptr,
                       col_chunk, chunk_col, row, (int64_t)nch, row_of, perm_in);
    IHS_CHECK_LAUNCH();
    size_t need = 0;
    IHS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, need, row_of, keys_out, perm_in, order,
                                               (int)nch, 0, nbits, st));
    if (need > tmp_bytes) fail(IHSBIN_EUNSUP, "CSC copy: chunk sort scratch");
    bytes = tmp_bytes;
    IHS_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, bytes, row_of, keys_out, perm_in, order,
                                               (int)nch, 0, nbits, st));
  }
  out.col_ptr = col_ptr;
  out.col_chunk = col_chunk;
  out.row = row;
  out.val = val;
  out.chunk_col = chunk_col;
  out.order = order;
  out.nchunks = nch;
}

// ---------------------------------------------------------- head / tail
namespace {
template <typename T>
__global__ void head_fill_kernel(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const T* __restrict__ v, int64_t n,
                                 const int32_t* __restrict__ head_pos, int64_t ldh,
                                 T* __restrict__ AH) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
      const int32_t pos = head_pos[ci[p]];
      if (pos >= 0) AH[i * ldh + pos] += v[p];  // duplicates in stored order
    }
}

__global__ void tail_count_kernel(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  int64_t n, const int32_t* __restrict__ head_pos,
                                  int32_t* __restrict__ cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int32_t c = 0;
    if (i < n)
      for (int32_t p = rp[i]; p < rp[i + 1]; ++p) c += head_pos[ci[p]] < 0 ? 1 : 0;
    cnt[i] = c;
  }
}

template <typename T>
__global__ void tail_fill_kernel(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const T* __restrict__ v, int64_t n,
                                 const int32_t* __restrict__ head_pos,
                                 const int32_t* __restrict__ trp, int32_t* __restrict__ tci,
                                 T* __restrict__ tv) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int32_t q = trp[i];
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
      if (head_pos[ci[p]] < 0) {
        tci[q] = ci[p];
        tv[q] = v[p];
        ++q;
      }
  }
}

__global__ void zero_bytes_kernel(uint32_t* __restrict__ p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}
}  // namespace

void build_head_tail(const MatView& A, const Csc& csc, PoolBuf& buf, HeadTail& out,
                     hipStream_t st) {
  out = HeadTail();
  if (A.format != IHSBIN_CSR) return;
  const int64_t n = A.n, d = A.d, nnz = A.nnz;
  constexpr int64_t kMaxHead = 256;
  std::vector<int32_t> cp(d + 1);
  IHS_HIP(hipMemcpyAsync(cp.data(), csc.col_ptr, sizeof(int32_t) * (size_t)(d + 1),
                         hipMemcpyDeviceToHost, st));
  IHS_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> head, pos(d, -1);
  const int64_t need = std::max<int64_t>(1, n / 16);
  // the densest columns first when more than kMaxHead qualify
  std::vector<int32_t> cand;
  for (int64_t c = 0; c < d; ++c)
    if (cp[c + 1] - cp[c] >= need) cand.push_back((int32_t)c);
  if ((int64_t)cand.size() > kMaxHead) {
    std::stable_sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
      return cp[a + 1] - cp[a] > cp[b + 1] - cp[b];
    });
    cand.resize(kMaxHead);
    std::sort(cand.begin(), cand.end());
  }
  head = cand;
  const int64_t h = (int64_t)head.size();
  if (h == 0) return;
  for (int64_t k = 0; k < h; ++k) pos[head[k]] = (int32_t)k;
  const int64_t ldh = cdiv(h, 4) * 4;
  const size_t es = A.dtype == IHSBIN_F32 ? 4 : 8;
  size_t scan_tmp = 0;
  IHS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_tmp, (const int32_t*)nullptr,
                                           (int32_t*)nullptr, (int)(n + 1), st));
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t bytes = al(4 * h) + al(4 * d) + al(es * (size_t)n * ldh) + al(4 * (n + 1)) +
                       al(4 * std::max<int64_t>(nnz, 1)) + al(es * std::max<int64_t>(nnz, 1)) +
                       al(4 * std::max<int64_t>(csc.nchunks, 1)) + al(4 * (n + 1)) + al(scan_tmp);
  char* p = static_cast<char*>(buf.ensure(bytes));
  auto take = [&](size_t b) {
    char* r = p;
    p += al(b);
    return r;
  };
  int32_t* head_d = reinterpret_cast<int32_t*>(take(4 * h));
  int32_t* pos_d = reinterpret_cast<int32_t*>(take(4 * d));
  void* AH = take(es * (size_t)n * ldh);
  int32_t* trp = reinterpret_cast<int32_t*>(take(4 * (n + 1)));
  int32_t* tci = reinterpret_cast<int32_t*>(take(4 * std::max<int64_t>(nnz, 1)));
  void* tv = take(es * std::max<int64_t>(nnz, 1));
  int32_t* torder = reinterpret_cast<int32_t*>(take(4 * std::max<int64_t>(csc.nchunks, 1)));
  int32_t* cnt = reinterpret_cast<int32_t*>(take(4 * (n + 1)));
  void* tmp = take(scan_tmp);
  IHS_HIP(hipMemcpyAsync(head_d, head.data(), 4 * (size_t)h, hipMemcpyHostToDevice, st));
  IHS_HIP(hipMemcpyAsync(pos_d, pos.data(), 4 * (size_t)d, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(zero_bytes_kernel, dim3(grid_for(es * n * ldh / 4)), dim3(256), 0, st,
                     static_cast<uint32_t*>(AH), (int64_t)(es * n * ldh / 4));
  IHS_CHECK_LAUNCH();
  if (A.dtype == IHSBIN_F32)
    hipLaunchKernelGGL(head_fill_kernel<float>, dim3(grid_for(n)), dim3(256), 0, st, A.row_ptr,
                       A.col_idx, static_cast<const float*>(A.vals), n, pos_d, ldh,
                       static_cast<float*>(AH));
  else
    hipLaunchKernelGGL(head_fill_kernel<double>, dim3(grid_for(n)), dim3(256), 0, st, A.row_ptr,
                       A.col_idx, static_cast<const double*>(A.vals), n, pos_d, ldh,
                       static_cast<double*>(AH));
  IHS_CHECK_LAUNCH();
  hipLaunchKernelGGL(tail_count_kernel, dim3(grid_for(n + 1)), dim3(256), 0, st, A.row_ptr,
                     A.col_idx, n, pos_d, cnt);
  IHS_CHECK_LAUNCH();
  size_t sb = scan_tmp;
  IHS_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, sb, cnt, trp, (int)(n + 1), st));
  if (A.dtype == IHSBIN_F32)
    hipLaunchKernelGGL(tail_fill_kernel<float>, dim3(grid_for(n)), dim3(256), 0, st, A.row_ptr,
                       A.col_idx, static_cast<const float*>(A.vals), n, pos_d, trp, tci,
                       static_cast<float*>(tv));
  else
    hipLaunchKernelGGL(tail_fill_kernel<double>, dim3(grid_for(n)), dim3(256), 0, st, A.row_ptr,
                       A.col_idx, static_cast<const double*>(A.vals), n, pos_d, trp, tci,
                       static_cast<double*>(tv));
  IHS_CHECK_LAUNCH();
  // tail chunks in the copy's first-row order
  std::vector<int32_t> ord(std::max<int64_t>(csc.nchunks, 1)), ccol(std::max<int64_t>(csc.nchunks, 1));
  int32_t tnnz = 0;
  if (csc.nchunks > 0) {
    IHS_HIP(hipMemcpyAsync(ord.data(), csc.order, 4 * (size_t)csc.nchunks, hipMemcpyDeviceToHost,
                           st));
    IHS_HIP(hipMemcpyAsync(ccol.data(), csc.chunk_col, 4 * (size_t)csc.nchunks,
                           hipMemcpyDeviceToHost, st));
  }
  IHS_HIP(hipMemcpyAsync(&tnnz, trp + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  IHS_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> tord;
  for (int64_t k = 0; k < csc.nchunks; ++k)
    if (pos[ccol[ord[k]]] < 0) tord.push_back(ord[k]);
  if (!tord.empty())
    IHS_HIP(hipMemcpyAsync(torder, tord.data(), 4 * tord.size(), hipMemcpyHostToDevice, st));
  out.h = h;
  out.ldh = ldh;
  out.head_cols = head_d;
  out.head_pos = pos_d;
  out.AH = AH;
  out.tail = A;
  out.tail.row_ptr = trp;
  out.tail.col_idx = tci;
  out.tail.vals = tv;
  out.tail.nnz = tnnz;
  out.tail.csc = nullptr;
  out.tail.ht = nullptr;
  out.torder = torder;
  out.tnchunks = (int64_t)tord.size();
  IHS_HIP(hipStreamSynchronize(st));  // the host vectors above go out of scope
}

// P[t][j] = sum over the entries of chunk t of val * Y[row][j].  Lanes form
// groups of G = min(64, pow2ceil(w)) columns; the 64 / G groups of a wave take
// every (64/G)-th entry of the chunk and are added by a fixed butterfly.  The
// chunk's (row, val) pairs are loaded 64 at a time, one per lane, and handed
// to the groups with shuffles, so the loop issues only the loads of Y's rows
// (kGatherBatch in flight per lane); every lane adds its entries in
// increasing order.  Waves take the chunks in the order of `order`.
constexpr int kGatherBatch = 16;
template <typename T, typename TY>
__global__ __launch_bounds__(256) void csc_gather_kernel(
    const int32_t* __restrict__ col_ptr, const int32_t* __restrict__ col_chunk,
    const int32_t* __restrict__ chunk_col, const int32_t* __restrict__ order,
    const int32_t* __restrict__ row, const T* __restrict__ val, int64_t nchunks,
    const TY* __restrict__ Y, int64_t w, int64_t ldy, int G, int strips, double* __restrict__ P) {
  const int lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= nchunks * strips) return;
  const int64_t k = item / strips;
  const int strip = (int)(item - k * strips);
  const int64_t t = order ? order[k] : k;
  const int c = chunk_col[t];
  const int32_t q0 = col_ptr[c] + (int32_t)(t - col_chunk[c]) * kCscChunk;
  const int32_t q1 = min(q0 + kCscChunk, col_ptr[c + 1]);
  const int groups = 64 / G;
  const int grp = lane / G, cl = lane - grp * G;
  const int64_t j = (int64_t)strip * G + cl;
  const bool live = j < w;
  const int per = G;  // entries of a 64-entry block per group
  double acc = 0.0;
  for (int32_t b0 = q0; b0 < q1; b0 += 64) {
    const int cnt = q1 - b0 < 64 ? q1 - b0 : 64;
    int32_t my_row = 0;
    double my_val = 0.0;
    if (lane < cnt) {
      my_row = row[b0 + lane];
      my_val = (double)val[b0 + lane];
    }
    // group grp takes block entries grp, grp + groups, grp + 2 groups, ...
    for (int s0 = 0; s0 < per && s0 * groups < cnt; s0 += kGatherBatch) {
      double yv[kGatherBatch];
#pragma unroll
      for (int u = 0; u < kGatherBatch; ++u) {
        const int e = (s0 + u) * groups + grp;
        const int64_t r = __shfl(my_row, e & 63);
        yv[u] = (live && s0 + u < per && e < cnt) ? (double)Y[r * ldy + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kGatherBatch; ++u) {
        const int e = (s0 + u) * groups + grp;
        const double v = __shfl(my_val, e & 63);
        if (s0 + u < per && e < cnt) acc += v * yv[u];
      }
    }
  }
  for (int off = G; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
  if (grp == 0 && live) P[t * w + j] = acc;
}

// W[c][j] = sum of the chunk partials of column c in chunk order (0 if none)
__global__ void csc_reduce_kernel(const int32_t* __restrict__ col_chunk, int64_t d, int64_t w,
                                  const double* __restrict__ P, double* __restrict__ W,
                                  int64_t ldw, const int32_t* __restrict__ skip) {
  const int64_t total = d * w;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / w, j = e - c * w;
    if (skip && skip[c] >= 0) continue;  // a head column (written by its GEMM)
    double s = 0.0;
    for (int32_t t = col_chunk[c]; t < col_chunk[c + 1]; ++t) s += P[(int64_t)t * w + j];
    W[c * ldw + j] = s;
  }
}

int64_t csc_partial_doubles(const Csc& csc, int64_t w) { return csc.nchunks * w; }

void launch_csc_atb(const MatView& A, const Csc& csc, const void* Y, bool y_f32, int64_t w,
                    int64_t ldy, double* P, double* W, int64_t ldw, hipStream_t st,
                    const HeadTail* ht) {
  if (w <= 0) return;
  const int G = pow2ceil(w);
  const int strips = (int)cdiv(w, G);
  const bool split = ht && ht->h > 0;
  const int32_t* order = split ? ht->torder : csc.order;
  const int64_t nchunks = split ? ht->tnchunks : csc.nchunks;
  const int64_t items = nchunks * strips;
  if (items > 0) {
    const unsigned blocks = (unsigned)cdiv(items, 4);
    if (cdiv(items, 4) > INT32_MAX) fail(IHSBIN_EUNSUP, "CSC product: grid too large");
    const bool af = A.dtype == IHSBIN_F32;
    if (af && y_f32)
      hipLaunchKernelGGL((csc_gather_kernel<float, float>), dim3(blocks), dim3(256), 0, st,
                         csc.col_ptr, csc.col_chunk, csc.chunk_col, order, csc.row,
                         static_cast<const float*>(csc.val), nchunks,
                         static_cast<const float*>(Y), w, ldy, G, strips, P);
    else if (af)
      hipLaunchKernelGGL((csc_gather_kernel<float, double>), dim3(blocks), dim3(256), 0, st,
                         csc.col_ptr, csc.col_chunk, csc.chunk_col, order, csc.row,
                         static_cast<const float*>(csc.val), nchunks,
                         static_cast<const double*>(Y), w, ldy, G, strips, P);
    else if (y_f32)
      hipLaunchKernelGGL((csc_gather_kernel<double, float>), dim3(blocks), dim3(256), 0, st,
                         csc.col_ptr, csc.col_chunk, csc.chunk_col, order, csc.row,
                         static_cast<const double*>(csc.val), nchunks,
                         static_cast<const float*>(Y), w, ldy, G, strips, P);
    else
      hipLaunchKernelGGL((csc_gather_kernel<double, double>), dim3(blocks), dim3(256), 0, st,
                         csc.col_ptr, csc.col_chunk, csc.chunk_col, order, csc.row,
                         static_cast<const double*>(csc.val), nchunks,
                         static_cast<const double*>(Y), w, ldy, G, strips, P);
    IHS_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(csc_reduce_kernel, dim3(grid_for(A.d * w)), dim3(256), 0, st, csc.col_chunk,
                     A.d, w, P, W, ldw, split ? ht->head_pos : (const int32_t*)nullptr);
  IHS_CHECK_LAUNCH();
}

}  // namespace ihs
