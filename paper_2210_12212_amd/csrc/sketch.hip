// Sketch generation and application (Section 4: Gaussian, CountSketch, SJLT,
// SRHT).  Integer draws follow the SplitMix64 counter specification; the
// SRHT transform runs as LDS-resident Walsh-Hadamard passes over digits of
// the row index.
#include <cmath>

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

// Box-Muller on two 53-bit uniforms: u1 in (0, 1], u2 in [0, 1).
__global__ void gaussian_fill_kernel(uint64_t key, int64_t r0, int64_t rows, int64_t n,
                                     double scale, double* S) {
  const int64_t total = rows * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t q = (uint64_t)(r0 * n + t);
    const uint64_t x1 = sm_draw(key, 2ull * q);
    const uint64_t x2 = sm_draw(key, 2ull * q + 1ull);
    const double u1 = ((double)(x1 >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (double)(x2 >> 11) * 0x1.0p-53;
    S[t] = scale * sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
  }
}

void launch_gaussian_fill(uint64_t seed, int64_t m, int64_t r0, int64_t rows, int64_t n,
                          double* S, hipStream_t st) {
  int64_t blocks = cdiv(rows * n, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(gaussian_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     stream_key(seed, 3), r0, rows, n, 1.0 / std::sqrt((double)m), S);
  IHS_CHECK_LAUNCH();
}

// The same draws transposed: St[i][r - r0] = S[r][i] for r0 <= r < r0 + rows
// (row stride `rows`), the layout a product A^T St gathers from.
__global__ void gaussian_fill_t_kernel(uint64_t key, int64_t r0, int64_t rows, int64_t n,
                                       double scale, double* St) {
  const int64_t total = rows * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / rows, r = r0 + (t - i * rows);
    const uint64_t q = (uint64_t)(r * n + i);
    const uint64_t x1 = sm_draw(key, 2ull * q);
    const uint64_t x2 = sm_draw(key, 2ull * q + 1ull);
    const double u1 = ((double)(x1 >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (double)(x2 >> 11) * 0x1.0p-53;
    St[t] = scale * sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
  }
}

void launch_gaussian_fill_t(uint64_t seed, int64_t m, int64_t r0, int64_t rows, int64_t n,
                            double* St, hipStream_t st) {
  int64_t blocks = cdiv(rows * n, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(gaussian_fill_t_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     stream_key(seed, 3), r0, rows, n, 1.0 / std::sqrt((double)m), St);
  IHS_CHECK_LAUNCH();
}

// ----------------------------------------------------------- CountSketch
// One workgroup per row of A: row i is added, with its sign, to row idx of SA.
template <typename T>
__global__ void countsketch_dense_kernel(const T* __restrict__ A, int64_t n, int64_t d,
                                         int64_t ld, const int32_t* __restrict__ idx,
                                         const int8_t* __restrict__ sign, int s, double scale,
                                         double* SA) {
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    for (int b = 0; b < s; ++b) {
      const int64_t h = idx[i * s + b];
      const double sg = scale * (double)sign[i * s + b];
      for (int64_t c = threadIdx.x; c < d; c += blockDim.x)
        atomicAdd(SA + h * d + c, sg * (double)A[i * ld + c]);
    }
  }
}

template <typename T>
__global__ void countsketch_csr_kernel(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                       const T* __restrict__ v, int64_t n, int64_t d,
                                       const int32_t* __restrict__ idx,
                                       const int8_t* __restrict__ sign, int s, double scale,
                                       double* SA) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int b = 0; b < s; ++b) {
      const int64_t h = idx[i * s + b];
      const double sg = scale * (double)sign[i * s + b];
      for (int32_t p = rp[i]; p < rp[i + 1]; ++p) atomicAdd(SA + h * d + ci[p], sg * (double)v[p]);
    }
  }
}

void launch_countsketch_apply(const MatView& A, const int32_t* idx, const int8_t* sign, int s,
                              double* SA, hipStream_t st) {
  const double scale = 1.0 / std::sqrt((double)s);
  if (A.format == IHSBIN_DENSE) {
    const unsigned blocks = (unsigned)(A.n < 65536 ? A.n : 65536);
    if (A.dtype == IHSBIN_F32)
      hipLaunchKernelGGL(countsketch_dense_kernel<float>, dim3(blocks), dim3(256), 0, st,
                         (const float*)A.vals, A.n, A.d, A.ld, idx, sign, s, scale, SA);
    else
      hipLaunchKernelGGL(countsketch_dense_kernel<double>, dim3(blocks), dim3(256), 0, st,
                         (const double*)A.vals, A.n, A.d, A.ld, idx, sign, s, scale, SA);
  } else {
    int64_t blocks = cdiv(A.n, 256);
    if (blocks > 16384) blocks = 16384;
    if (A.dtype == IHSBIN_F32)
      hipLaunchKernelGGL(countsketch_csr_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                         A.row_ptr, A.col_idx, (const float*)A.vals, A.n, A.d, idx, sign, s, scale,
                         SA);
    else
      hipLaunchKernelGGL(countsketch_csr_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                         A.row_ptr, A.col_idx, (const double*)A.vals, A.n, A.d, idx, sign, s,
                         scale, SA);
  }
  IHS_CHECK_LAUNCH();
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

template <typename T, bool LOAD, int V>
__global__ __launch_bounds__(256) void fwht_reg_kernel(const T* __restrict__ A, int64_t n,
                                                       int64_t ld, const int8_t* __restrict__ sign,
                                                       double* Z, int64_t npad, int64_t d,
                                                       int64_t stride) {
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
#pragma unroll
          for (int j = 0; j < 16; ++j) Z[row_of(16 * kk + j) * d + col] = w[j];
        }
      }
    }
  }
}

template <typename T, bool LOAD>
static void launch_fwht_reg(int dg, unsigned blocks, hipStream_t st, const T* A, int64_t n,
                            int64_t ld, const int8_t* sign, double* Z, int64_t npad, int64_t d,
                            int64_t stride) {
  switch (dg) {
#define IHS_FWHT_CASE(DG, V)                                                                   \
  case DG:                                                                                     \
    hipLaunchKernelGGL((fwht_reg_kernel<T, LOAD, V>), dim3(blocks), dim3(256), 0, st, A, n, ld, \
                       sign, Z, npad, d, stride);                                              \
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

void launch_srht_transform(const MatView& A, const int8_t* sign, int64_t npad, double* Z,
                           hipStream_t st) {
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
  for (int dg : digits) {
    const int len = 1 << dg;
    if (dg >= 4) {
      const int64_t rjobs = (npad / ((int64_t)len * stride)) * stride * cdiv(A.d, kFwhtRC);
      const unsigned rblocks = (unsigned)(rjobs < 32768 ? rjobs : 32768);
      if (first && A.format == IHSBIN_DENSE) {
        if (A.dtype == IHSBIN_F32)
          launch_fwht_reg<float, true>(dg, rblocks, st, (const float*)A.vals, A.n, A.ld, sign, Z,
                                       npad, A.d, stride);
        else
          launch_fwht_reg<double, true>(dg, rblocks, st, (const double*)A.vals, A.n, A.ld, sign,
                                        Z, npad, A.d, stride);
      } else {
        launch_fwht_reg<double, false>(dg, rblocks, st, (const double*)nullptr, A.n, A.ld, sign, Z,
                                       npad, A.d, stride);
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
