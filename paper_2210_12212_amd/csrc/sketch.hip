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
    if (left > 9 && left < 18) take = (left + 1) / 2;
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
