// Gaussian sketch SA = S A (Section 4, first sketch family) on the FP8 matrix
// cores (OCP e4m3: 1 sign, 4 exponent, 3 mantissa bits, largest 448).
//
// S = S8 / sqrt(m) where S8 = E4M3(FP32(z)) of the same N(0, 1) draws the FP64
// sketch uses: an i.i.d. zero-mean Gaussian quantized to 3 mantissa bits is
// still sub-Gaussian, so Section 4.1's embedding argument applies to it as a
// sketch of its own.  A is scaled per column by a power of two 2^e_c (the
// smallest e_c with max_k |a_kc| <= 448 2^e_c) and split into three e4m3
// terms, each the rounding of 16 times what the earlier ones leave:
//
//   a = 2^e_c (t0 + t1 / 16 + t2 / 256) + r,   |r| <= 448 2^(e_c - 12),
//
// i.e. about 12 significant bits relative to the column's largest entry (the
// preconditioner built from it is a fixed SPD operator: the path keeps its
// fixed point; a coarser P_S only shows as a slower rate, which the spectral
// probe measures).  S A is formed from three FP8 products on the scaled MFMA
// (the 1/16^p of term p is the E8M0 scale of the S operand), summed in two
// FP32 levels as in the BF16 form, and multiplied by 2^e_c / sqrt(m) in FP64.
//
// Layout: XT[p][col][row] (the terms, bytes, rows contiguous, padded to a
// multiple of 64) and S8[row][k] (a chunk of sketch rows, same padding), so
// every 32-byte run a lane feeds one MFMA is contiguous in LDS.  Tile: 256
// sketch rows x 128 columns of A per workgroup (eight waves of 64 x 64, each
// 2 x 2 MFMAs of 32 x 32 x 64), K-slices of 64 rows of A double-buffered.
#include "ops.hpp"

namespace ihs {

namespace {
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kTM = 256, kTN = 128;  // sketch rows x columns of A per workgroup
constexpr int kBK = 64;              // rows of A per slice (bytes per LDS row)
constexpr int kPitch = kBK + 16;     // LDS bytes per row
constexpr int kTerms = 3;
constexpr int64_t kChunkBytes = int64_t(1) << 30;  // S8 rows generated at once
constexpr int64_t kPartDoubles = int64_t(1024) * kTM * kTN;  // split-K partials
constexpr int64_t kMaxSecond = 128;  // first-level sums per second-level sum

int64_t pad_rows(int64_t n) { return cdiv(n, kBK) * kBK; }
int64_t chunk_rows(int64_t m, int64_t npad) {
  int64_t rows = kChunkBytes / npad;
  rows = std::max<int64_t>(kTM, (rows / kTM) * kTM);
  return std::min(rows, cdiv(m, kTM) * kTM);
}
int64_t min_splits(int64_t npad) { return cdiv(npad, kMaxSplitRows * kMaxSecond); }
int64_t xt_bytes(int64_t d, int64_t npad) { return cdiv(kTerms * d * npad, 256) * 256; }
}  // namespace

// E4M3 code of x: round to nearest, ties to the even code, saturating at
// 448 (no infinities in the format; NaN input is not expected).
__device__ inline uint32_t e4m3_code(float x) {
  const uint32_t sign = x < 0.0f ? 0x80u : 0u;
  float a = fabsf(x);
  uint32_t code;
  if (a < 0x1.0p-6f) {
    code = (uint32_t)rintf(a * 0x1.0p9f);  // subnormals: multiples of 2^-9 (8 -> 2^-6)
  } else {
    int e;
    const float f = frexpf(a, &e);  // a = f 2^e, f in [0.5, 1)
    uint32_t mant = (uint32_t)rintf((2.0f * f - 1.0f) * 8.0f);
    int be = e - 1 + 7;
    if (mant == 8) {
      mant = 0;
      ++be;
    }
    code = be > 15 ? 0x7Eu : ((uint32_t)be << 3) | mant;
    if (code > 0x7Eu) code = 0x7Eu;
  }
  return sign | code;
}

__device__ inline double e4m3_value(uint32_t c) {
  const int e = (c >> 3) & 15, m = c & 7;
  const double v = e == 0 ? ldexp((double)m, -9) : ldexp(8.0 + m, e - 10);
  return (c & 0x80u) ? -v : v;
}

__global__ __launch_bounds__(256) void zero_u64_kernel(unsigned long long* __restrict__ p,
                                                       int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
    p[i] = 0ull;
}

// S8[r][k] = E4M3(FP32(z)) for sketch row r0 + r, column k < n (0 beyond n),
// z from the Box-Muller pairs as for the BF16 sketch (one thread per pair
// slot of a row).  The FP32 form of z decides the code when the codes of
// z (1 - 2^-17), z and z (1 + 2^-17) agree (rounding is monotone, and the FP32
// form is within a few units of FP32(z)); otherwise the FP64 form does.
__global__ __launch_bounds__(256) void gauss8_fill_kernel(uint64_t key, int64_t r0, int64_t rows,
                                                          int64_t n, int64_t npad,
                                                          uint8_t* __restrict__ S) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
    const int64_t q0 = (r0 + r) * n, k0 = -(q0 & 1);
    const int64_t slots = (n - k0 + 1) / 2;
    uint8_t* row = S + r * npad;
    for (int64_t t = tid; t < slots; t += stride) {
      const int64_t k = k0 + 2 * t;
      const uint64_t p = (uint64_t)(q0 + k) >> 1;
      const uint64_t x1 = sm_draw(key, 2ull * p), x2 = sm_draw(key, 2ull * p + 1ull);
      float z[2];
      box_muller32(x1, x2, z[0], z[1]);
      uint32_t code[2];
      bool near = false;
      for (int h = 0; h < 2; ++h) {
        code[h] = e4m3_code(z[h]);
        near |= e4m3_code(z[h] * (1.0f - 0x1.0p-17f)) != code[h] ||
                e4m3_code(z[h] * (1.0f + 0x1.0p-17f)) != code[h];
      }
      if (near) {
        double zc, zs;
        box_muller64(x1, x2, zc, zs);
        code[0] = e4m3_code((float)zc);
        code[1] = e4m3_code((float)zs);
      }
      if (k >= 0) row[k] = (uint8_t)code[0];
      if (k + 1 < n) row[k + 1] = (uint8_t)code[1];
    }
    for (int64_t k = n + tid; k < npad; k += stride) row[k] = 0;
  }
}

// colmax[c] = bits of max_k |A[k][c]| as a nonnegative double (max over
// unsigned integers of the bits: order-independent).
template <typename T>
__global__ __launch_bounds__(256) void col_absmax_kernel(const T* __restrict__ A, int64_t n,
                                                         int64_t d, int64_t lda,
                                                         unsigned long long* __restrict__ colmax) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= d) return;
  double mx = 0.0;
  for (int64_t k = blockIdx.y; k < n; k += gridDim.y) mx = fmax(mx, fabs((double)A[k * lda + c]));
  atomicMax(colmax + c, (unsigned long long)__double_as_longlong(mx));
}

// e_c = the smallest e with max |a_c| <= 448 2^e (0 for a zero column, and
// for a column holding an infinity or NaN, whose terms are then meaningless
// but finite: the loops below stop only for finite maxima).
__device__ inline int col_exponent(double mx) {
  if (!(mx > 0.0) || isinf(mx)) return 0;
  int e = ilogb(mx) - 8;
  while (mx > ldexp(448.0, e)) ++e;
  while (mx <= ldexp(448.0, e - 1)) --e;
  return e;
}

__global__ __launch_bounds__(256) void col_exponent_kernel(const unsigned long long* __restrict__ colmax,
                                                           int64_t d, int32_t* __restrict__ ex) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c < d) ex[c] = col_exponent(__longlong_as_double((long long)colmax[c]));
}

// XT[p][c][k] = term p of A[k][c] 2^-e_c; rows k >= n are zero (32 x 32 tiles
// via LDS; the row tiles are strided over gridDim.y).
template <typename T>
__global__ __launch_bounds__(256) void fp8_split_transpose_kernel(const T* __restrict__ A, int64_t n,
                                                                  int64_t d, int64_t lda,
                                                                  int64_t npad,
                                                                  const int32_t* __restrict__ ex,
                                                                  uint8_t* __restrict__ XT) {
  __shared__ double tile[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int64_t k0 = (int64_t)blockIdx.y * 32; k0 < npad; k0 += (int64_t)gridDim.y * 32) {
    for (int r = ty; r < 32; r += 8) {
      const int64_t k = k0 + r, c = c0 + tx;
      tile[r][tx] = (k < n && c < d) ? (double)A[k * lda + c] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int64_t c = c0 + r, k = k0 + tx;
      if (c < d) {
        double res = ldexp(tile[tx][r], -ex[c]);
        const int64_t o = c * npad + k;
#pragma unroll
        for (int p = 0; p < kTerms; ++p) {
          const uint32_t code = e4m3_code((float)res);
          XT[p * d * npad + o] = (uint8_t)code;
          res = (res - e4m3_value(code)) * 16.0;
        }
      }
    }
    __syncthreads();
  }
}

// out[r][c] (+ split * strideo) = scale 2^e_c sum_k S8[r][k] A~[k][c] over
// this split's rows k (A~ = the three terms), a 256 x 128 tile per workgroup
// of eight waves; sums in two FP32 levels (every kMaxSplitRows rows the
// running sum goes into a second FP32 tile); slices alternate between two
// LDS buffers with one barrier per slice.
__global__ __launch_bounds__(512) void sketch_fp8_kernel(const uint8_t* __restrict__ S,
                                                         int64_t rows,
                                                         const uint8_t* __restrict__ XT,
                                                         int64_t d, int64_t npad, int64_t k_per,
                                                         const int32_t* __restrict__ ex,
                                                         double scale, double* __restrict__ out,
                                                         int64_t ldo, int64_t strideo) {
  constexpr int kQ = kBK / 16;                                     // 16-byte pieces per row
  constexpr int kPS = kTM * kQ / 512, kPX = kTerms * kTN * kQ / 512;  // pieces per thread
  constexpr int kFlush = (int)(kMaxSplitRows / kBK);
  __shared__ __attribute__((aligned(16))) uint8_t Ss[2][kTM][kPitch];
  __shared__ __attribute__((aligned(16))) uint8_t Xs[2][kTerms][kTN][kPitch];
  const int64_t n0 = (int64_t)blockIdx.x * kTN, m0 = (int64_t)blockIdx.y * kTM;
  const int sp = blockIdx.z;
  const int64_t kb = (int64_t)sp * k_per;
  const int64_t ke = kb + k_per < npad ? kb + k_per : npad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 3) * 64, wn = (wave >> 2) * 64;
  const int64_t plane = d * npad;

  f32x16 acc[2][2], acc2[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        acc[i][j][r] = 0.0f;
        acc2[i][j][r] = 0.0f;
      }

  uint4 ps[kPS], px[kPX];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < kPS; ++e) {
      const int v = tid + 512 * e;
      const int row = v / kQ, q = v % kQ;
      ps[e] = m0 + row < rows
                  ? *reinterpret_cast<const uint4*>(S + (m0 + row) * npad + k0 + 16 * q)
                  : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int e = 0; e < kPX; ++e) {
      const int v = tid + 512 * e;
      const int p = v / (kTN * kQ), rem = v % (kTN * kQ);
      const int cc = rem / kQ, q = rem % kQ;
      px[e] = n0 + cc < d
                  ? *reinterpret_cast<const uint4*>(XT + p * plane + (n0 + cc) * npad + k0 + 16 * q)
                  : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int e = 0; e < kPS; ++e) {
      const int v = tid + 512 * e;
      *reinterpret_cast<uint4*>(&Ss[b][v / kQ][16 * (v % kQ)]) = ps[e];
    }
#pragma unroll
    for (int e = 0; e < kPX; ++e) {
      const int v = tid + 512 * e;
      const int p = v / (kTN * kQ), rem = v % (kTN * kQ);
      *reinterpret_cast<uint4*>(&Xs[b][p][rem / kQ][16 * (rem % kQ)]) = px[e];
    }
  };
  auto frag = [](const uint8_t* src) {
    const uint4 lo = *reinterpret_cast<const uint4*>(src);
    const uint4 hi = *reinterpret_cast<const uint4*>(src + 16);
    i32x8 f;
    f[0] = (int)lo.x; f[1] = (int)lo.y; f[2] = (int)lo.z; f[3] = (int)lo.w;
    f[4] = (int)hi.x; f[5] = (int)hi.y; f[6] = (int)hi.z; f[7] = (int)hi.w;
    return f;
  };
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc2[i][j] += acc[i][j];
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
      }
  };

  if (kb < ke) {
    load(kb);
    store(0);
  }
  __syncthreads();
  int slice = 0, buf = 0;
  const int r32 = lane & 31, kh = 32 * (lane >> 5);
  for (int64_t k0 = kb; k0 < ke; k0 += kBK) {
    const bool more = k0 + kBK < ke;
    if (more) load(k0 + kBK);
    i32x8 af[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) af[i] = frag(&Ss[buf][wm + 32 * i + r32][kh]);
#pragma unroll
    for (int p = kTerms - 1; p >= 0; --p) {  // smallest term first
      i32x8 bx[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) bx[j] = frag(&Xs[buf][p][wn + 32 * j + r32][kh]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
              af[i], bx[j], acc[i][j], 0, 0, 0, 127 - 4 * p, 0, 127);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    if (++slice == kFlush) {
      flush();
      slice = 0;
    }
  }
  flush();

  double* O = out + (int64_t)sp * strideo;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int64_t gn = n0 + wn + 32 * j + r32;
    if (gn >= d) continue;
    const double cs = ldexp(scale, ex[gn]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gm = m0 + wm + 32 * i + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
        if (gm < rows) O[gm * ldo + gn] = cs * (double)acc2[i][j][r];
      }
  }
}

int64_t sketch_fp8_work_bytes(int64_t m, int64_t n, int64_t d) {
  const int64_t npad = pad_rows(n);
  return xt_bytes(d, npad) + cdiv(chunk_rows(m, npad) * npad, 256) * 256 + 8 * d + 4 * d + 512;
}

int64_t gaussian_sketch_fp8_part_doubles(int64_t m, int64_t n, int64_t d) {
  const int64_t npad = pad_rows(n), s = min_splits(npad);
  return s > 1 ? std::max(kPartDoubles, s * chunk_rows(m, npad) * d) : kPartDoubles;
}

void gaussian_sketch_fp8(const MatView& A, uint64_t seed, int64_t m, double* SA, void* work,
                         double* part, int64_t part_doubles, hipStream_t st, int64_t r_begin) {
  if (A.format != IHSBIN_DENSE) fail(IHSBIN_EUNSUP, "FP8 Gaussian sketch of a CSR matrix");
  const int64_t n = A.n, d = A.d, npad = pad_rows(n);
  const int64_t rows = chunk_rows(m, npad);
  char* base = static_cast<char*>(work);
  uint8_t* XT = reinterpret_cast<uint8_t*>(base);
  uint8_t* S8 = reinterpret_cast<uint8_t*>(base + xt_bytes(d, npad));
  char* tail = base + xt_bytes(d, npad) + cdiv(rows * npad, 256) * 256;
  unsigned long long* colmax = reinterpret_cast<unsigned long long*>(tail);
  int32_t* ex = reinterpret_cast<int32_t*>(tail + 8 * d);
  const unsigned gc = (unsigned)cdiv(d, 256);
  const bool f32 = A.dtype == IHSBIN_F32;
  {
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)std::min<int64_t>(gc, 4096)), dim3(256), 0,
                       st, colmax, d);
    IHS_CHECK_LAUNCH();
    const unsigned gy = (unsigned)std::min<int64_t>(n, 512);
    if (f32)
      hipLaunchKernelGGL(col_absmax_kernel<float>, dim3(gc, gy), dim3(256), 0, st,
                         static_cast<const float*>(A.vals), n, d, A.ld, colmax);
    else
      hipLaunchKernelGGL(col_absmax_kernel<double>, dim3(gc, gy), dim3(256), 0, st,
                         static_cast<const double*>(A.vals), n, d, A.ld, colmax);
    IHS_CHECK_LAUNCH();
    hipLaunchKernelGGL(col_exponent_kernel, dim3(gc), dim3(256), 0, st, colmax, d, ex);
    IHS_CHECK_LAUNCH();
    const unsigned gx = (unsigned)cdiv(d, 32);
    const unsigned gs = (unsigned)std::min<int64_t>(cdiv(npad, 32), 32768);
    if (gx > 65535u) fail(IHSBIN_EUNSUP, "sketch: too many columns");
    if (f32)
      hipLaunchKernelGGL(fp8_split_transpose_kernel<float>, dim3(gx, gs), dim3(256), 0, st,
                         static_cast<const float*>(A.vals), n, d, A.ld, npad, ex, XT);
    else
      hipLaunchKernelGGL(fp8_split_transpose_kernel<double>, dim3(gx, gs), dim3(256), 0, st,
                         static_cast<const double*>(A.vals), n, d, A.ld, npad, ex, XT);
    IHS_CHECK_LAUNCH();
  }
  const double scale = 1.0 / std::sqrt((double)m);
  const uint64_t key = stream_key(seed, 3);
  const unsigned nt = (unsigned)cdiv(d, kTN);
  if (nt > 65535u) fail(IHSBIN_EUNSUP, "sketch: too many columns");
  for (int64_t r0 = r_begin; r0 < m; r0 += rows) {
    const int64_t rn = std::min(rows, m - r0);
    {
      const unsigned gx = (unsigned)std::min<int64_t>(cdiv(npad / 2 + 1, 256), 64);
      const unsigned gy = (unsigned)std::min<int64_t>(rn, 1024);
      hipLaunchKernelGGL(gauss8_fill_kernel, dim3(gx, gy), dim3(256), 0, st, key, r0, rn, n, npad,
                         S8);
      IHS_CHECK_LAUNCH();
    }
    const int64_t tiles = (int64_t)nt * cdiv(rn, kTM);
    // K-splits as the sums need them, and more to fill the device when the
    // tiles are few (each of those keeps at least 8 first-level sums of work
    // and their partials fit `part`)
    const int64_t s_min = min_splits(npad);
    int64_t s = std::max<int64_t>(s_min, 1024 / tiles);
    s = std::min(s, std::max<int64_t>(s_min, npad / (8 * kMaxSplitRows)));
    s = std::min(s, std::max<int64_t>(s_min, part_doubles / (rn * d)));
    const int64_t k_per = pad_rows(cdiv(npad, s));
    s = cdiv(npad, k_per);
    if (k_per > kMaxSplitRows * kMaxSecond) fail(IHSBIN_EINVAL, "sketch: split too long");
    if (cdiv(rn, kTM) > 65535 || s > 65535) fail(IHSBIN_EUNSUP, "sketch: grid too large");
    const dim3 grid(nt, (unsigned)cdiv(rn, kTM), (unsigned)s);
    if (s == 1) {
      hipLaunchKernelGGL(sketch_fp8_kernel, grid, dim3(512), 0, st, S8, rn, XT, d, npad, k_per, ex,
                         scale, SA + r0 * d, d, (int64_t)0);
      IHS_CHECK_LAUNCH();
    } else {
      if (s * rn * d > part_doubles) fail(IHSBIN_EINVAL, "sketch: partial buffer too small");
      hipLaunchKernelGGL(sketch_fp8_kernel, grid, dim3(512), 0, st, S8, rn, XT, d, npad, k_per, ex,
                         scale, part, d, rn * d);
      IHS_CHECK_LAUNCH();
      reduce_splits(part, (int)s, 1, rn, d, d, rn * d, SA + r0 * d, d, 0, 1.0, 0.0, st);
    }
  }
}

}  // namespace ihs
