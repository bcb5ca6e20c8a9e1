// Gaussian sketch SA = S A (Section 4, first sketch family) on the BF16
// matrix cores.
//
// S = G16 / sqrt(m) where G16 is the BF16 rounding (through FP32) of the same
// N(0, 1) draws the FP64 sketch uses: a Gaussian matrix quantized to 8
// mantissa bits is still an i.i.d. zero-mean sub-Gaussian sketch, so the
// embedding argument of Section 4.1 is untouched.  A is split into three BF16
// terms (exact for FP32 storage, 24 bits for FP64), so S A is formed from
// three BF16 products with FP32 sums over at most kMaxSplitRows rows of A,
// added in FP64 (in registers across the K-loop, or across K-splits).  The
// remaining error (~1e-6 of sum |s||a|) perturbs the preconditioner only.
//
// Layout: XS[p][col][row] (three terms of A, rows contiguous, padded to a
// multiple of 64) and S16[row][k] (a chunk of sketch rows, same padding), so
// every 16-byte piece staged into LDS is one MFMA fragment: 8 consecutive k.
// Tile: 128 sketch rows x 128 columns of A per workgroup (four waves of
// 64 x 64), K-slices of 64 rows of A, next slice prefetched into registers.
#include "ops.hpp"

namespace ihs {

namespace {
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 128;
constexpr int kBK = 64;  // row padding of S16 and XS (a multiple of every slice depth)
constexpr int64_t kChunkBytes = int64_t(1) << 30;  // S16 rows generated at once
constexpr int64_t kPartDoubles = int64_t(2048) * kT * kT;  // split-K partials
}  // namespace

// S16[r][k] = BF16(FP32(z)) for sketch row r0 + r, column k < n (0 beyond n);
// z is the Box-Muller draw of entry (r0 + r, k) of the m x n Gaussian sketch.
__global__ __launch_bounds__(256) void gauss16_fill_kernel(uint64_t key, int64_t r0, int64_t rows,
                                                           int64_t n, int64_t npad,
                                                           __bf16* __restrict__ S) {
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
    const uint64_t q0 = (uint64_t)((r0 + r) * n);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npad;
         k += (int64_t)gridDim.x * blockDim.x) {
      float z = 0.0f;
      if (k < n) {
        const uint64_t q = q0 + (uint64_t)k;
        const uint64_t x1 = sm_draw(key, 2ull * q);
        const uint64_t x2 = sm_draw(key, 2ull * q + 1ull);
        const double u1 = ((double)(x1 >> 11) + 1.0) * 0x1.0p-53;
        const double u2 = (double)(x2 >> 11) * 0x1.0p-53;
        z = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2));
      }
      S[r * npad + k] = (__bf16)z;
    }
  }
}

// out[r][c] (+ split * strideo) = scale * sum_k S16[r][k] A[k][c] over this
// split's rows k, from the three terms in XS.  BK rows of A per slice (a
// multiple of 32; the split bounds are multiples of BK).
template <int BK>
__global__ __launch_bounds__(256) void sketch_bf16x3_kernel(const __bf16* __restrict__ S,
                                                            int64_t rows,
                                                            const __bf16* __restrict__ XS,
                                                            int64_t d, int64_t npad, int64_t k_per,
                                                            double scale, double* __restrict__ out,
                                                            int64_t ldo, int64_t strideo) {
  constexpr int kPitch = BK + 8;  // bf16 per LDS row (16-byte pad)
  constexpr int kQ = BK / 8;      // 16-byte pieces per row and slice
  constexpr int kPS = kT * kQ / 256, kPX = 3 * kT * kQ / 256;  // pieces per thread
  constexpr int kFlush = (int)(kMaxSplitRows / BK);  // slices per FP32 partial sum
  __shared__ __attribute__((aligned(16))) __bf16 Ss[kT][kPitch];
  __shared__ __attribute__((aligned(16))) __bf16 Xs[3][kT][kPitch];
  const int64_t n0 = (int64_t)blockIdx.x * kT, m0 = (int64_t)blockIdx.y * kT;
  const int sp = blockIdx.z;
  const int64_t kb = (int64_t)sp * k_per;
  const int64_t ke = kb + k_per < npad ? kb + k_per : npad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  const int64_t plane = d * npad;

  f32x4 acc[4][4];
  double acc64[4][4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
    }

  // per slice: 128 rows x kQ pieces of S, 3 terms x 128 columns x kQ pieces of A
  bf16x8 ps[kPS], px[kPX];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < kPS; ++e) {
      const int v = tid + 256 * e;
      const int row = v / kQ, q = v % kQ;
      if (m0 + row < rows) {
        ps[e] = *reinterpret_cast<const bf16x8*>(S + (m0 + row) * npad + k0 + 8 * q);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) ps[e][i] = (__bf16)0.0f;
      }
    }
#pragma unroll
    for (int e = 0; e < kPX; ++e) {
      const int v = tid + 256 * e;
      const int p = v / (kT * kQ), rem = v % (kT * kQ);
      const int cc = rem / kQ, q = rem % kQ;
      if (n0 + cc < d) {
        px[e] = *reinterpret_cast<const bf16x8*>(XS + p * plane + (n0 + cc) * npad + k0 + 8 * q);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) px[e][i] = (__bf16)0.0f;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < kPS; ++e) {
      const int v = tid + 256 * e;
      *reinterpret_cast<bf16x8*>(&Ss[v / kQ][8 * (v % kQ)]) = ps[e];
    }
#pragma unroll
    for (int e = 0; e < kPX; ++e) {
      const int v = tid + 256 * e;
      const int p = v / (kT * kQ), rem = v % (kT * kQ);
      *reinterpret_cast<bf16x8*>(&Xs[p][rem / kQ][8 * (rem % kQ)]) = px[e];
    }
  };
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
        acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
  };

  if (kb < ke) load(kb);
  int slice = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    store();
    __syncthreads();
    if (k0 + BK < ke) load(k0 + BK);
    const int r16 = lane & 15;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      const int kq = kk + 8 * (lane >> 4);
      bf16x8 af[4], bx[3][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        af[i] = *reinterpret_cast<const bf16x8*>(&Ss[wm + 16 * i + r16][kq]);
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          bx[p][j] = *reinterpret_cast<const bf16x8*>(&Xs[p][wn + 16 * j + r16][kq]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // smallest term first
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bx[2][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bx[1][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bx[0][j], acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
    if (++slice == kFlush) {
      flush();
      slice = 0;
    }
  }
  flush();

  double* O = out + (int64_t)sp * strideo;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int64_t gn = n0 + wn + 16 * j + (lane & 15);
        if (gm < rows && gn < d) O[gm * ldo + gn] = scale * acc64[i][j][r];
      }
}

namespace {
int64_t pad_rows(int64_t n) { return cdiv(n, kBK) * kBK; }
int64_t chunk_rows(int64_t m, int64_t npad) {
  int64_t rows = kChunkBytes / (2 * npad);
  rows = std::max<int64_t>(kT, (rows / kT) * kT);
  return std::min(rows, cdiv(m, kT) * kT);
}
}  // namespace

int64_t sketch_bf16_work_bytes(int64_t m, int64_t n, int64_t d) {
  const int64_t npad = pad_rows(n);
  return 3 * d * npad * 2 + 256 + chunk_rows(m, npad) * npad * 2;
}

int64_t gaussian_sketch_bf16_part_doubles(int64_t, int64_t, int64_t) { return kPartDoubles; }

void gaussian_sketch_bf16(const MatView& A, uint64_t seed, int64_t m, double* SA, void* work,
                          double* part, int64_t part_doubles, hipStream_t st, int64_t r_begin) {
  if (A.format != IHSBIN_DENSE) fail(IHSBIN_EUNSUP, "BF16 Gaussian sketch of a CSR matrix");
  const int64_t n = A.n, d = A.d, npad = pad_rows(n);
  char* base = static_cast<char*>(work);
  __bf16* XS = reinterpret_cast<__bf16*>(base);
  __bf16* S16 = reinterpret_cast<__bf16*>(base + ((3 * d * npad * 2 + 255) / 256) * 256);
  launch_split3_transpose(A.vals, A.dtype == IHSBIN_F32, n, d, A.ld, npad, XS, st);
  const int64_t rows = chunk_rows(m, npad);
  const double scale = 1.0 / std::sqrt((double)m);
  const uint64_t key = stream_key(seed, 3);
  const unsigned nt = (unsigned)cdiv(d, kT);
  if (nt > 65535u) fail(IHSBIN_EUNSUP, "sketch: too many columns");
  for (int64_t r0 = r_begin; r0 < m; r0 += rows) {
    const int64_t rn = std::min(rows, m - r0);
    {
      const unsigned gx = (unsigned)std::min<int64_t>(cdiv(npad, 256), 64);
      const unsigned gy = (unsigned)std::min<int64_t>(rn, 1024);
      hipLaunchKernelGGL(gauss16_fill_kernel, dim3(gx, gy), dim3(256), 0, st, key, r0, rn, n, npad,
                         S16);
      IHS_CHECK_LAUNCH();
    }
    const int64_t tiles = (int64_t)nt * cdiv(rn, kT);
    // K-splits only to fill the device when the tiles are few: every split
    // keeps at least 8 flush intervals of work and its partials fit `part`
    int64_t s = std::max<int64_t>(1, 2048 / tiles);
    s = std::min(s, std::max<int64_t>(1, npad / (8 * kMaxSplitRows)));
    s = std::min(s, std::max<int64_t>(1, part_doubles / (rn * d)));
    int64_t k_per = pad_rows(cdiv(npad, s));
    s = cdiv(npad, k_per);
    if (cdiv(rn, kT) > 65535 || s > 65535) fail(IHSBIN_EUNSUP, "sketch: grid too large");
    const dim3 grid(nt, (unsigned)cdiv(rn, kT), (unsigned)s);
    // 64 rows of A per slice: 32-row slices left the single wave per SIMD
    // waiting on its loads (140 vs 174 TFLOP/s FP64-equivalent at
    // 32768 x 262144 x 2048)
    auto launch = [&](dim3 gr, double* o, int64_t so) {
      hipLaunchKernelGGL(sketch_bf16x3_kernel<64>, gr, dim3(256), 0, st, S16, rn, XS, d, npad,
                         k_per, scale, o, d, so);
    };
    if (s == 1) {
      launch(grid, SA + r0 * d, (int64_t)0);
      IHS_CHECK_LAUNCH();
    } else {
      if (s * rn * d > part_doubles) fail(IHSBIN_EINVAL, "sketch: partial buffer too small");
      launch(grid, part, rn * d);
      IHS_CHECK_LAUNCH();
      reduce_splits(part, (int)s, 1, rn, d, d, rn * d, SA + r0 * d, d, 0, 1.0, 0.0, st);
    }
  }
}

}  // namespace ihs
