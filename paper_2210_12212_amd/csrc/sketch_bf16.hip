// Gaussian sketch SA = S A (Section 4, first sketch family) on the BF16
// matrix cores.
//
// S = G16 / sqrt(m) where G16 is the BF16 rounding (through FP32) of the same
// N(0, 1) draws the FP64 sketch uses: a Gaussian matrix quantized to 8
// mantissa bits is still an i.i.d. zero-mean sub-Gaussian sketch, so the
// embedding argument of Section 4.1 is untouched.  A is split into two BF16
// terms a = a0 + a1 + r with |r| <= 2^-18 |a|, so S A is formed from two BF16
// products (exact in FP32) summed in two FP32 levels: sums over at most
// kMaxSplitRows rows of A, at most 128 of those added into a second FP32 sum,
// and K-splits beyond that added in FP64.  The dropped r is of the order of
// what the FP32 sums lose; together they stay within 2e-5 of sum |s||a| per
// entry and perturb the preconditioner only.
//
// Layout: XS[p][col][row] (the terms of A, rows contiguous, padded to a
// multiple of 64) and S16[row][k] (a chunk of sketch rows, same padding), so
// every 16-byte piece staged into LDS is one MFMA fragment: 8 consecutive k.
// Tile: 256 sketch rows x 128 columns of A per workgroup (eight waves of
// 64 x 64, two per SIMD), K-slices of 64 rows of A, next slice prefetched
// into registers and stored into the other of two LDS buffers.
#include "ops.hpp"

namespace ihs {

namespace {
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 256, kTN = 128;  // sketch rows x columns of A per workgroup
constexpr int kBK = 64;  // row padding of S16 and XS (a multiple of every slice depth)
constexpr int64_t kChunkBytes = int64_t(1) << 30;  // S16 rows generated at once
constexpr int64_t kPartDoubles = int64_t(1024) * kTM * kTN;  // split-K partials
constexpr int kTerms = 2;  // BF16 terms of A
}  // namespace

// S16[r][k] = BF16(FP32(z)) for sketch row r0 + r, column k < n (0 beyond n);
// z is entry q = (r0 + r) n + k of the Gaussian stream, from its Box-Muller
// pair (q / 2).  One thread per pair slot of a row: slot t holds columns
// k = k0 + 2t and k + 1, k0 = -1 when the row starts on an odd entry (halves
// outside the row are not written).  The FP32 form decides the rounding
// unless it lies within 64 FP32 units of a BF16 rounding tie, where the FP64
// form does (the FP32 error is a few units).
__global__ __launch_bounds__(256) void gauss16_fill_kernel(uint64_t key, int64_t r0, int64_t rows,
                                                           int64_t n, int64_t npad,
                                                           __bf16* __restrict__ S) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
    const int64_t q0 = (r0 + r) * n, k0 = -(q0 & 1);
    const int64_t slots = (n - k0 + 1) / 2;
    __bf16* row = S + r * npad;
    for (int64_t t = tid; t < slots; t += stride) {
      const int64_t k = k0 + 2 * t;
      const uint64_t p = (uint64_t)(q0 + k) >> 1;
      const uint64_t x1 = sm_draw(key, 2ull * p), x2 = sm_draw(key, 2ull * p + 1ull);
      float z[2];
      box_muller32(x1, x2, z[0], z[1]);
      bool near = false;
      for (int h = 0; h < 2; ++h) {
        const uint32_t low = __float_as_uint(z[h]) & 0xFFFFu;
        near |= low > 0x8000u - 64u && low < 0x8000u + 64u;
      }
      if (near) {
        double zc, zs;
        box_muller64(x1, x2, zc, zs);
        z[0] = (float)zc;
        z[1] = (float)zs;
      }
      if (k >= 0) row[k] = (__bf16)z[0];
      if (k + 1 < n) row[k + 1] = (__bf16)z[1];
    }
    for (int64_t k = n + tid; k < npad; k += stride) row[k] = (__bf16)0.0f;
  }
}

// out[r][c] (+ split * strideo) = scale * sum_k S16[r][k] A[k][c] over this
// split's rows k, from the NT terms in XS: a 256 x 128 tile per workgroup of
// eight waves (4 x 2 waves of 64 x 64).  BK rows of A per slice (a multiple of
// 32; the split bounds are multiples of BK).  Sums in two FP32 levels: every
// kMaxSplitRows rows the running tile sum is added into a second FP32 tile
// and restarted, which keeps two waves per SIMD (an FP64 second level does
// not fit).  The slices alternate between two LDS buffers: slice t + 1 is
// stored while slice t's products are still in the matrix cores, and one
// barrier per slice orders both.
template <int BK, int NT>
__global__ __launch_bounds__(512) void sketch_bf16_kernel(const __bf16* __restrict__ S,
                                                          int64_t rows,
                                                          const __bf16* __restrict__ XS,
                                                          int64_t d, int64_t npad, int64_t k_per,
                                                          double scale, double* __restrict__ out,
                                                          int64_t ldo, int64_t strideo) {
  constexpr int kPitch = BK + 8;  // bf16 per LDS row (16-byte pad)
  constexpr int kQ = BK / 8;      // 16-byte pieces per row and slice
  constexpr int kPS = kTM * kQ / 512, kPX = NT * kTN * kQ / 512;  // pieces per thread
  constexpr int kFlush = (int)(kMaxSplitRows / BK);  // slices per first-level sum
  __shared__ __attribute__((aligned(16))) __bf16 Ss[2][kTM][kPitch];
  __shared__ __attribute__((aligned(16))) __bf16 Xs[2][NT][kTN][kPitch];
  const int64_t n0 = (int64_t)blockIdx.x * kTN, m0 = (int64_t)blockIdx.y * kTM;
  const int sp = blockIdx.z;
  const int64_t kb = (int64_t)sp * k_per;
  const int64_t ke = kb + k_per < npad ? kb + k_per : npad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 3) * 64, wn = (wave >> 2) * 64;
  const int64_t plane = d * npad;

  f32x4 acc[4][4], acc2[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc2[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

  // per slice: 256 rows x kQ pieces of S, NT terms x 128 columns x kQ pieces of A
  bf16x8 ps[kPS], px[kPX];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < kPS; ++e) {
      const int v = tid + 512 * e;
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
      const int v = tid + 512 * e;
      const int p = v / (kTN * kQ), rem = v % (kTN * kQ);
      const int cc = rem / kQ, q = rem % kQ;
      if (n0 + cc < d) {
        px[e] = *reinterpret_cast<const bf16x8*>(XS + p * plane + (n0 + cc) * npad + k0 + 8 * q);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) px[e][i] = (__bf16)0.0f;
      }
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int e = 0; e < kPS; ++e) {
      const int v = tid + 512 * e;
      *reinterpret_cast<bf16x8*>(&Ss[b][v / kQ][8 * (v % kQ)]) = ps[e];
    }
#pragma unroll
    for (int e = 0; e < kPX; ++e) {
      const int v = tid + 512 * e;
      const int p = v / (kTN * kQ), rem = v % (kTN * kQ);
      *reinterpret_cast<bf16x8*>(&Xs[b][p][rem / kQ][8 * (rem % kQ)]) = px[e];
    }
  };
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc2[i][j] += acc[i][j];
        acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
  };

  if (kb < ke) {
    load(kb);
    store(0);
  }
  __syncthreads();
  int slice = 0, buf = 0;
  const int r16 = lane & 15;
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    const bool more = k0 + BK < ke;
    if (more) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      const int kq = kk + 8 * (lane >> 4);
      bf16x8 af[4], bx[NT][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        af[i] = *reinterpret_cast<const bf16x8*>(&Ss[buf][wm + 16 * i + r16][kq]);
#pragma unroll
      for (int p = 0; p < NT; ++p)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          bx[p][j] = *reinterpret_cast<const bf16x8*>(&Xs[buf][p][wn + 16 * j + r16][kq]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int p = NT - 1; p >= 0; --p)  // smallest term first
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bx[p][j], acc[i][j], 0, 0, 0);
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
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int64_t gn = n0 + wn + 16 * j + (lane & 15);
        if (gm < rows && gn < d) O[gm * ldo + gn] = scale * (double)acc2[i][j][r];
      }
}

namespace {
int64_t pad_rows(int64_t n) { return cdiv(n, kBK) * kBK; }
int64_t chunk_rows(int64_t m, int64_t npad) {
  int64_t rows = kChunkBytes / (2 * npad);
  rows = std::max<int64_t>(kTM, (rows / kTM) * kTM);
  return std::min(rows, cdiv(m, kTM) * kTM);
}
}  // namespace

int64_t sketch_bf16_work_bytes(int64_t m, int64_t n, int64_t d) {
  const int64_t npad = pad_rows(n);
  return kTerms * d * npad * 2 + 256 + chunk_rows(m, npad) * npad * 2;
}

namespace {
// K-splits that every sketch of n rows needs: a split's second-level FP32 sum
// adds at most kMaxSecond first-level sums
constexpr int64_t kMaxSecond = 128;
int64_t min_splits(int64_t npad) { return cdiv(npad, kMaxSplitRows * kMaxSecond); }
}  // namespace

int64_t gaussian_sketch_bf16_part_doubles(int64_t m, int64_t n, int64_t d) {
  const int64_t npad = pad_rows(n), s = min_splits(npad);
  return s > 1 ? std::max(kPartDoubles, s * chunk_rows(m, npad) * d) : kPartDoubles;
}

void gaussian_sketch_bf16(const MatView& A, uint64_t seed, int64_t m, double* SA, void* work,
                          double* part, int64_t part_doubles, hipStream_t st, int64_t r_begin) {
  if (A.format != IHSBIN_DENSE) fail(IHSBIN_EUNSUP, "BF16 Gaussian sketch of a CSR matrix");
  const int64_t n = A.n, d = A.d, npad = pad_rows(n);
  char* base = static_cast<char*>(work);
  __bf16* XS = reinterpret_cast<__bf16*>(base);
  __bf16* S16 = reinterpret_cast<__bf16*>(base + ((kTerms * d * npad * 2 + 255) / 256) * 256);
  launch_split_transpose(A.vals, A.dtype == IHSBIN_F32, n, d, A.ld, npad, XS, kTerms, st);
  const int64_t rows = chunk_rows(m, npad);
  const double scale = 1.0 / std::sqrt((double)m);
  const uint64_t key = stream_key(seed, 3);
  const unsigned nt = (unsigned)cdiv(d, kTN);
  if (nt > 65535u) fail(IHSBIN_EUNSUP, "sketch: too many columns");
  for (int64_t r0 = r_begin; r0 < m; r0 += rows) {
    const int64_t rn = std::min(rows, m - r0);
    {
      const unsigned gx = (unsigned)std::min<int64_t>(cdiv(npad / 2 + 1, 256), 64);
      const unsigned gy = (unsigned)std::min<int64_t>(rn, 1024);
      hipLaunchKernelGGL(gauss16_fill_kernel, dim3(gx, gy), dim3(256), 0, st, key, r0, rn, n, npad,
                         S16);
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
    int64_t k_per = pad_rows(cdiv(npad, s));
    s = cdiv(npad, k_per);
    if (k_per > kMaxSplitRows * kMaxSecond) fail(IHSBIN_EINVAL, "sketch: split too long");
    if (cdiv(rn, kTM) > 65535 || s > 65535) fail(IHSBIN_EUNSUP, "sketch: grid too large");
    const dim3 grid(nt, (unsigned)cdiv(rn, kTM), (unsigned)s);
    auto launch = [&](dim3 gr, double* o, int64_t so) {
      hipLaunchKernelGGL((sketch_bf16_kernel<64, kTerms>), gr, dim3(512), 0, st, S16, rn, XS, d,
                         npad, k_per, scale, o, d, so);
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
