// Sketched Gram G = X^T X (X = SA, m x d FP64) on the BF16 matrix cores.
//
// Every FP64 entry is split into three BF16 terms x = x0 + x1 + x2 (each the
// round-to-nearest BF16 of what the previous terms leave; the remainders are
// exact in FP64), which carry 24 significant bits.  A product of two entries
// is taken as the six term products with i + j <= 2, accumulated in FP32 by
// v_mfma_f32_16x16x32_bf16; the dropped terms are below 2^-24 relative.  Each
// workgroup covers one K range (split-K), so an FP32 sum runs over at most
// kMaxSplitRows rows before the split partials are added in FP64.
//
// The preconditioner only has to be a fixed SPD operator: a Gram accurate to
// ~1e-6 relative changes (SA)^T SA + lam0 I by far less than lam0 on the
// configured workloads, so the convergence rate is unchanged, and the IHS
// recursion, which uses the same factor everywhere, keeps its fixed point.
//
// A first pass splits X once and stores the three terms transposed,
// XS[p][col][row] (rows contiguous, padded to a multiple of 32), so the
// product kernel stages 16-byte pieces straight into LDS, where each MFMA
// fragment (8 consecutive rows of one column) is one 16-byte read.
// Tile: 128 x 128 of G per workgroup (four waves, 64 x 64 each: 4 x 4 blocks
// of 16 x 16), K-slices of 32 rows of X.  Only tiles touching the lower
// triangle are computed.
#include "gemm.hpp"
#include "ops.hpp"

namespace ihs {

namespace {
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 128;          // tile edge
constexpr int kBK = 32;          // rows of X per slice
constexpr int kPitch = kBK + 8;  // bf16 per LDS row (16-byte pad)

__device__ __forceinline__ void split3(double x, __bf16& a, __bf16& b, __bf16& c) {
  a = (__bf16)(float)x;
  const double r1 = x - (double)(float)a;
  b = (__bf16)(float)r1;
  const double r2 = r1 - (double)(float)b;
  c = (__bf16)(float)r2;
}
}  // namespace

// XS[p][c][k] = term p < NT of X[k][c]; rows k >= m are zero (32 x 32 tiles
// via LDS; the row tiles are strided over gridDim.y).  Three terms split an
// FP32 input exactly.
template <typename T, int NT>
__global__ __launch_bounds__(256) void split_transpose_kernel(const T* __restrict__ X, int64_t m,
                                                              int64_t d, int64_t ldx, int64_t mpad,
                                                              __bf16* __restrict__ XS) {
  __shared__ double tile[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int64_t k0 = (int64_t)blockIdx.y * 32; k0 < mpad; k0 += (int64_t)gridDim.y * 32) {
    for (int r = ty; r < 32; r += 8) {
      const int64_t k = k0 + r, c = c0 + tx;
      tile[r][tx] = (k < m && c < d) ? (double)X[k * ldx + c] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int64_t c = c0 + r, k = k0 + tx;
      if (c < d) {
        __bf16 a, b, e;
        split3(tile[tx][r], a, b, e);
        const int64_t o = c * mpad + k;
        XS[o] = a;
        XS[d * mpad + o] = b;
        if (NT == 3) XS[2 * d * mpad + o] = e;
      }
    }
    __syncthreads();
  }
}

void launch_split_transpose(const void* X, bool f32, int64_t m, int64_t d, int64_t ldx,
                            int64_t mpad, void* XS, int terms, hipStream_t st) {
  if (m <= 0 || d <= 0) return;
  if (terms != 2 && terms != 3) fail(IHSBIN_EINVAL, "split: 2 or 3 terms");
  const unsigned gx = (unsigned)cdiv(d, 32);
  const unsigned gy = (unsigned)std::min<int64_t>(cdiv(mpad, 32), 32768);
  if (gx > 65535u) fail(IHSBIN_EUNSUP, "split: too many columns");
  __bf16* out = static_cast<__bf16*>(XS);
  if (f32 && terms == 3)
    hipLaunchKernelGGL((split_transpose_kernel<float, 3>), dim3(gx, gy), dim3(256), 0, st,
                       static_cast<const float*>(X), m, d, ldx, mpad, out);
  else if (f32)
    hipLaunchKernelGGL((split_transpose_kernel<float, 2>), dim3(gx, gy), dim3(256), 0, st,
                       static_cast<const float*>(X), m, d, ldx, mpad, out);
  else if (terms == 3)
    hipLaunchKernelGGL((split_transpose_kernel<double, 3>), dim3(gx, gy), dim3(256), 0, st,
                       static_cast<const double*>(X), m, d, ldx, mpad, out);
  else
    hipLaunchKernelGGL((split_transpose_kernel<double, 2>), dim3(gx, gy), dim3(256), 0, st,
                       static_cast<const double*>(X), m, d, ldx, mpad, out);
  IHS_CHECK_LAUNCH();
}

__global__ __launch_bounds__(256) void gram_bf16x3_kernel(const __bf16* __restrict__ XS,
                                                          int64_t mpad, int64_t d,
                                                          int64_t rows_per,
                                                          double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) __bf16 As[3][kT][kPitch];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[3][kT][kPitch];
  const int64_t m0 = (int64_t)blockIdx.y * kT, n0 = (int64_t)blockIdx.x * kT;
  if (n0 > m0 + kT - 1) return;  // strictly upper tile
  const int sp = blockIdx.z;
  const int64_t kb = (int64_t)sp * rows_per;
  const int64_t ke = kb + rows_per < mpad ? kb + rows_per : mpad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  const bool diag = m0 == n0;
  const int64_t plane = d * mpad;

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // 3 terms x 128 columns x 4 pieces of 8 rows = 1536 pieces, 6 per thread;
  // the next slice's pieces are loaded into registers while the matrix cores
  // work on the current one
  bf16x8 pa[6], pb[6];
  auto load = [&](bf16x8 (&pr)[6], int64_t col0, int64_t k0) {
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int v = tid + 256 * e;
      const int p = v / (kT * 4), rem = v % (kT * 4);
      const int cc = rem >> 2, q = rem & 3;
      const int64_t col = col0 + cc;
      if (col < d) {
        pr[e] = *reinterpret_cast<const bf16x8*>(XS + p * plane + col * mpad + k0 + 8 * q);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) pr[e][i] = (__bf16)0.0f;
      }
    }
  };
  auto store = [&](__bf16 (*S)[kT][kPitch], const bf16x8 (&pr)[6]) {
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int v = tid + 256 * e;
      const int p = v / (kT * 4), rem = v % (kT * 4);
      const int cc = rem >> 2, q = rem & 3;
      *reinterpret_cast<bf16x8*>(&S[p][cc][8 * q]) = pr[e];
    }
  };

  if (kb < ke) {
    load(pa, m0, kb);
    if (!diag) load(pb, n0, kb);
  }
  for (int64_t k0 = kb; k0 < ke; k0 += kBK) {
    store(As, pa);
    if (!diag) store(Bs, pb);
    __syncthreads();
    if (k0 + kBK < ke) {
      load(pa, m0, k0 + kBK);
      if (!diag) load(pb, n0, k0 + kBK);
    }
    const __bf16 (*BsR)[kT][kPitch] = diag ? As : Bs;
    const int r16 = lane & 15, kq = 8 * (lane >> 4);
    bf16x8 af[3][4], bf[3][4];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        af[p][i] = *reinterpret_cast<const bf16x8*>(&As[p][wm + 16 * i + r16][kq]);
        bf[p][i] = *reinterpret_cast<const bf16x8*>(&BsR[p][wn + 16 * i + r16][kq]);
      }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // smallest terms first
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bf[2][j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bf[1][j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2][i], bf[0][j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bf[1][j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bf[0][j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bf[0][j], acc[i][j], 0, 0, 0);
      }
    __syncthreads();
  }

  double* P = part + (int64_t)sp * d * d;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int64_t gn = n0 + wn + 16 * j + (lane & 15);
        if (gm < d && gn < d) P[gm * d + gn] = (double)acc[i][j][r];
      }
}

int gram_bf16x3_splits(int64_t m) { return (int)cdiv(m, kMaxSplitRows); }
int64_t gram_bf16x3_work_bytes(int64_t m, int64_t d) {
  return 3 * d * (cdiv(m, kBK) * kBK) * (int64_t)sizeof(__bf16);
}

void gram_bf16x3(const double* X, int64_t m, int64_t d, int64_t ldx, void* work, double* part,
                 int splits, hipStream_t st) {
  if (m <= 0 || d <= 0) return;
  const int64_t mpad = cdiv(m, kBK) * kBK;
  __bf16* XS = static_cast<__bf16*>(work);
  launch_split_transpose(X, false, m, d, ldx, mpad, XS, 3, st);
  int64_t rows_per = cdiv(mpad, splits);
  rows_per = cdiv(rows_per, kBK) * kBK;
  const unsigned nt = (unsigned)cdiv(d, kT);
  if (nt > 65535u || splits > 65535) fail(IHSBIN_EUNSUP, "gram: grid too large");
  hipLaunchKernelGGL(gram_bf16x3_kernel, dim3(nt, nt, (unsigned)splits), dim3(256), 0, st, XS,
                     mpad, d, rows_per, part);
  IHS_CHECK_LAUNCH();
}

}  // namespace ihs
