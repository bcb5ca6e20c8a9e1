// FP64 GEMM on MFMA for gfx950.
//
// A 256-thread workgroup (four wave64s) computes a BM x BN tile of C; each
// wave owns a (BM/WM) x (BN/WN) sub-tile made of 16x16 accumulators fed by
// v_mfma_f64_16x16x4f64.  Operands are staged through LDS in K-slices of 16,
// stored K-major (As[k][m], Bs[k][n]) whatever the global layout, so one
// inner loop serves every transpose case.  FP32 operands are widened to FP64
// as they are staged (exact).  The next K-slice is prefetched into registers
// while the matrix cores work on the current one.
//
// Fragment layout of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register r of lane l
// holds D[4 r + l / 16][l % 16].
#include "gemm.hpp"

namespace ihs {

typedef double v4d __attribute__((ext_vector_type(4)));

template <typename TA, typename TB, bool TRA, bool TRB, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(256) void gemm_f64_kernel(Gemm g) {
  constexpr int BK = 16;
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  constexpr int AE = BM * BK / 256;
  constexpr int BE = (BK * BN + 255) / 256;
  static_assert(WM * WN == 4, "four waves");
  static_assert(FM >= 1 && FN >= 1, "tile");
  __shared__ double As[BK][BM];
  __shared__ double Bs[BK][BN];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave % WM) * (BM / WM);
  const int wn = (wave / WM) * (BN / WN);
  const int z = blockIdx.z;
  const int b = z / g.splits;
  const int sp = z % g.splits;
  const int64_t m0 = (int64_t)blockIdx.y * BM;
  const int64_t n0 = (int64_t)blockIdx.x * BN;
  if (g.lower_only && n0 > m0 + BM - 1) return;

  const int64_t aoff = g.amap ? (int64_t)g.amap[b] : (int64_t)b;
  const TA* __restrict__ A = static_cast<const TA*>(g.A) + aoff * g.strideA;
  const TB* __restrict__ B = static_cast<const TB*>(g.B) + (int64_t)b * g.strideB;

  // K range of this tile (triangular operands skip structural zeros)
  int64_t kb = 0, ke = g.K;
  if (g.tri == 1) ke = ke < m0 + BM ? ke : m0 + BM;
  if (g.tri == 2) kb = (m0 / BK) * BK;
  if (g.splits > 1) {
    int64_t tiles = (ke - kb + BK - 1) / BK;
    int64_t per = (tiles + g.splits - 1) / g.splits;
    int64_t s0 = kb + sp * per * BK;
    int64_t s1 = s0 + per * BK;
    kb = s0;
    ke = s1 < ke ? s1 : ke;
  }

  v4d acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  double ra[AE], rb[BE];
  auto loadA = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int idx = tid + e * 256;
      const int mm = TRA ? idx % BM : idx / BK;
      const int kk = TRA ? idx / BM : idx % BK;
      const int64_t gm = m0 + mm, gk = k0 + kk;
      double v = 0.0;
      if (gm < g.M && gk < ke) v = (double)(TRA ? A[gk * g.lda + gm] : A[gm * g.lda + gk]);
      ra[e] = v;
    }
  };
  auto loadB = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int idx = tid + e * 256;
      double v = 0.0;
      if (idx < BK * BN) {
        const int nn = TRB ? idx / BK : idx % BN;
        const int kk = TRB ? idx % BK : idx / BN;
        const int64_t gn = n0 + nn, gk = k0 + kk;
        if (gn < g.N && gk < ke) v = (double)(TRB ? B[gn * g.ldb + gk] : B[gk * g.ldb + gn]);
      }
      rb[e] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int idx = tid + e * 256;
      const int mm = TRA ? idx % BM : idx / BK;
      const int kk = TRA ? idx / BM : idx % BK;
      As[kk][mm] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int idx = tid + e * 256;
      if (idx < BK * BN) {
        const int nn = TRB ? idx / BK : idx % BN;
        const int kk = TRB ? idx % BK : idx / BN;
        Bs[kk][nn] = rb[e];
      }
    }
  };

  if (kb < ke) {
    loadA(kb);
    loadB(kb);
  }
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + BK < ke) {
      loadA(k0 + BK);
      loadB(k0 + BK);
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double af[FM], bf[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = As[ks + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < FN; ++j) bf[j] = Bs[ks + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }

  double* C = g.C + (int64_t)(g.splits > 1 ? z : b) * g.strideC;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm + i * 16 + 4 * r + (lane >> 4);
        const int64_t gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < g.M && gn < g.N) {
          double* p = C + gm * g.ldc + gn;
          if (g.splits > 1)
            *p = acc[i][j][r];
          else
            *p = g.alpha * acc[i][j][r] + (g.beta != 0.0 ? g.beta * *p : 0.0);
        }
      }
}

template <typename TA, typename TB, bool TRA, bool TRB>
static void launch_t(const Gemm& g, hipStream_t s) {
  const int z = g.batch * g.splits;
  if (g.N >= 48) {
    dim3 grid((unsigned)cdiv(g.N, 64), (unsigned)cdiv(g.M, 64), (unsigned)z);
    hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, TRA, TRB, 64, 64, 2, 2>), grid, dim3(256), 0, s, g);
  } else if (g.N >= 24) {
    dim3 grid((unsigned)cdiv(g.N, 32), (unsigned)cdiv(g.M, 64), (unsigned)z);
    hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, TRA, TRB, 64, 32, 2, 2>), grid, dim3(256), 0, s, g);
  } else {
    dim3 grid((unsigned)cdiv(g.N, 16), (unsigned)cdiv(g.M, 64), (unsigned)z);
    hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, TRA, TRB, 64, 16, 4, 1>), grid, dim3(256), 0, s, g);
  }
  IHS_CHECK_LAUNCH();
}

template <typename TA, typename TB>
static void launch_tt(const Gemm& g, bool ta, bool tb, hipStream_t s) {
  if (!ta && !tb) launch_t<TA, TB, false, false>(g, s);
  else if (ta && !tb) launch_t<TA, TB, true, false>(g, s);
  else if (!ta && tb) launch_t<TA, TB, false, true>(g, s);
  else launch_t<TA, TB, true, true>(g, s);
}

void gemm(const Gemm& g, DT ta, bool transA, DT tb, bool transB, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return;
  if (g.M / 64 >= 65535) fail(IHSBIN_EUNSUP, "gemm: M too large for one launch");
  if (ta == DT::F64 && tb == DT::F64) launch_tt<double, double>(g, transA, transB, s);
  else if (ta == DT::F32 && tb == DT::F64) launch_tt<float, double>(g, transA, transB, s);
  else if (ta == DT::F64 && tb == DT::F32) launch_tt<double, float>(g, transA, transB, s);
  else launch_tt<float, float>(g, transA, transB, s);
}

__global__ void reduce_splits_kernel(const double* __restrict__ part, int splits, int64_t M,
                                     int64_t N, int64_t ldp, int64_t sp, double* __restrict__ C,
                                     int64_t ldc, int64_t sc, double alpha, double beta) {
  const int b = blockIdx.y;
  const int64_t total = M * N;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / N, c = t % N;
    double acc = 0.0;
    for (int s = 0; s < splits; ++s) acc += part[((int64_t)b * splits + s) * sp + r * ldp + c];
    double* p = C + b * sc + r * ldc + c;
    *p = alpha * acc + (beta != 0.0 ? beta * *p : 0.0);
  }
}

void reduce_splits(const double* part, int splits, int batch, int64_t M, int64_t N, int64_t ldp,
                   int64_t stride_part, double* C, int64_t ldc, int64_t strideC, double alpha,
                   double beta, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  int64_t blocks = cdiv(M * N, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(reduce_splits_kernel, dim3((unsigned)blocks, (unsigned)batch), dim3(256), 0, s,
                     part, splits, M, N, ldp, stride_part, C, ldc, strideC, alpha, beta);
  IHS_CHECK_LAUNCH();
}

int pick_splits(int64_t M, int64_t N, int64_t K, int batch, int64_t target) {
  const int64_t bn = N >= 48 ? 64 : (N >= 24 ? 32 : 16);
  const int64_t tiles = cdiv(M, 64) * cdiv(N, bn) * batch;
  int64_t s = cdiv(target, tiles);
  const int64_t kt = cdiv(K, 16);
  if (s > kt / 4) s = kt / 4;  // keep at least four K-slices per split
  if (s < 1) s = 1;
  if (s > 64) s = 64;
  return (int)s;
}

}  // namespace ihs
