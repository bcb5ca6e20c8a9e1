// FP64 GEMM on MFMA for gfx950.
//
// A 256-thread workgroup (four wave64s) computes a BM x BN tile of C; each
// wave owns a (BM/WM) x (BN/WN) sub-tile of 16x16 accumulators fed by
// v_mfma_f64_16x16x4f64.  Operands are staged through LDS in K-slices of 16.
// FP32 operands are widened to FP64 when written to LDS (exact).  The next
// K-slice is prefetched into registers (16-byte vector loads where aligned and
// in bounds) while the matrix cores work on the current one.
//
// LDS layouts are chosen per operand orientation so that the MFMA fragment
// reads are free of bank conflicts: an operand whose contiguous global
// dimension is K is kept row-major with K padded to 18 doubles; one whose
// contiguous dimension is M or N is kept K-major with the row padded by 16
// doubles (row pitch = 128 bytes mod 256).
//
// Fragment layout of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register r of lane l
// holds D[4 r + l / 16][l % 16].
//
// Workgroups are dispatched round-robin over the 8 XCDs; the linear block id
// is remapped so that each XCD walks a contiguous range of tiles (N-tiles
// fastest), so tiles sharing an A row panel share that XCD's L2.
#include "gemm.hpp"

namespace ihs {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// The matrix-core instruction of a compute type and the row of accumulator
// register r held by a lane (column: lane % 16 for both).
//  FP64 v_mfma_f64_16x16x4f64: register r of lane l holds D[4 r + l / 16].
//  FP32 v_mfma_f32_16x16x4f32: register r of lane l holds D[4 (l / 16) + r].
template <typename TM>
struct Mfma;
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int lane) { return 4 * r + (lane >> 4); }
};
template <>
struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int lane) { return 4 * (lane >> 4) + r; }
};

// LDS pitches (in elements) that keep the MFMA fragment reads free of bank
// conflicts: K-major rows start 64 bytes (FP32) / 128 bytes (FP64) apart
// modulo the 256-byte bank period; row-major rows have an odd word stride.
template <typename T>
constexpr int kmajor_pitch(int x) {
  return sizeof(T) == 8 ? x + (48 - x % 32) % 32 : x + (80 - x % 64) % 64;
}
template <typename T>
constexpr int rowmajor_pitch(int bk) {
  return sizeof(T) == 8 ? bk + 2 : bk + 1;
}

template <typename T>
__device__ inline void ld4(const T* p, int, T (&o)[4]) {
  if constexpr (sizeof(T) == 4) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  } else {
    const double2 a = reinterpret_cast<const double2*>(p)[0];
    const double2 b = reinterpret_cast<const double2*>(p)[1];
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
  }
}

// Checked load of up to four consecutive elements (nv valid, rest zero).
template <typename T>
__device__ inline void ld4c(const T* p, int nv, T (&o)[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) o[j] = j < nv ? p[j] : T(0);
}

template <typename TA, typename TB, bool TRA, bool TRB, int BM, int BN, int BK, int WM, int WN,
          bool CHK, int NT, typename TM>
__device__ __forceinline__ void gemm_tile(const Gemm& g, const TA* __restrict__ A,
                                          const TB* __restrict__ B, int64_t m0, int64_t n0,
                                          int64_t kb, int64_t ke, int nblk,
                                          char* __restrict__ smem,
                                          typename Mfma<TM>::acc_t (&acc)[BM / WM / 16][BN / WN / 16]) {
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  constexpr int A_LD = TRA ? kmajor_pitch<TA>(BM) : rowmajor_pitch<TA>(BK);
  constexpr int B_LD = TRB ? rowmajor_pitch<TB>(BK) : kmajor_pitch<TB>(BN);
  constexpr int A_SZ = TRA ? BK * A_LD : BM * A_LD;
  constexpr int B_SZ = TRB ? BN * B_LD : BK * B_LD;
  constexpr int AVEC = BM * BK / 4;
  constexpr int BVEC = BK * BN / 4;
  constexpr int AV = (AVEC + NT - 1) / NT;
  constexpr int BV = (BVEC + NT - 1) / NT;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave % WM) * (BM / WM);
  const int wn = (wave / WM) * (BN / WN);

  TA ra[AV][4];
  TB rb[BV][4];
  auto loadA = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < AV; ++e) {
      const int vid = tid + e * NT;
      if (AVEC % NT != 0 && vid >= AVEC) break;
      int64_t r, c;
      if constexpr (!TRA) {
        r = m0 + vid / (BK / 4);
        c = k0 + 4 * (vid % (BK / 4));
      } else {
        r = k0 + vid / (BM / 4);
        c = m0 + 4 * (vid % (BM / 4));
      }
      const TA* p = A + r * g.lda + c;
      if constexpr (!CHK) {
        ld4<TA>(p, 4, ra[e]);
      } else {
        const int64_t rlim = TRA ? ke : g.M, clim = TRA ? g.M : ke;
        const int nv = r < rlim ? (int)(clim - c < 4 ? (clim - c > 0 ? clim - c : 0) : 4) : 0;
        ld4c<TA>(p, nv, ra[e]);
      }
    }
  };
  auto loadB = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < BV; ++e) {
      const int vid = tid + e * NT;
      if (BVEC % NT != 0 && vid >= BVEC) break;
      int64_t r, c;
      if constexpr (!TRB) {
        r = k0 + vid / (BN / 4);
        c = n0 + 4 * (vid % (BN / 4));
      } else {
        r = n0 + vid / (BK / 4);
        c = k0 + 4 * (vid % (BK / 4));
      }
      const TB* p = B + r * g.ldb + c;
      if constexpr (!CHK) {
        ld4<TB>(p, 4, rb[e]);
      } else {
        const int64_t rlim = TRB ? g.N : ke, clim = TRB ? ke : g.N;
        const int nv = r < rlim ? (int)(clim - c < 4 ? (clim - c > 0 ? clim - c : 0) : 4) : 0;
        ld4c<TB>(p, nv, rb[e]);
      }
    }
  };
  auto store = [&](TA* As, TB* Bs) {
#pragma unroll
    for (int e = 0; e < AV; ++e) {
      const int vid = tid + e * NT;
      if (AVEC % NT != 0 && vid >= AVEC) break;
      const int o = TRA ? (vid / (BM / 4)) * A_LD + 4 * (vid % (BM / 4))
                        : (vid / (BK / 4)) * A_LD + 4 * (vid % (BK / 4));
#pragma unroll
      for (int j = 0; j < 4; ++j) As[o + j] = ra[e][j];
    }
#pragma unroll
    for (int e = 0; e < BV; ++e) {
      const int vid = tid + e * NT;
      if (BVEC % NT != 0 && vid >= BVEC) break;
      const int o = TRB ? (vid / (BK / 4)) * B_LD + 4 * (vid % (BK / 4))
                        : (vid / (BN / 4)) * B_LD + 4 * (vid % (BN / 4));
#pragma unroll
      for (int j = 0; j < 4; ++j) Bs[o + j] = rb[e][j];
    }
  };
  auto compute = [&](const TA* As, const TB* Bs) {
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4), c16 = lane & 15;
      TM af[FM], bf[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        af[i] = (TM)(TRA ? As[kr * A_LD + wm + i * 16 + c16] : As[(wm + i * 16 + c16) * A_LD + kr]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bf[j] = (TM)(TRB ? Bs[(wn + j * 16 + c16) * B_LD + kr] : Bs[kr * B_LD + wn + j * 16 + c16]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = Mfma<TM>::mma(af[i], bf[j], acc[i][j]);
    }
  };

  if (kb >= ke) return;
  // a wave whose columns all lie past N only helps stage the operands
  const bool live = nblk > 0;
  constexpr int A_BYTES = (A_SZ * (int)sizeof(TA) + 15) / 16 * 16;
  constexpr int B_BYTES = (B_SZ * (int)sizeof(TB) + 15) / 16 * 16;
  constexpr int STAGE = A_BYTES + B_BYTES;
  // the two LDS stages are addressed arithmetically (no branch on the stage),
  // so the accumulators keep one register assignment through the loop
  auto As = [&](int buf) { return reinterpret_cast<TA*>(smem + buf * STAGE); };
  auto Bs = [&](int buf) { return reinterpret_cast<TB*>(smem + buf * STAGE + A_BYTES); };
  loadA(kb);
  loadB(kb);
  store(As(0), Bs(0));
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    const bool more = k0 + BK < ke;
    if (more) {
      loadA(k0 + BK);
      loadB(k0 + BK);
    }
    if (live) compute(As(buf), Bs(buf));
    if (more) store(As(buf ^ 1), Bs(buf ^ 1));
    __syncthreads();
    buf ^= 1;
  }
}

// TM: the matrix cores' compute type (double, or float for FP32 operands);
// TC: the type of C (float is used only with TM = float; split-K partials of
// an FP32 product are stored as double).
template <typename TA, typename TB, bool TRA, bool TRB, int BM, int BN, int BK, int WM, int WN,
          int NT = 256, typename TM = double, typename TC = double>
__global__ __launch_bounds__(NT) void gemm_f64_kernel(Gemm g) {
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  static_assert(WM * WN * 64 == NT, "one wave per sub-tile");
  static_assert(FM >= 1 && FN >= 1, "tile");
  constexpr int A_LD = TRA ? kmajor_pitch<TA>(BM) : rowmajor_pitch<TA>(BK);
  constexpr int B_LD = TRB ? rowmajor_pitch<TB>(BK) : kmajor_pitch<TB>(BN);
  constexpr int A_SZ = TRA ? BK * A_LD : BM * A_LD;
  constexpr int B_SZ = TRB ? BN * B_LD : BK * B_LD;
  constexpr int A_BYTES = (A_SZ * (int)sizeof(TA) + 15) / 16 * 16;
  constexpr int B_BYTES = (B_SZ * (int)sizeof(TB) + 15) / 16 * 16;
  __shared__ __attribute__((aligned(16))) char smem[2 * (A_BYTES + B_BYTES)];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = (wave % WM) * (BM / WM);
  const int wn = (wave / WM) * (BN / WN);

  // XCD-aware tile order: workgroups are dispatched round-robin over the 8
  // XCDs, so the linear id is remapped to give each XCD a contiguous range;
  // within (bz fixed) the range is walked in groups of kGroupM row tiles, all
  // of a group's row tiles for one column tile before the next column tile,
  // so the tiles resident on an XCD at a time share both their A row panels
  // and their B column panels in its L2.
  constexpr unsigned kGroupM = 8;
  const unsigned gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const unsigned total = gx * gy * gz;
  unsigned lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  if ((total & 7u) == 0) lin = (lin & 7u) * (total >> 3) + (lin >> 3);
  const unsigned bz = lin / (gx * gy);
  const unsigned in_z = lin - bz * (gx * gy);
  const unsigned first_by = (in_z / (kGroupM * gx)) * kGroupM;
  const unsigned gm = gy - first_by < kGroupM ? gy - first_by : kGroupM;
  const unsigned in_g = in_z - first_by * gx;
  const unsigned by = first_by + in_g % gm, bx = in_g / gm;

  const int z = (int)bz;
  const int bb = z / g.splits;
  const int sp = z % g.splits;
  const int b = bb % g.batch, b2 = bb / g.batch;
  const int64_t m0 = (int64_t)by * BM;
  const int64_t n0 = (int64_t)bx * BN;
  if (g.lower_only && n0 > m0 + BM - 1) return;

  const int64_t aoff = g.amap ? (int64_t)g.amap[b] : (int64_t)b;
  const TA* __restrict__ A = static_cast<const TA*>(g.A) + aoff * g.strideA + b2 * g.strideA2;
  const TB* __restrict__ B = static_cast<const TB*>(g.B) + (int64_t)b * g.strideB + b2 * g.strideB2;

  int64_t kb = 0, ke = g.K;
  if (g.tri == 1) ke = ke < m0 + BM ? ke : m0 + BM;
  if (g.tri == 2) kb = (m0 / BK) * BK;
  if (g.tri == 3) kb = (n0 / BK) * BK;
  if (g.tri == 4) ke = ke < n0 + BN ? ke : n0 + BN;
  if (g.splits > 1) {
    const int64_t tiles = (ke - kb + BK - 1) / BK;
    const int64_t per = (tiles + g.splits - 1) / g.splits;
    const int64_t s0 = kb + sp * per * BK;
    const int64_t s1 = s0 + per * BK;
    kb = s0;
    ke = s1 < ke ? s1 : ke;
  }

  typedef typename Mfma<TM>::acc_t acc_t;
  acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  // 16-column blocks of this wave that hold columns < N (wave-uniform)
  int nblk = (int)((g.N - (n0 + wn) + 15) / 16);
  nblk = __builtin_amdgcn_readfirstlane(nblk < 0 ? 0 : (nblk > FN ? FN : nblk));

  // interior tiles with whole K-slices and aligned operands take the fast path
  const int64_t nr = g.n_read > g.N ? g.n_read : g.N;
  const bool fast = g.vec_ok && m0 + BM <= g.M && n0 + BN <= nr && ((ke - kb) % BK) == 0;
  if (fast)
    gemm_tile<TA, TB, TRA, TRB, BM, BN, BK, WM, WN, false, NT, TM>(g, A, B, m0, n0, kb, ke, nblk,
                                                                    smem, acc);
  else
    gemm_tile<TA, TB, TRA, TRB, BM, BN, BK, WM, WN, true, NT, TM>(g, A, B, m0, n0, kb, ke, nblk,
                                                                   smem, acc);

  TC* C = reinterpret_cast<TC*>(g.C) +
          (g.splits > 1 ? (int64_t)z * g.strideC
                        : (int64_t)b * g.strideC + (int64_t)b2 * g.strideC2);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm + i * 16 + Mfma<TM>::row(r, lane);
        const int64_t gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < g.M && gn < g.N) {
          TC* p = C + gm * g.ldc + gn;
          if (g.splits > 1)
            *p = (TC)acc[i][j][r];
          else
            *p = (TC)(g.alpha * (double)acc[i][j][r] +
                      (g.beta != 0.0 ? g.beta * (double)*p : 0.0));
        }
      }
}

// Tile shapes: large-M problems use 128-256 row tiles; N picks the width.
enum class Tile { T64x64, T64x32, T64x16, T128x64, T256x32, T256x16 };

static Tile pick_tile(int64_t M, int64_t N) {
  if (M >= 1024) {
    if (N <= 16) return Tile::T256x16;
    if (N <= 32) return Tile::T256x32;
    return Tile::T128x64;
  }
  if (N >= 48) return Tile::T64x64;
  if (N >= 24) return Tile::T64x32;
  return Tile::T64x16;
}

static void tile_dims(Tile t, int& bm, int& bn) {
  switch (t) {
    case Tile::T64x64: bm = 64; bn = 64; break;
    case Tile::T64x32: bm = 64; bn = 32; break;
    case Tile::T64x16: bm = 64; bn = 16; break;
    case Tile::T128x64: bm = 128; bn = 64; break;
    case Tile::T256x32: bm = 256; bn = 32; break;
    default: bm = 256; bn = 16; break;
  }
}

template <typename TA, typename TB, bool TRA, bool TRB, int BM, int BN, int BK, int WM, int WN,
          int NT = 256, typename TM = double, typename TC = double>
static void launch_one(const Gemm& g, hipStream_t s) {
  dim3 grid((unsigned)cdiv(g.N, BN), (unsigned)cdiv(g.M, BM),
            (unsigned)(g.batch * g.batch2 * g.splits));
  if (g.batch2 > 1 && g.splits > 1) fail(IHSBIN_EUNSUP, "gemm: batch2 with split-K");
  if (grid.y > 65535u || grid.z > 65535u) fail(IHSBIN_EUNSUP, "gemm grid too large");
  hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, TRA, TRB, BM, BN, BK, WM, WN, NT, TM, TC>), grid,
                     dim3(NT), 0, s, g);
}

template <typename TA, typename TB, bool TRA, bool TRB>
static void launch_t(const Gemm& g, hipStream_t s) {
  switch (g.small_tiles ? Tile::T64x64 : pick_tile(g.M, g.N)) {
    case Tile::T64x64: launch_one<TA, TB, TRA, TRB, 64, 64, 16, 2, 2>(g, s); break;
    case Tile::T64x32: launch_one<TA, TB, TRA, TRB, 64, 32, 16, 2, 2>(g, s); break;
    case Tile::T64x16: launch_one<TA, TB, TRA, TRB, 64, 16, 16, 4, 1>(g, s); break;
    case Tile::T128x64: launch_one<TA, TB, TRA, TRB, 128, 64, 16, 2, 2>(g, s); break;
    case Tile::T256x32: launch_one<TA, TB, TRA, TRB, 256, 32, 16, 4, 1>(g, s); break;
    case Tile::T256x16: launch_one<TA, TB, TRA, TRB, 256, 16, 32, 4, 1>(g, s); break;
  }
  IHS_CHECK_LAUNCH();
}

static bool aligned16(const void* p, int64_t ld, int64_t stride, size_t es) {
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0 && ((size_t)ld * es) % 16 == 0 &&
         ((size_t)stride * es) % 16 == 0;
}

// Column-matched tiles: 128 x 16q with the four waves stacked along M, so every
// wave owns all 16q columns of its 32 rows (work stays balanced across SIMDs).
template <typename TA, bool TRA>
static void launch_cols(const Gemm& g, int q, hipStream_t s) {
  switch (q) {
    case 1: launch_one<TA, double, TRA, false, 128, 16, 32, 4, 1>(g, s); break;
    case 2: launch_one<TA, double, TRA, false, 128, 32, 16, 4, 1>(g, s); break;
    case 3: launch_one<TA, double, TRA, false, 128, 48, 16, 4, 1>(g, s); break;
    case 4: launch_one<TA, double, TRA, false, 128, 64, 16, 4, 1>(g, s); break;
    case 5: launch_one<TA, double, TRA, false, 128, 80, 16, 4, 1>(g, s); break;
    case 6: launch_one<TA, double, TRA, false, 128, 96, 16, 4, 1>(g, s); break;
    default: launch_one<TA, double, TRA, false, 128, 112, 16, 4, 1>(g, s); break;
  }
  IHS_CHECK_LAUNCH();
}

// The same column-matched tiles on the FP32 matrix cores: A FP32, B FP32,
// C FP32 (cf32) or FP64 (split-K partials).
template <bool TRA, typename TC>
static void launch_cols_f32(const Gemm& g, int q, hipStream_t s) {
  switch (q) {
    case 1: launch_one<float, float, TRA, false, 128, 16, 32, 4, 1, 256, float, TC>(g, s); break;
    case 2: launch_one<float, float, TRA, false, 128, 32, 16, 4, 1, 256, float, TC>(g, s); break;
    case 3: launch_one<float, float, TRA, false, 128, 48, 16, 4, 1, 256, float, TC>(g, s); break;
    case 4: launch_one<float, float, TRA, false, 128, 64, 16, 4, 1, 256, float, TC>(g, s); break;
    case 5: launch_one<float, float, TRA, false, 128, 80, 16, 4, 1, 256, float, TC>(g, s); break;
    case 6: launch_one<float, float, TRA, false, 128, 96, 16, 4, 1, 256, float, TC>(g, s); break;
    default: launch_one<float, float, TRA, false, 128, 112, 16, 4, 1, 256, float, TC>(g, s); break;
  }
  IHS_CHECK_LAUNCH();
}

// 256-row tiles with eight waves for tall products: each operand panel is
// re-read by half as many tiles as with 128 rows.
template <bool TRA, typename TC>
static void launch_cols_f32_tall(const Gemm& g, int q, hipStream_t s) {
  switch (q) {
    case 1: launch_one<float, float, TRA, false, 256, 16, 32, 8, 1, 512, float, TC>(g, s); break;
    case 2: launch_one<float, float, TRA, false, 256, 32, 16, 8, 1, 512, float, TC>(g, s); break;
    case 3: launch_one<float, float, TRA, false, 256, 48, 16, 8, 1, 512, float, TC>(g, s); break;
    case 4: launch_one<float, float, TRA, false, 256, 64, 16, 8, 1, 512, float, TC>(g, s); break;
    case 5: launch_one<float, float, TRA, false, 256, 80, 16, 8, 1, 512, float, TC>(g, s); break;
    case 6: launch_one<float, float, TRA, false, 256, 96, 16, 8, 1, 512, float, TC>(g, s); break;
    default: launch_one<float, float, TRA, false, 256, 112, 16, 8, 1, 512, float, TC>(g, s); break;
  }
  IHS_CHECK_LAUNCH();
}

void gemm_cols_f32(const Gemm& g_in, bool transA, bool c_f32, const ColTiles& ct, hipStream_t s) {
  if (g_in.M <= 0 || g_in.N <= 0) return;
  if (ct.q < 1 || ct.q > kColTileMaxQ || (int64_t)ct.c * 16 * ct.q < g_in.N)
    fail(IHSBIN_EINVAL, "gemm_cols_f32: column tiling does not cover N");
  if (c_f32 && (g_in.splits > 1 || g_in.beta != 0.0))
    fail(IHSBIN_EINVAL, "gemm_cols_f32: FP32 output without split-K or beta only");
  Gemm g = g_in;
  g.vec_ok = aligned16(g.A, g.lda, g.strideA, 4) && aligned16(g.B, g.ldb, g.strideB, 4);
  if (g.n_read > (int64_t)ct.c * 16 * ct.q) g.n_read = (int64_t)ct.c * 16 * ct.q;
  const bool tall = g.M >= 4096 && !g.lower_only && g.tri == 0;
  if (c_f32) {
    if (tall) {
      if (transA) launch_cols_f32_tall<true, float>(g, ct.q, s);
      else launch_cols_f32_tall<false, float>(g, ct.q, s);
    } else {
      if (transA) launch_cols_f32<true, float>(g, ct.q, s);
      else launch_cols_f32<false, float>(g, ct.q, s);
    }
  } else {
    if (tall) {
      if (transA) launch_cols_f32_tall<true, double>(g, ct.q, s);
      else launch_cols_f32_tall<false, double>(g, ct.q, s);
    } else {
      if (transA) launch_cols_f32<true, double>(g, ct.q, s);
      else launch_cols_f32<false, double>(g, ct.q, s);
    }
  }
}

ColTiles pick_col_tiles(int64_t N) {
  // cost ~ c (q + 1/4): a tile's fixed share (its pass over the A panel) is
  // about a quarter of one 16-column block's work; never cover more columns
  // than the padded width (16, 32 or a multiple of 64) that buffers are sized for
  const int64_t nb = cdiv(N, 16);
  const int64_t cap = nb <= 2 ? nb : 4 * cdiv(nb, 4);
  ColTiles best{(int)cdiv(nb, 4), 4};
  double best_cost = 1e300;
  for (int64_t c = cdiv(nb, kColTileMaxQ); c <= nb; ++c) {
    const int64_t q = cdiv(nb, c);
    if (c * q > cap) continue;
    const double cost = (double)c * ((double)q + 0.25);
    if (cost < best_cost) {
      best_cost = cost;
      best = ColTiles{(int)c, (int)q};
    }
    if (q == 1) break;
  }
  return best;
}

void gemm_cols(const Gemm& g_in, DT ta, bool transA, const ColTiles& ct, hipStream_t s) {
  if (g_in.M <= 0 || g_in.N <= 0) return;
  if (ct.q < 1 || ct.q > kColTileMaxQ || (int64_t)ct.c * 16 * ct.q < g_in.N)
    fail(IHSBIN_EINVAL, "gemm_cols: column tiling does not cover N");
  Gemm g = g_in;
  const size_t ea = ta == DT::F32 ? 4 : 8;
  g.vec_ok = aligned16(g.A, g.lda, g.strideA, ea) && aligned16(g.B, g.ldb, g.strideB, 8);
  if (g.n_read > (int64_t)ct.c * 16 * ct.q) g.n_read = (int64_t)ct.c * 16 * ct.q;
  if (ta == DT::F32) {
    if (transA) launch_cols<float, true>(g, ct.q, s);
    else launch_cols<float, false>(g, ct.q, s);
  } else {
    if (transA) launch_cols<double, true>(g, ct.q, s);
    else launch_cols<double, false>(g, ct.q, s);
  }
}

int pick_splits_cols(int64_t M, const ColTiles& ct, int64_t K, int64_t target) {
  // rounded down: a grid just above a whole number of resident rounds leaves
  // a nearly empty last round (22 splits of 48 tiles ran 17 % slower than 21)
  const int64_t tiles = cdiv(M, 128) * ct.c;
  int64_t sp = target / tiles;
  const int64_t kt = cdiv(K, 16);
  if (sp > kt / 8) sp = kt / 8;
  if (sp < 1) sp = 1;
  if (sp > 256) sp = 256;
  return (int)sp;
}


void gemm(const Gemm& g_in, DT ta, bool transA, DT tb, bool transB, hipStream_t s) {
  if (g_in.M <= 0 || g_in.N <= 0) return;
  Gemm g = g_in;
  const size_t ea = ta == DT::F32 ? 4 : 8, eb = tb == DT::F32 ? 4 : 8;
  g.vec_ok = aligned16(g.A, g.lda, g.strideA, ea) && aligned16(g.B, g.ldb, g.strideB, eb);
  const bool f64 = ta == DT::F64 && tb == DT::F64;
  if (f64 && !transA && !transB) launch_t<double, double, false, false>(g, s);
  else if (f64 && transA && !transB) launch_t<double, double, true, false>(g, s);
  else if (f64 && !transA && transB) launch_t<double, double, false, true>(g, s);
  else if (ta == DT::F32 && tb == DT::F64 && !transB) {
    if (transA) launch_t<float, double, true, false>(g, s);
    else launch_t<float, double, false, false>(g, s);
  } else if (ta == DT::F64 && tb == DT::F32 && !transA && !transB) {
    launch_t<double, float, false, false>(g, s);
  } else if (ta == DT::F32 && tb == DT::F32 && transA && !transB) {
    launch_t<float, float, true, false>(g, s);
  } else {
    fail(IHSBIN_EUNSUP, "gemm: operand type / transpose combination not built");
  }
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

int pick_splits_lower(int64_t n, int64_t K, int64_t target) {
  const int64_t nt = cdiv(n, 64);
  const int64_t tiles = nt * (nt + 1) / 2;
  int64_t s = cdiv(target, tiles);
  const int64_t kt = cdiv(K, 16);
  if (s > kt / 8) s = kt / 8;  // keep at least eight K-slices per split
  if (s < 1) s = 1;
  if (s > 64) s = 64;
  return (int)s;
}

int pick_splits(int64_t M, int64_t N, int64_t K, int batch, int64_t target) {
  int bm = 64, bn = 64;
  tile_dims(pick_tile(M, N), bm, bn);
  const int64_t tiles = cdiv(M, bm) * cdiv(N, bn) * batch;
  int64_t s = cdiv(target, tiles);
  const int64_t kt = cdiv(K, 16);
  if (s > kt / 8) s = kt / 8;  // keep at least eight K-slices per split
  if (s < 1) s = 1;
  if (s > 256) s = 256;
  return (int)s;
}

}  // namespace ihs
