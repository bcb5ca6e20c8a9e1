// Element-wise and reduction kernels of the basis recursion (Proposition,
// Eq. (equ:upd); Algorithm 2 / 5) and of the path composition (Algorithm 3 /
// 6), plus the Lanczos helpers used to estimate the spectrum of
// P_S (A^T A + lam0 I) for the step size.
//
// Column layout of the working set during step i: active interval a (in the
// order of the active list) owns the contiguous columns
// [a*i*K, (a+1)*i*K) of U, holding u_{i-1,j} (j < i) for every right-hand
// side kk at column (a*i + j)*K + kk.  Rows are the d coordinates.
#include "basis.hpp"

namespace ihs {

// Column block a of R = C block a / per (C: blocks of d x K).
__global__ void seed_rhs_kernel(const double* __restrict__ C, int64_t d, int64_t K, int na,
                                int per, double* __restrict__ R, int64_t ldr) {
  const int64_t total = d * K * na;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / (K * na), c = t % (K * na);
    const int64_t a = c / K;
    R[r * ldr + c] = C[((a / per) * d + r) * K + c % K];
  }
}

void launch_seed_rhs(const double* C, int64_t d, int64_t K, int na, double* R, int64_t ldr,
                     hipStream_t st, int per) {
  int64_t blocks = cdiv(d * K * na, 256);
  if (blocks > 16384) blocks = 16384;
  if (per < 1) per = na;
  hipLaunchKernelGGL(seed_rhs_kernel, dim3((unsigned)blocks), dim3(256), 0, st, C, d, K, na, per, R,
                     ldr);
  IHS_CHECK_LAUNCH();
}

// ut_{l,0} = u_{0,0} (= U column block of position a), for every a.
__global__ void store_first_kernel(const double* __restrict__ U, int64_t ldu, int64_t d, int64_t K,
                                   int na, const int32_t* __restrict__ ids, int64_t kcap,
                                   double* __restrict__ basis) {
  const int64_t total = d * K * na;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / (K * na), c = t % (K * na);
    const int a = (int)(c / K);
    const int64_t kk = c % K;
    basis[(((int64_t)ids[a] * kcap) * d + r) * K + kk] = U[r * ldu + c];
  }
}

void launch_store_first(const double* U, int64_t ldu, int64_t d, int64_t K, int na,
                        const int32_t* ids, int64_t kcap, double* basis, hipStream_t st) {
  int64_t blocks = cdiv(d * K * na, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(store_first_kernel, dim3((unsigned)blocks), dim3(256), 0, st, U, ldu, d, K, na,
                     ids, kcap, basis);
  IHS_CHECK_LAUNCH();
}

// R_j = tau_a (W_j + ref_a U_j) [j < i] + U_{j-1} [j >= 1], for j = 0..i.
__global__ void form_r_kernel(const double* __restrict__ W, const double* __restrict__ U,
                              int64_t ld, int64_t d, int64_t K, int na, int i,
                              const double* __restrict__ tau, const double* __restrict__ ref,
                              double* __restrict__ R) {
  const int64_t cw_new = (int64_t)(i + 1) * K;
  const int64_t cols = cw_new * na;
  const int64_t total = d * cols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / cols, c = t % cols;
    const int a = (int)(c / cw_new);
    const int64_t jc = c % cw_new;
    const int j = (int)(jc / K);
    const int64_t kk = jc % K;
    const int64_t base_old = (int64_t)a * i * K;
    double v = 0.0;
    if (j < i) {
      const int64_t co = base_old + (int64_t)j * K + kk;
      v = tau[a] * (W[r * ld + co] + ref[a] * U[r * ld + co]);
    }
    if (j >= 1) v += U[r * ld + base_old + (int64_t)(j - 1) * K + kk];
    R[r * ld + c] = v;
  }
}

void launch_form_r(const double* W, const double* U, int64_t ld, int64_t d, int64_t K, int na,
                   int i, const double* tau, const double* ref, double* R, hipStream_t st) {
  int64_t blocks = cdiv(d * K * na * (i + 1), 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(form_r_kernel, dim3((unsigned)blocks), dim3(256), 0, st, W, U, ld, d, K, na, i,
                     tau, ref, R);
  IHS_CHECK_LAUNCH();
}

// u_{i,j} = u_{i-1,j} - Z_j (u_{i-1,i} := 0); ut_j += u_{i,j};
// stop statistics per position a: ||sum_j mu^j u_{i,j}||^2 and
// ||sum_j mu^j ut_j||^2 at mu_lo and mu_hi, as per-block partial sums.
__global__ __launch_bounds__(256) void update_kernel(
    const double* __restrict__ U, const double* __restrict__ Z, double* __restrict__ Unew,
    int64_t ld, int64_t d, int64_t K, int i, const int32_t* __restrict__ ids, int64_t kcap,
    double* __restrict__ basis, const double* __restrict__ mu_lo, const double* __restrict__ mu_hi,
    double* __restrict__ partial) {
  __shared__ double red[4][256];
  const int a = blockIdx.y;
  const int64_t l = ids[a];
  const double ml = mu_lo[a], mh = mu_hi[a];
  const int64_t base_old = (int64_t)a * i * K;
  const int64_t base_new = (int64_t)a * (i + 1) * K;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  const int64_t total = d * K;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / K, kk = t % K;
    double il = 0.0, ih = 0.0, xl = 0.0, xh = 0.0, pl = 1.0, ph = 1.0;
    for (int j = 0; j <= i; ++j) {
      const double old = j < i ? U[r * ld + base_old + (int64_t)j * K + kk] : 0.0;
      const int64_t cn = base_new + (int64_t)j * K + kk;
      const double un = old - Z[r * ld + cn];
      Unew[r * ld + cn] = un;
      double* bp = basis + ((l * kcap + j) * d + r) * K + kk;
      const double ut = *bp + un;
      *bp = ut;
      il += pl * un;
      ih += ph * un;
      xl += pl * ut;
      xh += ph * ut;
      pl *= ml;
      ph *= mh;
    }
    s0 += il * il;
    s1 += ih * ih;
    s2 += xl * xl;
    s3 += xh * xh;
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  red[2][threadIdx.x] = s2;
  red[3][threadIdx.x] = s3;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) partial[((int64_t)a * gridDim.x + blockIdx.x) * 4 + threadIdx.x] = red[threadIdx.x][0];
}

int launch_update(const double* U, const double* Z, double* Unew, int64_t ld, int64_t d, int64_t K,
                  int na, int i, const int32_t* ids, int64_t kcap, double* basis,
                  const double* mu_lo, const double* mu_hi, double* partial, hipStream_t st) {
  int64_t bx = cdiv(d * K, 256);
  if (bx > 64) bx = 64;
  hipLaunchKernelGGL(update_kernel, dim3((unsigned)bx, (unsigned)na), dim3(256), 0, st, U, Z, Unew,
                     ld, d, K, i, ids, kcap, basis, mu_lo, mu_hi, partial);
  IHS_CHECK_LAUNCH();
  return (int)bx;
}

// Keep the column blocks of the positions listed in keep[] (old positions).
__global__ void compact_kernel(const double* __restrict__ Src, double* __restrict__ Dst, int64_t ld,
                               int64_t d, int64_t cw, int na_new, const int32_t* __restrict__ keep) {
  const int64_t cols = cw * na_new;
  const int64_t total = d * cols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / cols, c = t % cols;
    const int a = (int)(c / cw);
    Dst[r * ld + c] = Src[r * ld + (int64_t)keep[a] * cw + c % cw];
  }
}

void launch_compact(const double* Src, double* Dst, int64_t ld, int64_t d, int64_t cw, int na_new,
                    const int32_t* keep, hipStream_t st) {
  int64_t blocks = cdiv(d * cw * na_new, 256);
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) return;
  hipLaunchKernelGGL(compact_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Src, Dst, ld, d, cw,
                     na_new, keep);
  IHS_CHECK_LAUNCH();
}

// x(lam_t) = tau_t sum_{j<k_t} mu_t^j ut_{l_t, j}, Horner from the top term.
template <typename TO>
__global__ void eval_kernel(const double* __restrict__ basis, int64_t kcap, int64_t d, int64_t K,
                            const EvalItem* __restrict__ items, TO* __restrict__ X, int64_t ldx) {
  const EvalItem it = items[blockIdx.y];
  const int64_t total = d * K;
  const double* B = basis + (int64_t)it.l * kcap * d * K;
  TO* Xt = X + (int64_t)blockIdx.y * d * ldx;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / K, kk = t % K;
    double acc = 0.0;
    for (int j = it.k - 1; j >= 0; --j) acc = acc * it.mu + B[((int64_t)j * d + r) * K + kk];
    Xt[r * ldx + kk] = (TO)(it.tau * acc);
  }
}

void launch_eval(const double* basis, int64_t kcap, int64_t d, int64_t K, const EvalItem* items,
                 int64_t T, void* X, int64_t ldx, int x_dtype, hipStream_t st) {
  int64_t bx = cdiv(d * K, 256);
  if (bx > 256) bx = 256;
  for (int64_t t0 = 0; t0 < T; t0 += 65535) {
    const int64_t tn = (T - t0) < 65535 ? (T - t0) : 65535;
    if (x_dtype == IHSBIN_F32)
      hipLaunchKernelGGL(eval_kernel<float>, dim3((unsigned)bx, (unsigned)tn), dim3(256), 0, st,
                         basis, kcap, d, K, items + t0, (float*)X + t0 * d * ldx, ldx);
    else
      hipLaunchKernelGGL(eval_kernel<double>, dim3((unsigned)bx, (unsigned)tn), dim3(256), 0, st,
                         basis, kcap, d, K, items + t0, (double*)X + t0 * d * ldx, ldx);
    IHS_CHECK_LAUNCH();
  }
}

// ------------------------------------------------------------- Lanczos
__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

// q_0 for column a: uniform(-1, 1) draws, normalized.
__global__ __launch_bounds__(256) void lanczos_start_kernel(uint64_t key, int64_t d, int64_t ld,
                                                            double* Q0) {
  __shared__ double red[256];
  const int a = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < d; r += blockDim.x) {
    const uint64_t x = sm_draw(key, (uint64_t)(a * d + r));
    const double v = (double)(x >> 11) * 0x1.0p-52 - 1.0;
    Q0[r * ld + a] = v;
    s += v * v;
  }
  const double nrm = sqrt(block_sum(s, red));
  for (int64_t r = threadIdx.x; r < d; r += blockDim.x) Q0[r * ld + a] /= nrm;
}

void launch_lanczos_start(uint64_t seed, int64_t d, int na, int64_t ld, double* Q0, hipStream_t st) {
  hipLaunchKernelGGL(lanczos_start_kernel, dim3(na), dim3(256), 0, st, stream_key(seed, 4), d, ld, Q0);
  IHS_CHECK_LAUNCH();
}

// S[:, a] += lam0[a] * T[:, a]
__global__ void add_shift_kernel(double* S, const double* __restrict__ T, int64_t d, int na,
                                 int64_t ld, const double* __restrict__ lam0) {
  const int64_t total = d * na;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / na, a = t % na;
    S[r * ld + a] += lam0[a] * T[r * ld + a];
  }
}

void launch_add_shift(double* S, const double* T, int64_t d, int na, int64_t ld, const double* lam0,
                      hipStream_t st) {
  int64_t blocks = cdiv(d * na, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(add_shift_kernel, dim3((unsigned)blocks), dim3(256), 0, st, S, T, d, na, ld,
                     lam0);
  IHS_CHECK_LAUNCH();
}

// Full re-orthogonalization (two classical Gram-Schmidt passes) of w against
// q_0..q_j, alpha_j = <q_j, B q_j>, beta_{j+1} = ||w||, q_{j+1} = w / beta.
// Each pass computes all j+1 inner products at once (one reduction), then
// subtracts the projection.  One workgroup per column a.
constexpr int kLanczosMax = 64;

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(256) void lanczos_orth_kernel(double* Q, double* Wv, int64_t d,
                                                           int64_t ld, int j, int J, double* alpha,
                                                           double* beta) {
  __shared__ double red[kLanczosMax][4];
  __shared__ double h[kLanczosMax];
  __shared__ double bsum[4];
  const int a = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nq = j + 1;
  double al = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int q = 0; q < nq; ++q) {
      const double* Qq = Q + (int64_t)q * d * ld;
      double s = 0.0;
      for (int64_t r = tid; r < d; r += blockDim.x) s += Qq[r * ld + a] * Wv[r * ld + a];
      s = wave_sum(s);
      if (lane == 0) red[q][wave] = s;
    }
    __syncthreads();
    if (tid < nq) h[tid] = red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
    __syncthreads();
    al += h[j];
    for (int64_t r = tid; r < d; r += blockDim.x) {
      double w = Wv[r * ld + a];
      for (int q = 0; q < nq; ++q) w -= h[q] * Q[(int64_t)q * d * ld + r * ld + a];
      Wv[r * ld + a] = w;
    }
    __syncthreads();
  }
  double s = 0.0;
  for (int64_t r = tid; r < d; r += blockDim.x) s += Wv[r * ld + a] * Wv[r * ld + a];
  s = wave_sum(s);
  if (lane == 0) bsum[wave] = s;
  __syncthreads();
  const double b = sqrt(bsum[0] + bsum[1] + bsum[2] + bsum[3]);
  double* Qn = Q + (int64_t)(j + 1) * d * ld;
  for (int64_t r = tid; r < d; r += blockDim.x)
    Qn[r * ld + a] = b > 0.0 ? Wv[r * ld + a] / b : 0.0;
  if (tid == 0) {
    alpha[a * J + j] = al;
    beta[a * J + j] = b;
  }
}

void launch_lanczos_orth(double* Q, double* Wv, int64_t d, int na, int64_t ld, int j, int J,
                         double* alpha, double* beta, hipStream_t st) {
  if (j + 1 > kLanczosMax) fail(IHSBIN_EINVAL, "too many Lanczos steps");
  hipLaunchKernelGGL(lanczos_orth_kernel, dim3(na), dim3(256), 0, st, Q, Wv, d, ld, j, J, alpha,
                     beta);
  IHS_CHECK_LAUNCH();
}

// y_b = L_{map[b]} x_b (lower triangular, row-major d x d): one wave per row
// (general fallback for d above the LDS staging limit).
__global__ __launch_bounds__(256) void trmv_lower_kernel(const double* __restrict__ L, int64_t d,
                                                         int64_t ldl, int64_t ms,
                                                         const int32_t* __restrict__ map, int nb,
                                                         const double* __restrict__ X, int64_t ldx,
                                                         double* __restrict__ Y, int64_t ldy) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t t = wave; t < d * nb; t += nwaves) {
    const int b = (int)(t / d);
    const int64_t r = t % d;
    const double* row = L + (int64_t)map[b] * ms + r * ldl;
    double s0 = 0.0, s1 = 0.0;
    for (int64_t k = lane; k <= r; k += 128) {
      s0 += row[k] * X[k * ldx + b];
      if (k + 64 <= r) s1 += row[k + 64] * X[(k + 64) * ldx + b];
    }
    const double s = wave_sum(s0 + s1);
    if (lane == 0) Y[r * ldy + b] = s;
  }
}

// Same product with the vectors staged in LDS: block (chunk, b) takes
// kTrmvLRows rows of L_b, one wave per row, streaming each row once with
// 16-byte loads for NV vectors (columns b and b + nm share the factor).
constexpr int kTrmvLRows = 32;
constexpr int64_t kTrmvLdsMax = 8192;

template <int NV>
__global__ __launch_bounds__(256) void trmv_lower_lds_kernel(const double* __restrict__ L,
                                                             int64_t d, int64_t ldl, int64_t ms,
                                                             const int32_t* __restrict__ map,
                                                             int nm, const double* __restrict__ X,
                                                             int64_t ldx, double* __restrict__ Y,
                                                             int64_t ldy) {
  __shared__ double xs[NV][kTrmvLdsMax / NV];
  const int b = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * kTrmvLRows;
  const int64_t rend = (r0 + kTrmvLRows) < d ? (r0 + kTrmvLRows) : d;
  for (int64_t k = threadIdx.x; k < rend; k += blockDim.x)
#pragma unroll
    for (int v = 0; v < NV; ++v) xs[v][k] = X[k * ldx + b + v * nm];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* Lb = L + (int64_t)map[b] * ms;
  // 16-byte loads need every row start 16-byte aligned
  const bool vec = (ldl & 1) == 0 && ((reinterpret_cast<uintptr_t>(Lb) & 15) == 0);
  for (int64_t r = r0 + w; r < rend; r += 4) {
    const double* row = Lb + r * ldl;
    double s[NV][2];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v][0] = s[v][1] = 0.0;
    int64_t k = 2 * lane;
    if (vec) {
      for (; k + 128 + 1 <= r; k += 256) {
        const double2 a0 = *reinterpret_cast<const double2*>(row + k);
        const double2 a1 = *reinterpret_cast<const double2*>(row + k + 128);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          s[v][0] += a0.x * xs[v][k] + a0.y * xs[v][k + 1];
          s[v][1] += a1.x * xs[v][k + 128] + a1.y * xs[v][k + 129];
        }
      }
    }
    for (; k <= r; k += 128) {
      const double a0 = row[k];
      const double a1 = k + 1 <= r ? row[k + 1] : 0.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) s[v][0] += a0 * xs[v][k] + a1 * xs[v][k + 1 <= r ? k + 1 : k];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double t = wave_sum(s[v][0] + s[v][1]);
      if (lane == 0) Y[r * ldy + b + v * nm] = t;
    }
  }
}

// y_b = L_{map[b]}^T x_b, two stages.  Stage 1: one workgroup per (b, 64-column
// panel, 256-row chunk) streams the chunk's rows r >= c0 of the panel once for
// NV vectors and writes partial sums; stage 2 adds the chunk partials in a
// fixed order.
constexpr int kTrmvRows = 256;

template <int NV>
__global__ __launch_bounds__(256) void trmv_upper_t_partial_kernel(
    const double* __restrict__ L, int64_t d, int64_t ldl, int64_t ms,
    const int32_t* __restrict__ map, int nm, const double* __restrict__ X, int64_t ldx,
    double* __restrict__ part) {
  __shared__ double red[NV][4][64];
  const int64_t panels = (d + 63) / 64, chunks = (d + kTrmvRows - 1) / kTrmvRows;
  const int64_t job = blockIdx.x;
  const int b = (int)(job / (panels * chunks));
  const int64_t pc = job % (panels * chunks);
  const int64_t c0 = (pc / chunks) * 64, r0 = (pc % chunks) * kTrmvRows;
  const int cc = threadIdx.x & 63, g = threadIdx.x >> 6;
  const double* Lb = L + (int64_t)map[b] * ms;
  const int64_t c = c0 + cc;
  double s[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) s[v] = 0.0;
  if (c < d && r0 + kTrmvRows > c0) {
    const int64_t rs = r0 > c0 ? r0 : c0, re = (r0 + kTrmvRows) < d ? (r0 + kTrmvRows) : d;
    for (int64_t r = rs + g; r < re; r += 4) {
      const double a = Lb[r * ldl + c];
#pragma unroll
      for (int v = 0; v < NV; ++v) s[v] += a * X[r * ldx + b + v * nm];
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) red[v][g][cc] = s[v];
  __syncthreads();
  if (g == 0 && c < d) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
      part[((int64_t)(b + v * nm) * chunks + (pc % chunks)) * d + c] =
          red[v][0][cc] + red[v][1][cc] + red[v][2][cc] + red[v][3][cc];
  }
}

__global__ void trmv_upper_t_sum_kernel(const double* __restrict__ part, int64_t d, int nb,
                                        int64_t chunks, double* __restrict__ Y, int64_t ldy) {
  const int64_t total = d * nb;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(t / d);
    const int64_t c = t % d;
    double s = 0.0;
    for (int64_t q = c / kTrmvRows; q < chunks; ++q) s += part[((int64_t)b * chunks + q) * d + c];
    Y[c * ldy + b] = s;
  }
}

void launch_trmv(const double* L, int64_t d, const int32_t* map, int nb, bool transpose,
                 const double* X, int64_t ldx, double* Y, int64_t ldy, double* scratch,
                 hipStream_t st, int nv) {
  launch_trmv_block(L, d, d, d * d, map, nb, transpose, X, ldx, Y, ldy, scratch, st, nv);
}

void launch_trmv_block(const double* L, int64_t d, int64_t ldl, int64_t ms, const int32_t* map,
                       int nb, bool transpose, const double* X, int64_t ldx, double* Y,
                       int64_t ldy, double* scratch, hipStream_t st, int nv) {
  if (nv != 1 && nv != 2) fail(IHSBIN_EINVAL, "trmv: nv must be 1 or 2");
  if (nb % nv) fail(IHSBIN_EINVAL, "trmv: columns not a multiple of nv");
  const int nm = nb / nv;
  if (!transpose) {
    if (nv == 2 && d <= kTrmvLdsMax / 2 && nm <= 65535) {
      hipLaunchKernelGGL(trmv_lower_lds_kernel<2>, dim3((unsigned)cdiv(d, kTrmvLRows), (unsigned)nm),
                         dim3(256), 0, st, L, d, ldl, ms, map, nm, X, ldx, Y, ldy);
    } else if (d <= kTrmvLdsMax && nb <= 65535) {
      // one vector per block; the second half of a paired layout reuses map
      for (int v = 0; v < nv; ++v)
        hipLaunchKernelGGL(trmv_lower_lds_kernel<1>,
                           dim3((unsigned)cdiv(d, kTrmvLRows), (unsigned)nm), dim3(256), 0, st, L,
                           d, ldl, ms, map, nm, X + v * nm, ldx, Y + v * nm, ldy);
    } else {
      int64_t blocks = cdiv(d * nm * 64, 256);
      if (blocks > 65536) blocks = 65536;
      for (int v = 0; v < nv; ++v)
        hipLaunchKernelGGL(trmv_lower_kernel, dim3((unsigned)blocks), dim3(256), 0, st, L, d, ldl,
                           ms, map, nm, X + v * nm, ldx, Y + v * nm, ldy);
    }
  } else {
    const int64_t chunks = cdiv(d, kTrmvRows);
    const dim3 grid((unsigned)(cdiv(d, 64) * chunks * nm));
    if (nv == 2)
      hipLaunchKernelGGL(trmv_upper_t_partial_kernel<2>, grid, dim3(256), 0, st, L, d, ldl, ms, map,
                         nm, X, ldx, scratch);
    else
      hipLaunchKernelGGL(trmv_upper_t_partial_kernel<1>, grid, dim3(256), 0, st, L, d, ldl, ms, map,
                         nm, X, ldx, scratch);
    IHS_CHECK_LAUNCH();
    int64_t blocks = cdiv(d * nb, 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(trmv_upper_t_sum_kernel, dim3((unsigned)blocks), dim3(256), 0, st, scratch, d,
                       nb, chunks, Y, ldy);
  }
  IHS_CHECK_LAUNCH();
}

int64_t trmv_scratch_doubles(int64_t d, int nb) { return cdiv(d, kTrmvRows) * d * nb; }

}  // namespace ihs
