// Vector kernels of the adaptive sketch-dimension search (Section 5.1,
// Algorithm 4): the inner products it reads back and its fused update.
// Sums run in a fixed order (per-block tree, then one block over the block
// partials), so repeated runs give the same bits.
#include "ops.hpp"

namespace ihs {

namespace {
constexpr int kDotThreads = 256;
constexpr int kDotBlocksMax = 512;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int h = kDotThreads / 2; h > 0; h >>= 1) {
    if (t < h) sh[t] += sh[t + h];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
}  // namespace

// part[b][0..2] = block b's sums of D.G, D.W and D.D over a grid-stride range
// (W may be null: its sum is then 0).
__global__ __launch_bounds__(kDotThreads) void dots3_kernel(const double* __restrict__ D,
                                                            const double* __restrict__ G,
                                                            const double* __restrict__ W,
                                                            int64_t count,
                                                            double* __restrict__ part) {
  __shared__ double sh[kDotThreads];
  double sg = 0.0, sw = 0.0, sd = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kDotThreads;
  for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < count; i += stride) {
    const double dv = D[i];
    sg += dv * G[i];
    if (W) sw += dv * W[i];
    sd += dv * dv;
  }
  sg = block_sum(sg, sh);
  sw = block_sum(sw, sh);
  sd = block_sum(sd, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = sg;
    part[3 * blockIdx.x + 1] = sw;
    part[3 * blockIdx.x + 2] = sd;
  }
}

__global__ __launch_bounds__(kDotThreads) void dots3_final_kernel(const double* __restrict__ part,
                                                                  int nb,
                                                                  double* __restrict__ out) {
  __shared__ double sh[kDotThreads];
  for (int q = 0; q < 3; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kDotThreads) s += part[3 * b + q];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[q] = s;
  }
}

// X -= tau D;  Gr -= tau (W + lam D)   (W = A^T A D, so W + lam D = H D)
__global__ __launch_bounds__(256) void alg4_step_kernel(double* __restrict__ X,
                                                        double* __restrict__ Gr,
                                                        const double* __restrict__ D,
                                                        const double* __restrict__ W,
                                                        int64_t count, double tau, double lam) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const double dv = D[i];
  X[i] -= tau * dv;
  Gr[i] -= tau * (W[i] + lam * dv);
}

// X = 0, Gr = -C (the gradient at X = 0)
__global__ __launch_bounds__(256) void alg4_init_kernel(const double* __restrict__ C,
                                                        double* __restrict__ X,
                                                        double* __restrict__ Gr, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  X[i] = 0.0;
  Gr[i] = -C[i];
}

int dots3_part_doubles() { return 3 * kDotBlocksMax; }

void launch_dots3(const double* D, const double* G, const double* W, int64_t count, double* part,
                  double* out, hipStream_t st) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocksMax, cdiv(count, 4 * kDotThreads)));
  hipLaunchKernelGGL(dots3_kernel, dim3(nb), dim3(kDotThreads), 0, st, D, G, W, count, part);
  IHS_CHECK_LAUNCH();
  hipLaunchKernelGGL(dots3_final_kernel, dim3(1), dim3(kDotThreads), 0, st, part, nb, out);
  IHS_CHECK_LAUNCH();
}

void launch_alg4_step(double* X, double* Gr, const double* D, const double* W, int64_t count,
                      double tau, double lam, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(alg4_step_kernel, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, st, X, Gr,
                     D, W, count, tau, lam);
  IHS_CHECK_LAUNCH();
}

void launch_alg4_init(const double* C, double* X, double* Gr, int64_t count, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(alg4_init_kernel, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, st, C, X,
                     Gr, count);
  IHS_CHECK_LAUNCH();
}

}  // namespace ihs
