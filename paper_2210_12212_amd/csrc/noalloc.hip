// Path evaluation that allocates no device memory, for callers that cannot
// allocate (code under graph capture, tight serving loops): the lambdas and
// the per-lambda evaluation items are staged in one fixed array per device.
#include <mutex>

#include "basis.hpp"
#include "path.hpp"

namespace ihs {

// Most lambdas one call may evaluate; the scratch holds them (8 bytes each)
// and their evaluation items.
constexpr int64_t kNoallocMaxT = int64_t(1) << 18;
constexpr size_t kNoallocItemsOffset = sizeof(double) * (size_t)kNoallocMaxT;
constexpr size_t kNoallocBytes = kNoallocItemsOffset + sizeof(EvalItem) * (size_t)kNoallocMaxT;

// 8 MiB per device, held until the process ends.  Host code uses it only
// through the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) fail(IHSBIN_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      fail(IHSBIN_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    g_scratch[device] = p;
  }
  return g_scratch[device];
}

// items[t] for lambda lam[t]: its interval (the first boundary grid[j] >= lam,
// j >= 1, gives interval j - 1, clamped to [0, L)), that interval's term
// count and step size, and mu = tau (lam - ref).  The same comparisons and
// the same double operations as the host computation of ihsbin_path_eval.
__global__ void noalloc_items_kernel(const double* __restrict__ lam, int64_t T,
                                     const char* __restrict__ plan, int L,
                                     EvalItem* __restrict__ items) {
  const double* grid = reinterpret_cast<const double*>(plan);
  const double* tau = grid + L + 1;
  const double* ref = tau + L;
  const int32_t* kk = reinterpret_cast<const int32_t*>(ref + L);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double x = lam[t];
    int lo = 1, hi = L + 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (grid[mid] < x) lo = mid + 1;
      else hi = mid;
    }
    int l = lo - 1;
    l = l < 0 ? 0 : (l > L - 1 ? L - 1 : l);
    EvalItem it;
    it.l = l;
    it.k = kk[l];
    it.tau = tau[l];
    it.mu = tau[l] * (x - ref[l]);
    items[t] = it;
  }
}

}  // namespace ihs

using namespace ihs;

int ihsbin_path_eval_noalloc(ihsbin_path* p, const double* lambdas, int64_t T, void* X,
                             int64_t ldx, int32_t x_dtype) {
  try {
    if (!p) return IHSBIN_EINVAL;
    if (T < 0 || T > kNoallocMaxT || (T > 0 && (!lambdas || !X))) return IHSBIN_EINVAL;
    if (ldx < p->K || (x_dtype != IHSBIN_F32 && x_dtype != IHSBIN_F64)) return IHSBIN_EINVAL;
    if (!p->plan_ptr()) return IHSBIN_EINVAL;
    if (T == 0) return IHSBIN_OK;
    const double slack = 1e-12;
    for (int64_t t = 0; t < T; ++t) {
      const double lam = lambdas[t];
      if (!(lam >= p->lam_min * (1 - slack)) || !(lam <= p->lam_max * (1 + slack)))
        return IHSBIN_ERANGE;
    }
    DeviceGuard dg(p->device);
    char* base = static_cast<char*>(noalloc_scratch(p->device));
    double* lam_d = reinterpret_cast<double*>(base);
    EvalItem* items = reinterpret_cast<EvalItem*>(base + kNoallocItemsOffset);
    IHS_HIP(hipMemcpyAsync(lam_d, lambdas, sizeof(double) * (size_t)T, hipMemcpyHostToDevice,
                           p->stream));
    int64_t blocks = cdiv(T, 256);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(noalloc_items_kernel, dim3((unsigned)blocks), dim3(256), 0, p->stream, lam_d,
                       T, p->plan_ptr(), p->L, items);
    IHS_CHECK_LAUNCH();
    launch_eval(p->basis_ptr(), p->kcap, p->d, p->K, items, T, X, ldx, x_dtype, p->stream);
    IHS_HIP(hipStreamSynchronize(p->stream));
    return IHSBIN_OK;
  } catch (const Error& e) {
    return e.status;
  } catch (...) {
    return IHSBIN_EHIP;
  }
}
