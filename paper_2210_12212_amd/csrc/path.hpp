// The path handle of the C ABI: the per-interval plan on the host and the
// basis (and evaluation staging) on the device.
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"

struct ihsbin_path {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t d = 0, K = 0, m_used = 0, kcap = 0;
  int L = 0;
  double lam_min = 0, lam_max = 0;
  int centred = 1;
  int dual = 0;  // built on the dual problem (n < d); the basis is in x-space
  std::vector<double> grid, lam0, tau, rate, ref;
  std::vector<int32_t> k;
  ihs::DevBuf basis, items;
  // the plan on the device for ihsbin_path_eval_noalloc: grid (L + 1
  // doubles), tau (L), ref (L), then k (L int32)
  ihs::DevBuf plan;
  // paths built together (ihsbin_path_build_batch) share one basis and one
  // plan allocation; these are freed with the last of them
  std::shared_ptr<ihs::DevBuf> shared_basis, shared_plan;
  size_t basis_off = 0, plan_off = 0;  // bytes into the shared buffers
  const double* basis_ptr() const {
    return shared_basis ? reinterpret_cast<const double*>(shared_basis->as<char>() + basis_off)
                        : basis.as<double>();
  }
  const char* plan_ptr() const {
    return shared_plan ? shared_plan->as<char>() + plan_off : plan.as<char>();
  }
};

namespace ihs {
// The device address of the allocation-free entry point's scratch array on
// `device` (looked up once per device, with that device current).
void* noalloc_scratch(int device);
}  // namespace ihs
