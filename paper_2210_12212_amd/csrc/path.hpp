// The path handle of the C ABI: the per-interval plan on the host and the
// basis (and evaluation staging) on the device.
#pragma once

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
};
