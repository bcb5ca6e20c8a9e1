// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ihsbin.h"

namespace ihs {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] inline void fail(int status, const std::string& msg) { throw Error(status, msg); }

#define IHS_HIP(call)                                                               \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      ::ihs::fail(e_ == hipErrorOutOfMemory ? IHSBIN_ENOMEM : IHSBIN_EHIP,          \
                  std::string(#call " failed: ") + hipGetErrorString(e_));          \
  } while (0)

#define IHS_CHECK_LAUNCH() IHS_HIP(hipGetLastError())

// ------------------------------------------------------- device buffers
// Device bytes held through one context (its pool and workspaces) and their
// high-water mark.
struct MemStats {
  int64_t live = 0, peak = 0;
  void add(int64_t b) {
    live += b;
    if (live > peak) peak = live;
  }
  void sub(int64_t b) { live -= b; }
};

// Waits until queued work may no longer read a buffer about to be freed: the
// owning stream when one is bound (every user of the buffer runs on it),
// otherwise the whole device.
inline void sync_for_free(bool scoped, hipStream_t s) {
  if (scoped) (void)hipStreamSynchronize(s);
  else (void)hipDeviceSynchronize();
}

// A grow-only device allocation.  Contents are not preserved on growth.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool scoped = false;
  hipStream_t stream = nullptr;
  MemStats* stats = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void bind(hipStream_t s, MemStats* st) {
    scoped = true;
    stream = s;
    stats = st;
  }
  void release() {
    if (p) {
      sync_for_free(scoped, stream);
      (void)hipFree(p);
      if (stats) stats->sub((int64_t)bytes);
    }
    p = nullptr;
    bytes = 0;
  }
  void* ensure(size_t n) {
    if (n <= bytes && p) return p;
    release();
    if (n == 0) n = 256;
    IHS_HIP(hipMalloc(&p, n));
    bytes = n;
    if (stats) stats->add((int64_t)n);
    return p;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Device memory reused across calls on one context.  A block handed back is
// reused by later work on the context's stream without synchronizing: stream
// order puts every earlier reader before the next writer.  Idle memory above
// `keep` bytes is released (after the owning stream, or the device, is idle).
struct Pool {
  static constexpr size_t kKeepBytes = size_t(32) << 30;
  size_t keep = kKeepBytes;
  bool scoped = false;
  hipStream_t stream = nullptr;
  MemStats* stats = nullptr;
  std::multimap<size_t, void*> idle;
  std::map<void*, size_t> block_bytes;
  size_t idle_bytes = 0;
  Pool() = default;
  Pool(const Pool&) = delete;
  Pool& operator=(const Pool&) = delete;
  ~Pool() { release_idle(); }
  void bind(hipStream_t s, MemStats* st) {
    scoped = true;
    stream = s;
    stats = st;
  }
  void* get(size_t n) {
    n = (n + 65535) / 65536 * 65536;
    auto it = idle.lower_bound(n);
    // reuse a block of up to twice the request (or 64 MiB more)
    if (it != idle.end() && (it->first <= 2 * n || it->first <= n + (size_t(64) << 20))) {
      void* p = it->second;
      idle_bytes -= it->first;
      idle.erase(it);
      return p;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, n);
    if (e == hipErrorOutOfMemory && !idle.empty()) {
      (void)hipGetLastError();
      release_idle();
      e = hipMalloc(&p, n);
    }
    if (e != hipSuccess)
      fail(e == hipErrorOutOfMemory ? IHSBIN_ENOMEM : IHSBIN_EHIP,
           std::string("hipMalloc failed: ") + hipGetErrorString(e));
    block_bytes[p] = n;
    if (stats) stats->add((int64_t)n);
    return p;
  }
  void put(void* p) {
    if (!p) return;
    const size_t n = block_bytes[p];
    idle.emplace(n, p);
    idle_bytes += n;
    if (idle_bytes > keep) release_idle();
  }
  void release_idle() {
    if (idle.empty()) return;
    sync_for_free(scoped, stream);
    for (auto& kv : idle) {
      (void)hipFree(kv.second);
      block_bytes.erase(kv.second);
      if (stats) stats->sub((int64_t)kv.first);
    }
    idle.clear();
    idle_bytes = 0;
  }
};
// A grow-only buffer borrowed from a Pool and handed back on destruction.
struct PoolBuf {
  Pool* pool;
  void* p = nullptr;
  size_t bytes = 0;
  explicit PoolBuf(Pool& pl) : pool(&pl) {}
  PoolBuf(const PoolBuf&) = delete;
  PoolBuf& operator=(const PoolBuf&) = delete;
  ~PoolBuf() { pool->put(p); }
  void release() {
    pool->put(p);
    p = nullptr;
    bytes = 0;
  }
  void* ensure(size_t n) {
    if (n <= bytes && p) return p;
    pool->put(p);
    if (n == 0) n = 256;
    p = pool->get(n);
    bytes = n;
    return p;
  }
};

// ------------------------------------------------------------- context
struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  MemStats mem;  // declared before every buffer that reports to it
  // algorithmic bytes of the passes over A and their n x w intermediates
  // since the last reset (the build's bytes_moved)
  double bytes_moved = 0.0;
  Pool pool;     // build-local buffers (declared first: outlives the workspaces below)
  // scratch shared by the step kernels of one call
  DevBuf ws_y, ws_part, ws_small, ws_sketch, ws_tmp, ws_status, ws_f32, ws_ps;
  // a private stream (default priority) that work is captured on into HIP
  // graphs, created on first use and destroyed with the context
  hipStream_t capture_stream = nullptr;
  // every buffer of the context is used on `stream` only
  void bind() {
    pool.bind(stream, &mem);
    for (DevBuf* b : {&ws_y, &ws_part, &ws_small, &ws_sketch, &ws_tmp, &ws_status, &ws_f32, &ws_ps})
      b->bind(stream, &mem);
  }
  // hand idle pool blocks and the workspaces back to the device
  void trim() {
    pool.release_idle();
    for (DevBuf* b : {&ws_y, &ws_part, &ws_small, &ws_sketch, &ws_tmp, &ws_status, &ws_f32, &ws_ps})
      b->release();
  }
};

}  // namespace ihs

// The context handle of the C ABI.
struct ihsbin_ctx {
  ihs::Ctx c;
};

namespace ihs {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    IHS_HIP(hipGetDevice(&prev));
    if (prev != dev) IHS_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// ---------------------------------------------------- SplitMix64 draws
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) in counter form: output i of a
// generator whose state starts at `key` is mix(key + (i + 1) * GAMMA).
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sm_draw(uint64_t key, uint64_t i) {
  return sm_mix(key + (i + 1ull) * kGamma);
}
// Stream keys: output t of SplitMix64(seed).  t = 0 CountSketch/SJLT,
// 1 SRHT signs, 2 SRHT rows, 3 Gaussian entries, 4 Lanczos start vectors.
inline uint64_t stream_key(uint64_t seed, uint64_t t) { return sm_draw(seed, t); }
// Multiply-shift of the top 32 bits into [0, bound).
__host__ __device__ inline uint32_t sm_range(uint64_t x, uint32_t bound) {
  return (uint32_t)(((x >> 32) * (uint64_t)bound) >> 32);
}

// Gaussian sketch entries by Box-Muller: draw pair p = (x1, x2) = (draw 2p,
// draw 2p + 1) gives entry 2p = rho cos(2 pi u2) and entry 2p + 1 =
// rho sin(2 pi u2), rho = sqrt(-2 ln u1), with u1 = (x1 / 2^11 + 1) 2^-53 in
// (0, 1] and u2 = (x2 / 2^11) 2^-53 in [0, 1).  FP64 form:
__device__ inline void box_muller64(uint64_t x1, uint64_t x2, double& zc, double& zs) {
  const double u1 = ((double)(x1 >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(x2 >> 11) * 0x1.0p-53;
  const double rho = sqrt(-2.0 * log(u1));
  const double th = 6.283185307179586476925286766559 * u2;
  zc = rho * cos(th);
  zs = rho * sin(th);
}

// The same pair in FP32, each within a few units in the last place of its
// FP32 rounding: the uniforms' complements are formed exactly in integers, so
// ln u1 near u1 = 1 is log1p of an exact -(1 - u1), and the angle is reduced
// to a quarter turn (and to its complement past an eighth) before FP32 sees it.
__device__ inline void box_muller32(uint64_t x1, uint64_t x2, float& zc, float& zs) {
  const uint64_t k1 = (x1 >> 11) + 1;  // u1 = k1 2^-53
  float lg;
  if (k1 >= (1ull << 52)) {
    lg = ::log1pf(-(float)((1ull << 53) - k1) * 0x1.0p-53f);
  } else {
    lg = ::logf((float)k1 * 0x1.0p-53f);
  }
  const float rho = sqrtf(-2.0f * lg);
  const uint64_t j = x2 >> 11;  // u2 = j 2^-53: quarter q, phi = 2 pi g 2^-53
  const uint32_t q = (uint32_t)(j >> 51);
  const uint64_t g = j & ((1ull << 51) - 1);
  constexpr float kTwoPi53 = 6.28318530717958647692f * 0x1.0p-53f;
  float c, sn;  // cos(phi), sin(phi)
  if (g < (1ull << 50)) {
    const float phi = (float)g * kTwoPi53;
    c = cosf(phi);
    sn = sinf(phi);
  } else {
    const float psi = (float)((1ull << 51) - g) * kTwoPi53;  // pi/2 - phi
    c = sinf(psi);
    sn = cosf(psi);
  }
  // cos and sin of q pi/2 + phi
  zc = rho * (q == 0 ? c : q == 1 ? -sn : q == 2 ? -c : sn);
  zs = rho * (q == 0 ? sn : q == 1 ? c : q == 2 ? -sn : -c);
}

// ------------------------------------------------------------ helpers
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Diagnostic log to stderr, enabled by the environment variable IHSBIN_LOG=1.
bool log_enabled();
void logf(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

struct Csc;
struct HeadTail;
struct MatView {  // a validated ihsbin_matrix
  int format, dtype;
  int64_t n, d, ld, nnz;
  const void* vals;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const Csc* csc = nullptr;  // CSR only, optional: its column-major copy
  const HeadTail* ht = nullptr;  // CSR only, optional: its dense head columns
};

MatView check_matrix(const ihsbin_matrix* A);

// Bytes of one read of A's stored values (and CSR indices).
inline double matrix_bytes(const MatView& A) {
  const double e = A.dtype == IHSBIN_F32 ? 4.0 : 8.0;
  return A.format == IHSBIN_DENSE ? (double)A.n * (double)A.d * e
                                  : (double)A.nnz * (e + 4.0) + 4.0 * (double)(A.n + 1);
}

}  // namespace ihs
