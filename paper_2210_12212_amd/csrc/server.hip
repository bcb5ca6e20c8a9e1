// Request server: independent path builds run concurrently on one device.
//
// Each worker owns a context with its own stream (default priority), so
// builds of different requests overlap on the device while every single
// build runs exactly the kernels it runs alone.  Requests are admitted in
// arrival order when the sum of the admitted builds' memory estimates
// (ihsbin_build_footprint) stays within the budget; a build that still runs
// out of memory is queued again at the front and then runs alone.  A
// finished build's path is handed to the caller (the basis stays resident
// for later evaluations); its transient memory returns to the worker, which
// keeps at most keep_bytes of it between builds.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "common.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
  int64_t id = 0;
  ihsbin_matrix A{};
  const void* B = nullptr;
  int64_t K = 0, ldb = 0;
  double lam_min = 0, lam_max = 0;
  ihsbin_opts o{};
  std::vector<double> taus;
  ihsbin_alg4_opts a4{};
  bool has_a4 = false;
  int64_t footprint = 0;
  bool exclusive = false;  // run with nothing else in flight (after ENOMEM)
  Clock::time_point t_submit, t_start, t_end;
  bool done = false;
  int status = IHSBIN_OK;
  int worker = -1;
  ihsbin_path* path = nullptr;
  ihsbin_report rep{};
  std::string message;
};

}  // namespace

struct ihsbin_server {
  int device = 0;
  ihsbin_server_opts o{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<int64_t, std::shared_ptr<Request>> open;  // submitted, not yet collected
  int64_t next_id = 1;
  int64_t inflight_bytes = 0;
  int inflight = 0;
  bool stop = false;
  ihsbin_server_stats st{};
  std::string last_error;
  std::vector<std::thread> threads;
  std::vector<ihsbin_ctx*> ctxs;
  std::vector<hipStream_t> streams;

  bool fits(const Request& r) const {
    if (inflight == 0) return true;
    return !r.exclusive && inflight_bytes + r.footprint <= o.hbm_budget;
  }

  void work(int w) {
    (void)hipSetDevice(device);
    ihsbin_ctx* ctx = ctxs[w];
    for (;;) {
      std::shared_ptr<Request> r;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return (stop && queue.empty()) || (!queue.empty() && fits(*queue.front())); });
        if (queue.empty()) return;  // stopping, nothing left
        r = queue.front();
        queue.pop_front();
        inflight_bytes += r->footprint;
        ++inflight;
        st.queued = (int32_t)queue.size();
        if (inflight > st.max_concurrent) st.max_concurrent = inflight;
        if (inflight_bytes > st.max_inflight_bytes) st.max_inflight_bytes = inflight_bytes;
        r->t_start = Clock::now();
        r->worker = w;
      }
      ihsbin_opts bo = r->o;
      bo.taus = r->taus.empty() ? nullptr : r->taus.data();
      bo.alg4 = r->has_a4 ? &r->a4 : nullptr;
      ihsbin_path* p = nullptr;
      ihsbin_report rep;
      std::memset(&rep, 0, sizeof(rep));
      const int rc = ihsbin_path_build(ctx, &r->A, r->B, r->K, r->ldb, r->lam_min, r->lam_max,
                                       &bo, &p, &rep);
      std::string msg = rc == IHSBIN_OK ? "" : ihsbin_last_error(ctx);
      if (ctx->c.mem.live > o.keep_bytes) {
        try {
          ihs::DeviceGuard g(device);
          ctx->c.trim();
        } catch (...) {
        }
      }
      std::lock_guard<std::mutex> lk(mu);
      inflight_bytes -= r->footprint;
      --inflight;
      if (rc == IHSBIN_ENOMEM && !r->exclusive) {
        // the estimate was not enough next to the other builds: run it alone
        if (p) ihsbin_path_free(p);
        r->exclusive = true;
        queue.push_front(r);
        ++st.retried;
      } else {
        r->t_end = Clock::now();
        r->status = rc;
        r->path = p;
        r->rep = rep;
        r->message = msg;
        r->done = true;
        ++st.completed;
        cv_done.notify_all();
      }
      st.queued = (int32_t)queue.size();
      cv_work.notify_all();
    }
  }
};

void ihsbin_server_opts_default(ihsbin_server_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->workers = 4;
  o->hbm_budget = 0;
  o->keep_bytes = int64_t(1) << 30;
}

int ihsbin_server_create(ihsbin_server** out, int device, const ihsbin_server_opts* opts) {
  if (!out) return IHSBIN_EINVAL;
  *out = nullptr;
  ihsbin_server_opts o;
  if (opts) o = *opts;
  else ihsbin_server_opts_default(&o);
  if (o.workers < 1 || o.workers > 16 || o.hbm_budget < 0 || o.keep_bytes < 0)
    return IHSBIN_EINVAL;
  auto s = std::make_unique<ihsbin_server>();
  try {
    int n = 0;
    IHS_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return IHSBIN_EINVAL;
    ihs::DeviceGuard g(device);
    if (o.hbm_budget == 0) {
      size_t fr = 0, tot = 0;
      IHS_HIP(hipMemGetInfo(&fr, &tot));
      o.hbm_budget = (int64_t)(0.9 * (double)fr);
    }
    s->device = device;
    s->o = o;
    s->st.budget = o.hbm_budget;
    for (int w = 0; w < o.workers; ++w) {
      hipStream_t stm = nullptr;
      IHS_HIP(hipStreamCreateWithFlags(&stm, hipStreamNonBlocking));
      s->streams.push_back(stm);
      ihsbin_ctx* c = nullptr;
      const int rc = ihsbin_create(&c, device, stm);
      if (rc != IHSBIN_OK) ihs::fail(rc, "context creation failed");
      c->c.pool.keep = (size_t)o.keep_bytes;
      s->ctxs.push_back(c);
    }
    for (int w = 0; w < o.workers; ++w) s->threads.emplace_back([p = s.get(), w] { p->work(w); });
  } catch (const ihs::Error& e) {
    for (auto* c : s->ctxs) ihsbin_destroy(c);
    for (auto stm : s->streams) (void)hipStreamDestroy(stm);
    return e.status;
  } catch (...) {
    for (auto* c : s->ctxs) ihsbin_destroy(c);
    for (auto stm : s->streams) (void)hipStreamDestroy(stm);
    return IHSBIN_EHIP;
  }
  *out = s.release();
  return IHSBIN_OK;
}

int ihsbin_server_submit(ihsbin_server* s, const ihsbin_matrix* A, const void* B, int64_t K,
                         int64_t ldb, double lam_min, double lam_max, const ihsbin_opts* opts,
                         int64_t* id) {
  if (!s || !id) return IHSBIN_EINVAL;
  auto r = std::make_shared<Request>();
  try {
    (void)ihs::check_matrix(A);
    if (!B || K < 1 || ldb < K) ihs::fail(IHSBIN_EINVAL, "need B, K >= 1 and ldb >= K");
    if (opts) r->o = *opts;
    else ihsbin_opts_default(&r->o);
    const int rc = ihsbin_build_footprint(A, K, lam_min, lam_max, &r->o, &r->footprint);
    if (rc != IHSBIN_OK) ihs::fail(rc, "bad request (shape, lambda range or options)");
    if (r->footprint > s->o.hbm_budget)
      ihs::fail(IHSBIN_ENOMEM, "request needs more device memory than the server's budget");
    if (r->o.taus) {
      const double beta = lam_max / lam_min;
      const int L = r->o.L > 0 ? r->o.L
                               : (beta > 1.0 ? std::max(1, (int)std::floor(2.0 * std::log(beta))) : 1);
      r->taus.assign(r->o.taus, r->o.taus + L);
    }
    if (r->o.alg4) {
      r->a4 = *r->o.alg4;
      r->has_a4 = true;
    }
  } catch (const ihs::Error& e) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->last_error = e.what();
    return e.status;
  }
  r->A = *A;
  r->B = B;
  r->K = K;
  r->ldb = ldb;
  r->lam_min = lam_min;
  r->lam_max = lam_max;
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return IHSBIN_EINVAL;
  r->id = s->next_id++;
  *id = r->id;
  s->open[r->id] = r;
  s->queue.push_back(r);
  ++s->st.submitted;
  s->st.queued = (int32_t)s->queue.size();
  s->cv_work.notify_all();
  return IHSBIN_OK;
}

int ihsbin_server_wait(ihsbin_server* s, int64_t id, int64_t timeout_ms, void* stream,
                       ihsbin_path** path, ihsbin_request_info* info) {
  if (!s) return IHSBIN_EINVAL;
  if (path) *path = nullptr;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->open.find(id);
  if (it == s->open.end()) return IHSBIN_EINVAL;
  std::shared_ptr<Request> r = it->second;
  auto ready = [&] { return r->done; };
  if (timeout_ms < 0) s->cv_done.wait(lk, ready);
  else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
    return IHSBIN_EAGAIN;
  s->open.erase(it);
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = r->status;
    info->worker = r->worker;
    info->footprint = r->footprint;
    info->ms_queue = ms_between(r->t_submit, r->t_start);
    info->ms_build = ms_between(r->t_start, r->t_end);
    info->ms_total = ms_between(r->t_submit, r->t_end);
    info->report = r->rep;
    std::strncpy(info->message, r->message.c_str(), sizeof(info->message) - 1);
  }
  if (r->path && path) {
    // the worker's stream runs other builds from now on
    const int rc = ihsbin_path_set_stream(r->path, stream);
    if (rc != IHSBIN_OK) {
      ihsbin_path_free(r->path);
      return rc;
    }
    *path = r->path;
  } else if (r->path) {
    ihsbin_path_free(r->path);
  }
  return r->status;
}

int ihsbin_server_get_stats(ihsbin_server* s, ihsbin_server_stats* out) {
  if (!s || !out) return IHSBIN_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->workers = s->o.workers;
  out->inflight = s->inflight;
  out->inflight_bytes = s->inflight_bytes;
  return IHSBIN_OK;
}

const char* ihsbin_server_last_error(ihsbin_server* s) {
  if (!s) return "";
  std::lock_guard<std::mutex> lk(s->mu);
  return s->last_error.c_str();
}

int ihsbin_server_destroy(ihsbin_server* s) {
  if (!s) return IHSBIN_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  for (auto& t : s->threads) t.join();
  for (auto& kv : s->open)
    if (kv.second->path) ihsbin_path_free(kv.second->path);
  s->open.clear();
  for (auto* c : s->ctxs) ihsbin_destroy(c);
  for (auto stm : s->streams) (void)hipStreamDestroy(stm);
  delete s;
  return IHSBIN_OK;
}
