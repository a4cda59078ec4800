// Request server: continuous batching of kernel-sum requests on one GPU.
//
// Requests (a forward sum, optionally followed by its backward) are queued by
// ksum_server_submit and started by a worker thread as soon as an execution slot
// (a HIP stream) is free and their workspace fits the server's HBM arena, so
// requests that arrive while others run are admitted as slots and memory free
// up and execute concurrently with them.  Plans are made once per distinct
// (d, P, kernel, parameters) and kept, with their directions and tables resident.
// Every kernel of the library is deterministic, so a request's result does not
// depend on what runs beside it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "internal.h"

namespace ksum {
namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

// First-fit sub-allocator over one device allocation (offsets 256-byte aligned,
// neighbouring free blocks merged on release).
class Arena {
 public:
  bool init(size_t bytes) {
    size_ = bytes;
    if (hipMalloc(&base_, bytes) != hipSuccess) {
      base_ = nullptr;
      return false;
    }
    free_[0] = bytes;
    return true;
  }
  void release() {
    if (base_) (void)hipFree(base_);
    base_ = nullptr;
  }
  size_t size() const { return size_; }
  // returns the offset, or SIZE_MAX when no free block is large enough
  size_t alloc(size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_ += bytes;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void free(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  char *ptr(size_t off) const { return static_cast<char *>(base_) + off; }
  size_t used() const { return used_; }

 private:
  void *base_ = nullptr;
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

// A plan is shared by requests whose (d, P, kernel) and parameter fields agree; the
// fields are compared one by one (a struct's padding bytes carry no value).  The
// directions pointer and the device are not part of a request's plan.
struct PlanKey {
  int32_t d, P, kernel;
  ksum_params params;
  auto fields() const {
    const ksum_params &q = params;
    return std::make_tuple(d, P, kernel, q.sigma, q.seed, q.n_coeff, q.coeff_eps, q.T, q.oversample, q.window_m,
                           q.method, q.precision, q.slice_batch, q.check_finite);
  }
  bool operator<(const PlanKey &o) const { return fields() < o.fields(); }
};

struct Pending {
  ksum_request req;
  double t_submit;
  int skipped;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  Pending job{};
  size_t off = 0, bytes = 0;
  double t_start = 0;
  int32_t status = 0;
};

}  // namespace
}  // namespace ksum

using namespace ksum;

struct ksum_server {
  int32_t device = 0;
  std::vector<Slot> slots;
  Arena arena;
  std::map<PlanKey, ksum_plan *> plans;
  std::list<Pending> queue;
  std::vector<ksum_completion> done;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  size_t peak = 0;
  int64_t submitted = 0, finished = 0;

  ksum_plan *plan_for(const ksum_request &r, int32_t *status) {
    PlanKey k{r.d, r.P, (int32_t)r.kernel, r.params};
    k.params.directions = nullptr;
    auto it = plans.find(k);
    if (it != plans.end()) return it->second;
    ksum_params p = r.params;
    p.directions = nullptr;
    p.device = device;
    ksum_plan *pl = nullptr;
    *status = ksum_plan_create(r.d, r.P, r.kernel, &p, &pl);
    if (*status != KSUM_OK) return nullptr;
    plans[k] = pl;
    return pl;
  }

  // workspace bytes of a request: forward, and backward when gradients are asked for
  static size_t request_bytes(const ksum_plan *pl, const ksum_request &r) {
    size_t f = 0, b = 0;
    if (ksum_workspace_size(pl, r.N, r.M, &f) != KSUM_OK) return SIZE_MAX;
    if (r.grad_s && ksum_backward_workspace_size(pl, r.N, r.M, &b) != KSUM_OK) return SIZE_MAX;
    return std::max(f, b);
  }

  void finish(const Pending &job, int32_t status, double t_start, double t_end, size_t bytes) {
    ksum_completion c{};
    c.tag = job.req.tag;
    c.status = status;
    c.t_submit = job.t_submit;
    c.t_start = t_start;
    c.t_end = t_end;
    c.ws_bytes = bytes;
    done.push_back(c);
    ++finished;
  }

  // Starts queued requests on free slots: first come, first served, except that a
  // request whose workspace does not fit right now lets later ones pass (at most
  // 16 of them, then it blocks the queue until it fits).
  void admit() {
    std::vector<std::list<Pending>::iterator> waiting;
    for (auto qi = queue.begin(); qi != queue.end();) {
      int free_slot = -1;
      for (size_t s = 0; s < slots.size(); ++s)
        if (!slots[s].busy) {
          free_slot = (int)s;
          break;
        }
      if (free_slot < 0) return;
      int32_t st = KSUM_OK;
      ksum_plan *pl = plan_for(qi->req, &st);
      if (!pl) {
        finish(*qi, st, now_s(), now_s(), 0);
        qi = queue.erase(qi);
        continue;
      }
      const size_t bytes = request_bytes(pl, qi->req);
      if (bytes == SIZE_MAX || bytes > arena.size()) {
        finish(*qi, bytes == SIZE_MAX ? KSUM_EINVAL : KSUM_ENOMEM, now_s(), now_s(), bytes);
        qi = queue.erase(qi);
        continue;
      }
      const size_t off = arena.alloc(bytes);
      if (off == SIZE_MAX) {
        waiting.push_back(qi);
        ++qi;
        continue;
      }
      for (auto &wq : waiting) {
        if (wq->skipped >= 16) {          // would pass a request that may not be passed again
          arena.free(off, bytes);
          return;
        }
      }
      for (auto &wq : waiting) ++wq->skipped;
      Slot &sl = slots[free_slot];
      sl.busy = true;
      sl.job = *qi;
      sl.off = off;
      sl.bytes = bytes;
      sl.t_start = now_s();
      const ksum_request &r = sl.job.req;
      void *ws = arena.ptr(off);
      int32_t status = KSUM_OK;
      // the inputs are complete once the caller's event has fired
      if (r.ready_event && hipStreamWaitEvent(sl.stream, static_cast<hipEvent_t>(r.ready_event), 0) != hipSuccess)
        status = KSUM_EDEVICE;
      if (status == KSUM_OK)
        status = ksum_execute(pl, r.x, r.N, r.y, r.M, r.w, r.s, ws, bytes, sl.stream);
      if (status == KSUM_OK && r.grad_s)
        status = ksum_backward(pl, r.x, r.N, r.y, r.M, r.w, r.grad_s, r.grad_x, r.grad_y, r.grad_w, ws, bytes,
                               sl.stream);
      sl.status = status;
      if (hipEventRecord(sl.done, sl.stream) != hipSuccess && sl.status == KSUM_OK) sl.status = KSUM_EDEVICE;
      peak = std::max(peak, arena.used());
      qi = queue.erase(qi);
    }
  }

  bool reap() {
    bool any = false;
    for (auto &sl : slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      const int32_t status = (q == hipSuccess) ? sl.status : KSUM_EDEVICE;
      finish(sl.job, status, sl.t_start, now_s(), sl.bytes);
      arena.free(sl.off, sl.bytes);
      sl.busy = false;
      any = true;
    }
    return any;
  }

  bool idle() const {
    if (!queue.empty()) return false;
    for (const auto &sl : slots)
      if (sl.busy) return false;
    return true;
  }

  void run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      reap();
      admit();
      if (stop && idle()) break;
      if (idle()) {
        cv.notify_all();
        cv.wait(lk, [&] { return stop || !queue.empty(); });
      } else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      }
    }
    cv.notify_all();
  }
};

extern "C" {

ksum_status ksum_server_create(int32_t device, int32_t slots, size_t hbm_bytes, ksum_server **out) {
  if (!out) return KSUM_EINVAL;
  *out = nullptr;
  if (slots < 1 || slots > 64 || hbm_bytes < 4096 || device < 0) {
    set_error("slots must be in [1, 64], hbm_bytes >= 4096, device >= 0");
    return KSUM_EINVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= device) {
    set_error("no HIP device with the requested ordinal");
    return KSUM_EDEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) return KSUM_EDEVICE;
  ksum_server *sv = new (std::nothrow) ksum_server();
  if (!sv) return KSUM_ENOMEM;
  sv->device = device;
  if (!sv->arena.init(hbm_bytes)) {
    delete sv;
    set_error("could not allocate the server arena");
    return KSUM_ENOMEM;
  }
  sv->slots.resize(slots);
  for (auto &sl : sv->slots) {
    // non-blocking streams at the default priority: plan creation on the worker
    // (synchronous copies on the null stream) does not wait for running requests
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      set_error("could not create streams");
      ksum_server_destroy(sv);
      return KSUM_EDEVICE;
    }
  }
  sv->worker = std::thread([sv] { sv->run(); });
  *out = sv;
  return KSUM_OK;
}

ksum_status ksum_server_submit(ksum_server *sv, const ksum_request *req) {
  if (!sv || !req) return KSUM_EINVAL;
  if (!req->x || !req->y || !req->w || !req->s || req->N < 1 || req->M < 1) {
    set_error("request needs x, y, w, s and N, M >= 1");
    return KSUM_EINVAL;
  }
  const ksum_status st = ksum_check_params(req->d, req->P, req->kernel, &req->params);
  if (st != KSUM_OK) return st;
  std::lock_guard<std::mutex> lk(sv->mu);
  Pending p{};
  p.req = *req;
  p.req.params.directions = nullptr;
  p.t_submit = now_s();
  sv->queue.push_back(p);
  ++sv->submitted;
  sv->cv.notify_all();
  return KSUM_OK;
}

ksum_status ksum_server_poll(ksum_server *sv, ksum_completion *out, int32_t max_out, int32_t *n_out) {
  if (!sv || !n_out || (max_out > 0 && !out)) return KSUM_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  const int32_t n = (int32_t)std::min<size_t>(sv->done.size(), (size_t)std::max(max_out, 0));
  for (int32_t i = 0; i < n; ++i) out[i] = sv->done[i];
  sv->done.erase(sv->done.begin(), sv->done.begin() + n);
  *n_out = n;
  return KSUM_OK;
}

ksum_status ksum_server_drain(ksum_server *sv) {
  if (!sv) return KSUM_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cv.wait(lk, [&] { return sv->idle(); });
  return KSUM_OK;
}

ksum_status ksum_server_stats(ksum_server *sv, ksum_server_info *info) {
  if (!sv || !info) return KSUM_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  info->submitted = sv->submitted;
  info->finished = sv->finished;
  info->queued = (int64_t)sv->queue.size();
  int64_t running = 0;
  for (const auto &sl : sv->slots) running += sl.busy ? 1 : 0;
  info->running = running;
  info->arena_bytes = sv->arena.size();
  info->arena_used = sv->arena.used();
  info->arena_peak = sv->peak;
  info->plans = (int64_t)sv->plans.size();
  return KSUM_OK;
}

ksum_status ksum_server_destroy(ksum_server *sv) {
  if (!sv) return KSUM_OK;
  if (sv->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stop = true;
      sv->cv.notify_all();
    }
    sv->worker.join();
  }
  for (auto &sl : sv->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  for (auto &kv : sv->plans) ksum_plan_destroy(kv.second);
  sv->arena.release();
  delete sv;
  return KSUM_OK;
}

}  // extern "C"
