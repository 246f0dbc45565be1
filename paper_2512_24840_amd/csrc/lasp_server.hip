// Fit server (include/lasp.h, lasp_server_*): continuous batching of fit
// requests over one slot pool per spectral shape, admitted by HBM footprint
// against one device-wide budget.  Host code only: every number is computed
// by the pool calls' kernels; this file allocates slots, sizes the pools,
// orders the launches and keeps the request timestamps.
//
// Threading: a worker thread drives the device (admission, steps, finishes,
// completion checks); submit, poll and stats hand requests and results over
// under one mutex.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lasp.h"
#include "lasp_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator of contiguous slot ranges in [0, capacity).
class SlotRanges {
 public:
  explicit SlotRanges(int capacity = 0) : cap_(capacity) {
    if (capacity > 0) free_.push_back({0, capacity});
  }
  int capacity() const { return cap_; }
  int used() const { return used_; }
  // Start of a free range of n slots, or -1.
  int alloc(int n) {
    for (size_t i = 0; i < free_.size(); ++i) {
      if (free_[i].len < n) continue;
      const int s = free_[i].start;
      free_[i].start += n;
      free_[i].len -= n;
      if (free_[i].len == 0) free_.erase(free_.begin() + i);
      used_ += n;
      return s;
    }
    return -1;
  }
  void release(int start, int n) {
    used_ -= n;
    auto it = std::lower_bound(free_.begin(), free_.end(), start,
                               [](const Range &r, int s) { return r.start < s; });
    it = free_.insert(it, Range{start, n});
    merge();
  }
  // One past the last occupied slot.
  int high_water() const {
    if (free_.empty() || free_.back().start + free_.back().len < cap_) return cap_;
    return free_.back().start;
  }
  // New capacity; shrinking requires cap >= high_water().
  void set_capacity(int cap) {
    const int hw = high_water();
    if (!free_.empty() && free_.back().start + free_.back().len == cap_) free_.pop_back();
    if (cap > hw) free_.push_back({hw, cap - hw});
    cap_ = cap;
    merge();
  }

 private:
  struct Range {
    int start, len;
  };
  void merge() {
    std::vector<Range> out;
    for (const Range &r : free_) {
      if (!out.empty() && out.back().start + out.back().len == r.start)
        out.back().len += r.len;
      else
        out.push_back(r);
    }
    free_.swap(out);
  }
  int cap_ = 0, used_ = 0;
  std::vector<Range> free_;
};

struct Request {
  int64_t id = 0;
  int shape = 0, n = 0;
  const float *obs = nullptr, *ivar = nullptr, *init = nullptr;
  float *out_params = nullptr;
  double *out_cov = nullptr, *out_chi2 = nullptr;
  uint32_t *out_status = nullptr;
  int slot0 = -1, steps = 0;
  int64_t admit_tick = -1;
  bool stopped = false;
  double t_submit = 0, t_admit = 0, t_done = 0;
  hipEvent_t done_ev = nullptr;
};

struct Lane {
  lasp_pool *pool = nullptr;
  hipStream_t st = nullptr;
  size_t slot_bytes = 0, fixed_bytes = 0;
  int stop_window = 0;
  bool waits_for_bytes = false;  // head request held back by the budget
  SlotRanges slots;
  std::deque<Request *> queue;
  std::vector<Request *> active, finishing;
  hipEvent_t tick_ev[2] = {nullptr, nullptr};
  int tick_parity = 0;
  bool tick_pending[2] = {false, false};
  // stopping rules: per-slot stopped flags copied to pinned memory, the
  // event marking the copy complete, and the tick the flags were taken at
  int32_t *done_dev = nullptr, *done_host = nullptr;
  int done_cap = 0;
  hipEvent_t snap_ev = nullptr;
  bool snap_pending = false;
  int64_t snap_tick = -1;
};

}  // namespace

struct lasp_server {
  lasp_server_opts o{};
  int device = 0;
  Clock::time_point t0;
  std::vector<Lane> lanes;

  std::mutex mu;
  std::condition_variable work_cv;  // worker: new requests or stop
  std::condition_variable done_cv;  // pollers: a request finished
  std::deque<Request *> incoming;   // submitted, not yet in a lane queue
  std::vector<lasp_request_info> completed;
  bool accepting_shapes = true;
  bool stop = false;
  int err_code = LASP_OK;
  std::string err_msg;
  int64_t next_id = 0, submitted = 0, n_completed = 0;
  std::atomic<int64_t> ticks{0}, resizes{0};
  // worker-side counts published for stats (under mu)
  int32_t n_queued = 0, n_active = 0, n_finishing = 0;
  size_t in_use = 0;
  std::vector<int32_t> cap_pub, used_pub;

  std::thread worker;
};

namespace {

double seconds_since(const lasp_server *s) {
  return std::chrono::duration<double>(Clock::now() - s->t0).count();
}

int round_up(int n, int q) { return (n + q - 1) / q * q; }

size_t pools_bytes(const lasp_server *s) {
  size_t b = 0;
  for (const Lane &l : s->lanes) b += lasp_pool_bytes(l.pool);
  return b;
}

// Records a worker failure (the message of the failing call on this thread).
void worker_fail(lasp_server *s, int code, const char *what) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->err_code == LASP_OK) {
    s->err_code = code;
    s->err_msg = std::string(what) + ": " + lasp_last_error();
  }
  s->done_cv.notify_all();
}

// Resizes a lane's pool (live prefix [0, high water) kept) and its slot map.
int resize_lane(lasp_server *s, Lane &l, int cap) {
  const int hw = l.slots.high_water();
  int rc = lasp_pool_resize(l.pool, cap, std::min(hw, cap));
  if (rc) return rc;
  l.slots.set_capacity(cap);
  s->resizes++;
  return LASP_OK;
}

// The stopped-flag buffers of a lane with the stopping rules on, sized to
// its pool.
int ensure_flag_buffers(Lane &l) {
  const int cap = l.slots.capacity();
  if (l.stop_window == 0 || cap <= l.done_cap) return LASP_OK;
  if (l.done_dev) {
    (void)hipStreamSynchronize(l.st);
    (void)hipFree(l.done_dev);
    (void)hipHostFree(l.done_host);
    l.done_dev = nullptr;
    l.done_host = nullptr;
    l.done_cap = 0;
    l.snap_pending = false;
  }
  if (hipMalloc((void **)&l.done_dev, sizeof(int32_t) * cap) != hipSuccess ||
      hipHostMalloc((void **)&l.done_host, sizeof(int32_t) * cap) != hipSuccess)
    return lasp::set_error(LASP_E_NOMEM, "stopped-flag buffers");
  l.done_cap = cap;
  return LASP_OK;
}

// Tries to place the head request of lane li; may grow the lane's pool
// within the budget.  Returns 1 if admitted, 0 if it must wait, < 0 on error.
int try_admit(lasp_server *s, int li) {
  Lane &l = s->lanes[li];
  Request *r = l.queue.front();
  int slot0 = l.slots.alloc(r->n);
  if (slot0 < 0) {
    // a shape does not grow while another shape's request waits for bytes
    for (int i = 0; i < (int)s->lanes.size(); ++i)
      if (i != li && s->lanes[i].waits_for_bytes) return 0;
    const int q = s->o.capacity_quantum;
    const int need_cap = round_up(l.slots.high_water() + r->n, q);
    const size_t extra = (size_t)(need_cap - l.slots.capacity()) * l.slot_bytes;
    if (pools_bytes(s) + extra > s->o.hbm_budget) return 0;
    int rc = resize_lane(s, l, need_cap);
    if (rc == LASP_E_NOMEM) return 0;  // the device is fuller than the budget says
    if (rc) return rc;
    rc = ensure_flag_buffers(l);
    if (rc) return rc;
    slot0 = l.slots.alloc(r->n);
    if (slot0 < 0) return lasp::set_error(LASP_E_DEVICE, "slot map after growth");
  }
  int rc = lasp_pool_load(l.pool, slot0, r->n, r->obs, r->ivar, r->init, s->o.n_steps);
  if (rc) {
    l.slots.release(slot0, r->n);
    return rc;
  }
  l.queue.pop_front();
  r->slot0 = slot0;
  r->t_admit = seconds_since(s);
  r->admit_tick = s->ticks;
  l.active.push_back(r);
  return 1;
}

// Gives back the unused top of every pool other than `except` (in quanta).
int shrink_others(lasp_server *s, int except) {
  const int q = s->o.capacity_quantum;
  for (int i = 0; i < (int)s->lanes.size(); ++i) {
    if (i == except) continue;
    Lane &l = s->lanes[i];
    const int target = std::max(q, round_up(l.slots.high_water(), q));
    if (target < l.slots.capacity()) {
      int rc = resize_lane(s, l, target);
      if (rc) return rc;
    }
  }
  return LASP_OK;
}

// Enqueues the evaluation of a finished request into the caller's outputs.
int finish_request(lasp_server *s, Lane &l, Request *r) {
  int rc = lasp_pool_finish(l.pool, r->slot0, r->n, r->out_params, s->o.want_cov ? r->out_cov : nullptr,
                            r->out_status, r->out_chi2);
  if (rc) return rc;
  hipError_t e = hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(r->done_ev, l.st);
  if (e != hipSuccess) return lasp::set_error(LASP_E_DEVICE, hipGetErrorString(e));
  l.finishing.push_back(r);
  return LASP_OK;
}

// One tick: admission, one launch sequence per shape, finished requests.
int tick(lasp_server *s) {
  // admission, per shape in arrival order; a shape whose head waits for
  // bytes makes the other pools give back their unused tops
  for (int li = 0; li < (int)s->lanes.size(); ++li) {
    Lane &l = s->lanes[li];
    bool shrunk = false;
    l.waits_for_bytes = false;
    while (!l.queue.empty()) {
      int rc = try_admit(s, li);
      if (rc < 0) return rc;
      if (rc == 1) continue;
      if (shrunk) {
        l.waits_for_bytes = true;
        break;
      }
      rc = shrink_others(s, li);
      if (rc) return rc;
      shrunk = true;
    }
  }
  for (Lane &l : s->lanes) {
    if (l.active.empty()) continue;
    int remaining = 0;
    for (Request *r : l.active) remaining = std::max(remaining, s->o.n_steps - r->steps);
    const int k = std::min(s->o.steps_per_tick, remaining);
    int rc = lasp_pool_step(l.pool, l.slots.high_water(), k);
    if (rc) return rc;
    for (Request *r : l.active) r->steps += k;
    std::vector<Request *> fin;
    for (Request *r : l.active)
      if (r->steps >= s->o.n_steps) fin.push_back(r);
    // stopping rules: requests whose fits have all stopped, from flags taken
    // at an earlier tick (only for requests admitted before those flags)
    if (l.snap_pending && hipEventQuery(l.snap_ev) == hipSuccess) {
      for (Request *r : l.active) {
        if (r->steps >= s->o.n_steps || r->admit_tick > l.snap_tick) continue;
        bool all = true;
        for (int i = 0; i < r->n && all; ++i) all = l.done_host[r->slot0 + i] != 0;
        if (all) {
          r->stopped = true;
          fin.push_back(r);
        }
      }
      l.snap_pending = false;
    }
    for (Request *r : fin) {
      l.active.erase(std::find(l.active.begin(), l.active.end(), r));
      rc = finish_request(s, l, r);
      if (rc) return rc;
    }
    if (l.stop_window > 0 && !l.snap_pending && !l.active.empty()) {
      const int hw = l.slots.high_water();
      rc = lasp_pool_progress(l.pool, 0, hw, nullptr, l.done_dev);
      if (rc) return rc;
      hipError_t e = hipMemcpyAsync(l.done_host, l.done_dev, sizeof(int32_t) * hw,
                                    hipMemcpyDeviceToHost, l.st);
      if (e == hipSuccess) e = hipEventRecord(l.snap_ev, l.st);
      if (e != hipSuccess) return lasp::set_error(LASP_E_DEVICE, hipGetErrorString(e));
      l.snap_pending = true;
      l.snap_tick = s->ticks;
    }
    // at most two ticks of a lane in flight: wait for the one before last
    const int p = l.tick_parity;
    hipError_t e = hipEventRecord(l.tick_ev[p], l.st);
    if (e != hipSuccess) return lasp::set_error(LASP_E_DEVICE, hipGetErrorString(e));
    l.tick_pending[p] = true;
    l.tick_parity ^= 1;
    if (l.tick_pending[p ^ 1]) {
      e = hipEventSynchronize(l.tick_ev[p ^ 1]);
      if (e != hipSuccess) return lasp::set_error(LASP_E_DEVICE, hipGetErrorString(e));
      l.tick_pending[p ^ 1] = false;
    }
  }
  s->ticks++;
  return LASP_OK;
}

// Reports requests whose outputs are complete on the device and frees their
// slots.  Returns the number reported.
int collect(lasp_server *s) {
  int n = 0;
  for (size_t li = 0; li < s->lanes.size(); ++li) {
    Lane &l = s->lanes[li];
    for (size_t i = 0; i < l.finishing.size();) {
      Request *r = l.finishing[i];
      if (hipEventQuery(r->done_ev) != hipSuccess) {
        ++i;
        continue;
      }
      (void)hipEventDestroy(r->done_ev);
      l.slots.release(r->slot0, r->n);
      r->t_done = seconds_since(s);
      lasp_request_info info{};
      info.id = r->id;
      info.shape = r->shape;
      info.count = r->n;
      info.max_steps = std::min(r->steps, s->o.n_steps);
      info.stopped = r->stopped ? 1 : 0;
      info.t_submit = r->t_submit;
      info.t_admit = r->t_admit;
      info.t_done = r->t_done;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->completed.push_back(info);
        s->n_completed++;
      }
      delete r;
      l.finishing.erase(l.finishing.begin() + i);
      ++n;
    }
  }
  if (n) s->done_cv.notify_all();
  return n;
}

void publish(lasp_server *s) {
  int32_t q = 0, a = 0, f = 0;
  for (const Lane &l : s->lanes) {
    q += (int32_t)l.queue.size();
    a += (int32_t)l.active.size();
    f += (int32_t)l.finishing.size();
  }
  const size_t bytes = pools_bytes(s);
  std::lock_guard<std::mutex> lk(s->mu);
  s->n_queued = q + (int32_t)s->incoming.size();
  s->n_active = a;
  s->n_finishing = f;
  s->in_use = bytes;
  for (size_t i = 0; i < s->lanes.size(); ++i) {
    s->cap_pub[i] = s->lanes[i].slots.capacity();
    s->used_pub[i] = s->lanes[i].slots.used();
  }
}

void worker_main(lasp_server *s) {
  if (hipSetDevice(s->device) != hipSuccess) {
    worker_fail(s, LASP_E_DEVICE, "hipSetDevice");
    return;
  }
  for (;;) {
    {
      // the lane list is fixed once requests arrive; before that it may grow
      // under the lock, so it is read under the lock here
      std::unique_lock<std::mutex> lk(s->mu);
      bool busy = false;
      for (const Lane &l : s->lanes)
        busy = busy || !l.queue.empty() || !l.active.empty() || !l.finishing.empty();
      if (!busy)
        s->work_cv.wait(lk, [s] { return s->stop || !s->incoming.empty(); });
      if (s->stop || s->err_code != LASP_OK) return;
      while (!s->incoming.empty()) {
        Request *r = s->incoming.front();
        s->incoming.pop_front();
        s->lanes[r->shape].queue.push_back(r);
      }
    }
    bool stepping = false;
    for (const Lane &l : s->lanes) stepping = stepping || !l.queue.empty() || !l.active.empty();
    if (stepping) {
      int rc = tick(s);
      if (rc) {
        worker_fail(s, rc, "server tick");
        return;
      }
    }
    const int got = collect(s);
    publish(s);
    if (!stepping && !got) std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

void destroy_lanes(lasp_server *s) {
  for (Lane &l : s->lanes) {
    if (l.st) (void)hipStreamSynchronize(l.st);
    for (Request *r : l.queue) delete r;
    for (Request *r : l.active) delete r;
    for (Request *r : l.finishing) {
      if (r->done_ev) (void)hipEventDestroy(r->done_ev);
      delete r;
    }
    if (l.pool) (void)lasp_pool_destroy(l.pool);
    for (hipEvent_t e : l.tick_ev)
      if (e) (void)hipEventDestroy(e);
    if (l.snap_ev) (void)hipEventDestroy(l.snap_ev);
    if (l.done_dev) (void)hipFree(l.done_dev);
    if (l.done_host) (void)hipHostFree(l.done_host);
    if (l.st) (void)hipStreamDestroy(l.st);
  }
  s->lanes.clear();
  for (Request *r : s->incoming) delete r;
  s->incoming.clear();
}

}  // namespace

extern "C" {

void lasp_server_default_opts(lasp_server_opts *o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->hbm_budget = 0;
  o->n_steps = 500;
  o->steps_per_tick = 25;
  o->want_cov = 0;
  o->capacity_quantum = 1024;
}

int lasp_server_create(const lasp_server_opts *opts, lasp_server **out) {
  if (!out) return lasp::set_error(LASP_E_ARG, "out is NULL");
  *out = nullptr;
  if (!opts) return lasp::set_error(LASP_E_ARG, "opts is NULL");
  if (opts->n_steps < 0 || opts->steps_per_tick < 1 || opts->capacity_quantum < 1)
    return lasp::set_error(LASP_E_ARG, "need n_steps >= 0, steps_per_tick >= 1, capacity_quantum >= 1");
  lasp_server *s = new lasp_server();
  s->o = *opts;
  s->t0 = Clock::now();
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess && s->o.hbm_budget == 0) {
    size_t free_b = 0, total_b = 0;
    e = hipMemGetInfo(&free_b, &total_b);
    s->o.hbm_budget = free_b / 4 * 3;
  }
  if (e != hipSuccess) {
    delete s;
    return lasp::set_error(LASP_E_DEVICE, hipGetErrorString(e));
  }
  s->lanes.reserve(LASP_SERVER_MAX_SHAPES);
  s->worker = std::thread(worker_main, s);
  *out = s;
  return LASP_OK;
}

int lasp_server_add_shape(lasp_server *s, const double *wave_grid, const float *basis,
                          const lasp_opts *opts, int32_t *shape_id) {
  if (!s || !opts || !shape_id) return lasp::set_error(LASP_E_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->accepting_shapes) return lasp::set_error(LASP_E_ARG, "shapes must be added before the first submit");
  if ((int)s->lanes.size() >= LASP_SERVER_MAX_SHAPES)
    return lasp::set_error(LASP_E_ARG, "too many shapes");
  lasp_opts po = *opts;
  po.n_spec = s->o.capacity_quantum;
  po.status = nullptr;
  po.out_chi2 = nullptr;
  po.out_steps = nullptr;
  po.out_mask = nullptr;
  po.polish_iters = 0;
  po.clean_every = 0;
  Lane l;
  l.slot_bytes = lasp_pool_slot_bytes(&po, wave_grid);
  if (l.slot_bytes == 0) return lasp::set_error(LASP_E_ARG, "invalid shape options");
  l.stop_window = po.stop_window;
  const size_t have = pools_bytes(s);
  hipError_t e = hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking);
  for (int k = 0; e == hipSuccess && k < 2; ++k)
    e = hipEventCreateWithFlags(&l.tick_ev[k], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&l.snap_ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    for (hipEvent_t ev : l.tick_ev)
      if (ev) (void)hipEventDestroy(ev);
    if (l.snap_ev) (void)hipEventDestroy(l.snap_ev);
    if (l.st) (void)hipStreamDestroy(l.st);
    return lasp::set_error(LASP_E_DEVICE, hipGetErrorString(e));
  }
  po.stream = l.st;
  int rc = lasp_pool_create(wave_grid, basis, &po, &l.pool);
  if (rc == LASP_OK && have + lasp_pool_bytes(l.pool) > s->o.hbm_budget) {
    (void)lasp_pool_destroy(l.pool);
    l.pool = nullptr;
    rc = lasp::set_error(LASP_E_NOMEM, "the shape's first slots exceed the server's HBM budget");
  }
  if (rc == LASP_OK) {
    l.slots = SlotRanges(po.n_spec);
    l.fixed_bytes = lasp_pool_bytes(l.pool) - (size_t)po.n_spec * l.slot_bytes;
    rc = ensure_flag_buffers(l);
  }
  if (rc) {
    std::string msg = lasp_last_error();
    if (l.pool) (void)lasp_pool_destroy(l.pool);
    for (hipEvent_t ev : l.tick_ev) (void)hipEventDestroy(ev);
    (void)hipEventDestroy(l.snap_ev);
    if (l.done_dev) (void)hipFree(l.done_dev);
    if (l.done_host) (void)hipHostFree(l.done_host);
    (void)hipStreamDestroy(l.st);
    return lasp::set_error(rc, msg.c_str());
  }
  // stream-ordered pool set-up finished before the worker may use it
  e = hipStreamSynchronize(l.st);
  *shape_id = (int32_t)s->lanes.size();
  s->lanes.push_back(l);
  s->cap_pub.push_back(l.slots.capacity());
  s->used_pub.push_back(0);
  s->in_use = pools_bytes(s);
  if (e != hipSuccess) return lasp::set_error(LASP_E_DEVICE, hipGetErrorString(e));
  return LASP_OK;
}

int lasp_server_submit(lasp_server *s, int32_t shape, int32_t count, const float *obs,
                       const float *ivar, const float *init_params, float *out_params,
                       double *out_cov, uint32_t *out_status, double *out_chi2,
                       int64_t *request_id) {
  if (!s || !obs || !ivar || !init_params || !out_params || !request_id)
    return lasp::set_error(LASP_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->err_code) return lasp::set_error(s->err_code, s->err_msg.c_str());
  if (shape < 0 || shape >= (int)s->lanes.size()) return lasp::set_error(LASP_E_ARG, "unknown shape");
  if (count < 1) return lasp::set_error(LASP_E_ARG, "count must be >= 1");
  if (s->o.want_cov && !out_cov) return lasp::set_error(LASP_E_ARG, "want_cov needs out_cov");
  // the largest pool this shape can ever have: the budget less the other
  // shapes' smallest pools (one quantum each) and its own fixed part
  // (slot and fixed bytes are set when a shape is added and never change)
  const Lane &l = s->lanes[shape];
  size_t others = 0;
  for (int i = 0; i < (int)s->lanes.size(); ++i) {
    if (i == shape) continue;
    const Lane &o = s->lanes[i];
    others += o.fixed_bytes + (size_t)s->o.capacity_quantum * o.slot_bytes;
  }
  const size_t room =
      s->o.hbm_budget > others + l.fixed_bytes ? s->o.hbm_budget - others - l.fixed_bytes : 0;
  const size_t max_slots = room / l.slot_bytes / s->o.capacity_quantum * s->o.capacity_quantum;
  if ((size_t)count > max_slots) {
    char buf[200];
    snprintf(buf, sizeof buf, "a request of %d spectra can never fit the HBM budget (at most %zu "
             "of this shape)", count, max_slots);
    return lasp::set_error(LASP_E_NOMEM, buf);
  }
  Request *r = new Request();
  r->id = s->next_id++;
  r->shape = shape;
  r->n = count;
  r->obs = obs;
  r->ivar = ivar;
  r->init = init_params;
  r->out_params = out_params;
  r->out_cov = out_cov;
  r->out_status = out_status;
  r->out_chi2 = out_chi2;
  r->t_submit = seconds_since(s);
  s->incoming.push_back(r);
  s->accepting_shapes = false;
  s->submitted++;
  s->n_queued++;
  *request_id = r->id;
  s->work_cv.notify_one();
  return LASP_OK;
}

int lasp_server_poll(lasp_server *s, lasp_request_info *done, int32_t max_done,
                     int32_t timeout_ms, int32_t *n_done) {
  if (!s || !n_done || max_done < 0 || (max_done > 0 && !done))
    return lasp::set_error(LASP_E_ARG, "bad arguments");
  *n_done = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (timeout_ms > 0 && s->completed.empty() && s->err_code == LASP_OK)
    s->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                        [s] { return !s->completed.empty() || s->err_code != LASP_OK; });
  const int n = std::min<int>(max_done, (int)s->completed.size());
  for (int i = 0; i < n; ++i) done[i] = s->completed[i];
  s->completed.erase(s->completed.begin(), s->completed.begin() + n);
  *n_done = n;
  if (s->err_code) return lasp::set_error(s->err_code, s->err_msg.c_str());
  return LASP_OK;
}

int lasp_server_stats(lasp_server *s, lasp_server_counters *st) {
  if (!s || !st) return lasp::set_error(LASP_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  memset(st, 0, sizeof(*st));
  st->hbm_budget = s->o.hbm_budget;
  st->hbm_in_use = s->in_use;
  st->submitted = s->submitted;
  st->completed = s->n_completed;
  st->ticks = s->ticks;
  st->resizes = s->resizes;
  st->queued = s->n_queued;
  st->active = s->n_active;
  st->finishing = s->n_finishing;
  st->n_shapes = (int32_t)s->lanes.size();
  for (size_t i = 0; i < s->lanes.size(); ++i) {
    st->capacity[i] = s->cap_pub[i];
    st->used_slots[i] = s->used_pub[i];
  }
  if (s->err_code) return lasp::set_error(s->err_code, s->err_msg.c_str());
  return LASP_OK;
}

int lasp_server_destroy(lasp_server *s) {
  if (!s) return LASP_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->work_cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(s->device);
  destroy_lanes(s);
  (void)hipSetDevice(cur);
  delete s;
  return LASP_OK;
}

}  // extern "C"
