// Serving loop: the continuous-batching scheduler (pinv_sched.h) driving
// libpinv on the device.  Builds run on one HIP stream, grouped applies on
// another, so new builds overlap with the applies of requests whose plans
// are cached.  A worker thread ticks the scheduler; callers submit requests
// and poll completions from any thread.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pinv.h"
#include "pinv_sched.h"

// Library-internal (pinv_api.hip): scratch and build workspaces back to the
// device when memory is short; the device's build and apply streams for
// serving, created once per process.
void pinv_context_trim_scratch(pinv_context* c);
bool pinv_serving_streams(int device, hipStream_t* build, hipStream_t* apply);

namespace {

// An encoding with its arrays copied (requests outlive the caller's buffers).
struct OwnedEncoding {
  pinv_encoding e{};
  std::vector<double> k, t, coil, b0, species;
  std::vector<int32_t> vox;
  explicit OwnedEncoding(const pinv_encoding& s) {
    e = s;
    const size_t V = (size_t)s.nx * s.ny;
    k.assign(s.k, s.k + 2 * (size_t)s.nk);
    e.k = k.data();
    if (s.t) {
      t.assign(s.t, s.t + (size_t)s.nk);
      e.t = t.data();
    }
    if (s.coil) {
      coil.assign(s.coil, s.coil + 2 * (size_t)s.ncoil * V);
      e.coil = coil.data();
    }
    if (s.b0_hz) {
      b0.assign(s.b0_hz, s.b0_hz + V);
      e.b0_hz = b0.data();
    }
    if (s.species_hz) {
      species.assign(s.species_hz, s.species_hz + s.nspecies);
      e.species_hz = species.data();
    }
    if (s.voxels && s.nvox > 0) {
      vox.assign(s.voxels, s.voxels + s.nvox);
      e.voxels = vox.data();
    }
  }
};

struct HipBackend {
  struct Request {
    std::shared_ptr<OwnedEncoding> enc;
    pinv_build_opts opts{};
    const void* data = nullptr;
    void* image = nullptr;
    int64_t F = 0;
    int32_t refine = 0;
  };
  typedef pinv_plan* PlanHandle;
  struct BatchHandle {
    hipEvent_t ev = nullptr;
  };
  typedef pinv_sched::Scheduler<HipBackend>::Item Item;

  pinv_context* ctx = nullptr;
  hipStream_t build_stream = nullptr, apply_stream = nullptr;

  int start_build(const Request& r, pinv_plan** h) {
    pinv_build_opts o = r.opts;
    o.flags |= PINV_FLAG_UNCACHED;
    const pinv_status s = pinv_build(ctx, &r.enc->e, &o, build_stream, h);
    if (s != PINV_OK) fprintf(stderr, "pinv server: build failed: %s\n", pinv_last_error());
    return s;
  }
  int build_state(pinv_plan* h) {
    const pinv_status s = pinv_plan_query(h);
    if (s != PINV_OK && s != PINV_ERR_BUSY)
      fprintf(stderr, "pinv server: build failed: %s\n", pinv_last_error());
    return s;
  }
  size_t resident_bytes(pinv_plan* h) {
    pinv_plan_info i;
    return pinv_plan_info_get(h, &i) == PINV_OK ? i.device_bytes : 0;
  }
  int apply(const std::vector<Item>& items, BatchHandle* b) {
    // one grouped call per run of equal refinement steps
    size_t i = 0;
    while (i < items.size()) {
      const int32_t refine = items[i].req->refine;
      std::vector<pinv_apply_item> v;
      while (i < items.size() && items[i].req->refine == refine) {
        v.push_back(pinv_apply_item{items[i].plan, items[i].req->data, items[i].req->image,
                                    items[i].req->F});
        ++i;
      }
      const pinv_status s = pinv_apply_grouped(ctx, (int32_t)v.size(), v.data(), refine, apply_stream);
      if (s != PINV_OK) {
        fprintf(stderr, "pinv server: apply failed: %s\n", pinv_last_error());
        return s;
      }
    }
    if (hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) return PINV_ERR_DEVICE;
    if (hipEventRecord(b->ev, apply_stream) != hipSuccess) return PINV_ERR_DEVICE;
    return 0;
  }
  bool batch_done(BatchHandle& b) {
    const hipError_t q = hipEventQuery(b.ev);
    if (q == hipErrorNotReady) return false;
    (void)hipEventDestroy(b.ev);
    b.ev = nullptr;
    pinv_context_trim_scratch(ctx);   // refinement scratch back under memory pressure
    return true;
  }
  void release(pinv_plan* h) { pinv_plan_release(h); }
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct pinv_server {
  pinv_context* ctx = nullptr;
  int device = 0;
  HipBackend be;
  std::unique_ptr<pinv_sched::Scheduler<HipBackend>> sch;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  std::atomic<bool> stop{false};
  std::chrono::steady_clock::time_point t0;
};

static void worker_loop(pinv_server* s) {
  (void)hipSetDevice(s->device);
  while (!s->stop.load()) {
    bool idle;
    {
      std::lock_guard<std::mutex> g(s->mu);
      s->sch->tick(seconds_since(s->t0));
      idle = s->sch->idle();
    }
    if (idle) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait_for(lk, std::chrono::milliseconds(20));
    } else {
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
  }
}

extern "C" {

pinv_status pinv_server_create(pinv_context* ctx, int device, const pinv_server_opts* o,
                               pinv_server** out) {
  if (!ctx || !o || !out) return PINV_ERR_INVALID;
  if (o->max_group < 1 || o->max_inflight < 1 || o->max_builds < 1 || o->hbm_budget_bytes == 0)
    return PINV_ERR_INVALID;
  if (hipSetDevice(device) != hipSuccess) return PINV_ERR_DEVICE;
  pinv_server* s = new pinv_server();
  s->ctx = ctx;
  s->device = device;
  s->be.ctx = ctx;
  if (!pinv_serving_streams(device, &s->be.build_stream, &s->be.apply_stream)) {
    delete s;
    return PINV_ERR_DEVICE;
  }
  pinv_sched::Options so;
  so.budget = o->hbm_budget_bytes;
  so.max_group = std::min<int>(o->max_group, 32);
  so.max_inflight = o->max_inflight;
  so.max_builds = o->max_builds;
  s->sch.reset(new pinv_sched::Scheduler<HipBackend>(&s->be, so));
  s->t0 = std::chrono::steady_clock::now();
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return PINV_OK;
}

pinv_status pinv_server_submit(pinv_server* s, const pinv_request* r, uint64_t* ticket) {
  if (!s || !r || !r->enc) return PINV_ERR_INVALID;
  if (r->F < 0 || (r->F > 0 && (!r->data || !r->image)) || r->refine_steps < 0 ||
      r->refine_steps > 4)
    return PINV_ERR_INVALID;
  uint64_t key = 0;
  size_t foot = 0;
  const pinv_status st = pinv_encoding_key(r->enc, &r->opts, &key, &foot);
  if (st != PINV_OK) return st;
  HipBackend::Request q;
  q.enc = std::make_shared<OwnedEncoding>(*r->enc);
  q.opts = r->opts;
  q.data = r->data;
  q.image = r->image;
  q.F = r->F;
  q.refine = r->refine_steps;
  uint64_t t;
  {
    std::lock_guard<std::mutex> g(s->mu);
    t = s->sch->submit(key, foot, q, r->tag, seconds_since(s->t0));
  }
  s->cv.notify_one();
  if (ticket) *ticket = t;
  return PINV_OK;
}

pinv_status pinv_server_poll(pinv_server* s, pinv_completion* out, int32_t max, int32_t* n) {
  if (!s || (max > 0 && !out) || !n) return PINV_ERR_INVALID;
  std::vector<pinv_sched::Completion> c;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->sch->take_completions(&c, (size_t)std::max(0, max));
  }
  for (size_t i = 0; i < c.size(); ++i)
    out[i] = pinv_completion{c[i].ticket, c[i].tag, c[i].status, c[i].built,
                             c[i].t_arrival, c[i].t_dispatch, c[i].t_done};
  *n = (int32_t)c.size();
  return PINV_OK;
}

pinv_status pinv_server_drain(pinv_server* s, double timeout_s) {
  if (!s) return PINV_ERR_INVALID;
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    {
      std::lock_guard<std::mutex> g(s->mu);
      if (s->sch->idle()) return PINV_OK;
    }
    if (timeout_s > 0 && seconds_since(t0) > timeout_s) return PINV_ERR_BUSY;
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
}

pinv_status pinv_server_stats_get(pinv_server* s, pinv_server_stats* out) {
  if (!s || !out) return PINV_ERR_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  const pinv_sched::Stats& st = s->sch->stats();
  out->builds = st.builds;
  out->build_failures = st.build_failures;
  out->evictions = st.evictions;
  out->hits = st.hits;
  out->batches = st.batches;
  out->items = st.items;
  out->completed = st.completed;
  out->invariant_violations = st.invariant_violations;
  out->used = st.used;
  out->peak_used = st.peak_used;
  out->budget = st.budget;
  out->cached_plans = (int32_t)st.cached_plans;
  out->pending = (int32_t)st.pending;
  out->running = (int32_t)st.running;
  return PINV_OK;
}

pinv_status pinv_server_destroy(pinv_server* s) {
  if (!s) return PINV_ERR_INVALID;
  s->stop = true;
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->be.apply_stream);
  (void)hipStreamSynchronize(s->be.build_stream);
  s->sch.reset();   // releases every plan it holds
  delete s;         // the streams are the library's, kept for the next server
  return PINV_OK;
}

}  // extern "C"
