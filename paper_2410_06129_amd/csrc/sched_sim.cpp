// The serving scheduler (pinv_sched.h) on a simulated device with a virtual
// clock, for CPU tests of admission, eviction, batching and completion.  The
// simulated device runs builds one after another on a build queue and grouped
// applies one after another on an apply queue; it counts any apply that uses
// a plan already released.
#include <stddef.h>
#include <stdint.h>

#include <unordered_map>
#include <vector>

#include "pinv_sched.h"

namespace {

struct SimBackend {
  struct Request {
    double build_s = 0, apply_s = 0;
    size_t resident = 0;
    int fail = 0;
  };
  typedef int PlanHandle;
  struct BatchHandle {
    double t_done = 0;
  };
  typedef pinv_sched::Scheduler<SimBackend>::Item Item;
  struct SimPlan {
    double t_ready;
    size_t resident;
    int fail;
    bool live;
  };

  double now = 0, build_free = 0, apply_free = 0;
  int next = 1;
  std::unordered_map<int, SimPlan> plans;
  uint64_t use_after_release = 0, releases = 0;

  int start_build(const Request& r, int* h) {
    const double t0 = now > build_free ? now : build_free;
    build_free = t0 + r.build_s;
    *h = next++;
    plans[*h] = SimPlan{build_free, r.resident, r.fail, true};
    return 0;
  }
  int build_state(int h) {
    const SimPlan& p = plans[h];
    if (now < p.t_ready) return pinv_sched::kBusy;
    return p.fail ? 3 : 0;
  }
  size_t resident_bytes(int h) { return plans[h].resident; }
  int apply(const std::vector<Item>& items, BatchHandle* b) {
    double t = now > apply_free ? now : apply_free;
    for (const Item& it : items) {
      if (!plans[it.plan].live) use_after_release++;
      t += it.req->apply_s;
    }
    apply_free = t;
    b->t_done = t;
    return 0;
  }
  bool batch_done(BatchHandle& b) { return now >= b.t_done; }
  void release(int h) {
    if (!plans[h].live) use_after_release++;
    plans[h].live = false;
    releases++;
  }
};

struct Sim {
  SimBackend be;
  pinv_sched::Scheduler<SimBackend>* sch;
};

}  // namespace

extern "C" {

void* sim_create(size_t budget, int max_group, int max_inflight, int max_builds) {
  Sim* s = new Sim();
  pinv_sched::Options o;
  o.budget = budget;
  o.max_group = max_group;
  o.max_inflight = max_inflight;
  o.max_builds = max_builds;
  s->sch = new pinv_sched::Scheduler<SimBackend>(&s->be, o);
  return s;
}

uint64_t sim_submit(void* p, uint64_t key, size_t footprint, size_t resident, double build_s,
                    double apply_s, int fail, uint64_t tag) {
  Sim* s = (Sim*)p;
  SimBackend::Request r;
  r.build_s = build_s;
  r.apply_s = apply_s;
  r.resident = resident;
  r.fail = fail;
  return s->sch->submit(key, footprint, r, tag, s->be.now);
}

void sim_advance(void* p, double dt) {
  Sim* s = (Sim*)p;
  s->be.now += dt;
  s->sch->tick(s->be.now);
}

int sim_idle(void* p) { return ((Sim*)p)->sch->idle() ? 1 : 0; }

double sim_now(void* p) { return ((Sim*)p)->be.now; }

int sim_completions(void* p, uint64_t* ticket, uint64_t* tag, int* status, int* built,
                    double* t_arr, double* t_disp, double* t_done, int max) {
  Sim* s = (Sim*)p;
  std::vector<pinv_sched::Completion> c;
  s->sch->take_completions(&c, (size_t)max);
  for (size_t i = 0; i < c.size(); ++i) {
    ticket[i] = c[i].ticket;
    tag[i] = c[i].tag;
    status[i] = c[i].status;
    built[i] = c[i].built;
    t_arr[i] = c[i].t_arrival;
    t_disp[i] = c[i].t_dispatch;
    t_done[i] = c[i].t_done;
  }
  return (int)c.size();
}

// out: builds, build_failures, evictions, hits, batches, items, completed,
//      invariant_violations, used, peak_used, budget, use_after_release
void sim_stats(void* p, uint64_t* out) {
  Sim* s = (Sim*)p;
  const pinv_sched::Stats& st = s->sch->stats();
  const uint64_t v[12] = {st.builds, st.build_failures, st.evictions, st.hits, st.batches,
                          st.items, st.completed, st.invariant_violations, st.used,
                          st.peak_used, st.budget, s->be.use_after_release};
  for (int i = 0; i < 12; ++i) out[i] = v[i];
}

void sim_destroy(void* p) {
  Sim* s = (Sim*)p;
  delete s->sch;
  delete s;
}

}  // extern "C"
