// Continuous-batching scheduler for reconstruction requests (pure C++17).
//
// R depends only on the encoding, so it is built once and reused by every
// later request with the same encoding (paper Sec. 4.5 and Sec. 5).  The
// scheduler keeps built plans in an LRU cache keyed by the encoding, admits
// new builds only while their device footprint fits the budget (evicting
// least-recently-used plans that no queued or running request holds), and
// packs the applies of all requests whose plans are ready into grouped
// launches.  Builds and applies are issued to the backend, which runs them on
// separate device queues, so work of requests that arrive while others run
// overlaps on the device.
//
// The backend is a template parameter: the HIP backend drives libpinv; a
// simulated backend with a virtual clock exercises the same logic on the CPU.
// Backend interface:
//   struct Request;               payload of one request (opaque here)
//   typedef ... PlanHandle;       a built or building plan
//   typedef ... BatchHandle;      one grouped apply
//   int  start_build(const Request&, PlanHandle*)      -> 0 ok, else status
//   int  build_state(PlanHandle)                       -> 0 done, 5 busy, else failure status
//   size_t resident_bytes(PlanHandle)                  bytes kept once built
//   int  apply(const std::vector<Item>&, BatchHandle*) -> 0 ok, else status
//   bool batch_done(BatchHandle&)
//   void release(PlanHandle)
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <list>
#include <unordered_map>
#include <vector>

namespace pinv_sched {

enum ReqState { R_PENDING = 0, R_READY = 1, R_RUNNING = 2, R_DONE = 3 };
enum PlanState { P_BUILDING = 0, P_READY = 1, P_FAILED = 2 };
constexpr int kBusy = 5;        // same value as PINV_ERR_BUSY
constexpr int kNoMem = 2;       // same value as PINV_ERR_NOMEM

struct Options {
  size_t budget = 0;            // device bytes for plans (resident + build workspace)
  int max_group = 32;           // requests per grouped apply
  int max_inflight = 2;         // grouped applies in flight
  int max_builds = 1;           // concurrent builds
};

struct Completion {
  uint64_t ticket;
  uint64_t tag;
  int status;                   // 0 ok
  int built;                    // 1 if this request triggered its plan's build
  double t_arrival, t_dispatch, t_done;
};

struct Stats {
  size_t used = 0, peak_used = 0, budget = 0;
  uint64_t builds = 0, build_failures = 0, evictions = 0, hits = 0;
  uint64_t batches = 0, items = 0, completed = 0;
  uint64_t invariant_violations = 0;   // evicting a held plan or exceeding the budget
  size_t cached_plans = 0, pending = 0, running = 0;
};

template <class Backend>
class Scheduler {
 public:
  typedef typename Backend::Request Request;
  typedef typename Backend::PlanHandle PlanHandle;
  typedef typename Backend::BatchHandle BatchHandle;

  struct Item {                 // one request handed to the backend's apply
    const Request* req;
    PlanHandle plan;
  };

  Scheduler(Backend* be, const Options& o) : be_(be), opt_(o) { st_.budget = o.budget; }

  ~Scheduler() {
    for (auto& kv : plans_) be_->release(kv.second.h);
  }

  // Enqueue a request; `footprint` is the device memory its build needs.
  uint64_t submit(uint64_t key, size_t footprint, const Request& r, uint64_t tag, double now) {
    Entry e;
    e.ticket = next_ticket_++;
    e.key = key;
    e.footprint = footprint;
    e.req = r;
    e.tag = tag;
    e.t_arrival = now;
    entries_.emplace(e.ticket, e);
    pending_.push_back(e.ticket);
    return e.ticket;
  }

  // One scheduling step at time `now`.
  void tick(double now) {
    poll_builds();
    poll_batches(now);
    route(now);
    dispatch(now);
    st_.pending = pending_.size();
    st_.cached_plans = plans_.size();
  }

  bool idle() const { return entries_.empty(); }
  const Stats& stats() const { return st_; }

  // Move finished requests to `out`.
  void take_completions(std::vector<Completion>* out, size_t max) {
    while (!done_.empty() && out->size() < max) {
      out->push_back(done_.front());
      done_.pop_front();
    }
  }

 private:
  struct Entry {
    uint64_t ticket = 0, key = 0, tag = 0;
    size_t footprint = 0;
    Request req;
    int state = R_PENDING;
    int built = 0;
    bool holds = false;         // counted in its plan's refs (from association to completion)
    double t_arrival = 0, t_dispatch = 0;
  };
  struct Plan {
    PlanHandle h;
    int state = P_BUILDING;
    int refs = 0;               // requests associated with it and not yet finished
    size_t charged = 0;         // bytes counted against the budget
    std::list<uint64_t>::iterator lru;
  };
  struct Batch {
    BatchHandle h;
    std::vector<uint64_t> tickets;
  };

  void charge(size_t b) {
    st_.used += b;
    st_.peak_used = std::max(st_.peak_used, st_.used);
    if (st_.used > opt_.budget) st_.invariant_violations++;
  }

  void finish(uint64_t ticket, int status, double now) {
    auto it = entries_.find(ticket);
    if (it == entries_.end()) return;
    Entry& e = it->second;
    done_.push_back(Completion{e.ticket, e.tag, status, e.built, e.t_arrival,
                               e.t_dispatch ? e.t_dispatch : now, now});
    st_.completed++;
    entries_.erase(it);
  }

  void poll_builds() {
    for (auto& kv : plans_) {
      Plan& p = kv.second;
      if (p.state != P_BUILDING) continue;
      const int s = be_->build_state(p.h);
      if (s == kBusy) continue;
      --building_;
      if (s == 0) {
        p.state = P_READY;
        const size_t res = be_->resident_bytes(p.h);
        if (res < p.charged) {
          st_.used -= p.charged - res;
          p.charged = res;
        }
      } else {
        p.state = P_FAILED;
        st_.used -= p.charged;   // a failed build keeps no memory
        p.charged = 0;
        st_.build_failures++;
        fail_code_[kv.first] = s;
      }
    }
  }

  void poll_batches(double now) {
    for (size_t i = 0; i < inflight_.size();) {
      if (!be_->batch_done(inflight_[i].h)) {
        ++i;
        continue;
      }
      for (uint64_t t : inflight_[i].tickets) {
        auto it = entries_.find(t);
        if (it == entries_.end()) continue;
        auto pit = plans_.find(it->second.key);
        if (pit != plans_.end()) {
          pit->second.refs--;
          touch(pit->first);
        }
        finish(t, 0, now);
        st_.running--;
      }
      inflight_.erase(inflight_.begin() + i);
    }
  }

  void touch(uint64_t key) {
    Plan& p = plans_[key];
    lru_.erase(p.lru);
    lru_.push_front(key);
    p.lru = lru_.begin();
  }

  // Evict least-recently-used ready plans that no request holds until `need`
  // more bytes fit.  Plans with references are never evicted.
  bool make_room(size_t need) {
    if (st_.used + need <= opt_.budget) return true;
    for (auto it = lru_.end(); it != lru_.begin();) {
      --it;
      const uint64_t key = *it;
      Plan& p = plans_[key];
      if (p.state == P_BUILDING || p.refs > 0) continue;
      if (p.refs < 0) st_.invariant_violations++;
      st_.used -= p.charged;
      be_->release(p.h);
      it = lru_.erase(it);
      plans_.erase(key);
      fail_code_.erase(key);
      st_.evictions++;
      if (st_.used + need <= opt_.budget) return true;
    }
    return st_.used + need <= opt_.budget;
  }

  void route(double now) {
    (void)now;
    for (auto it = pending_.begin(); it != pending_.end();) {
      Entry& e = entries_[*it];
      auto pit = plans_.find(e.key);
      if (pit != plans_.end()) {
        Plan& p = pit->second;
        if (!e.holds) {   // hold the plan from now on, so it cannot be evicted under us
          p.refs++;
          e.holds = true;
        }
        if (p.state == P_READY) {
          touch(e.key);
          if (!e.built) st_.hits++;
          e.state = R_READY;
          ready_.push_back(e.ticket);
          it = pending_.erase(it);
        } else if (p.state == P_FAILED) {
          const uint64_t t = e.ticket;
          p.refs--;
          it = pending_.erase(it);
          finish(t, fail_code_[pit->first], now);
        } else {
          ++it;   // its plan is building
        }
        continue;
      }
      // a new encoding: admit its build if a build slot and memory are free
      if (e.footprint > opt_.budget) {
        const uint64_t t = e.ticket;
        it = pending_.erase(it);
        finish(t, kNoMem, now);
        continue;
      }
      if (building_ >= opt_.max_builds || !make_room(e.footprint)) {
        ++it;     // wait; later requests whose plans are ready may still go
        continue;
      }
      Plan p;
      const int s = be_->start_build(e.req, &p.h);
      if (s != 0) {
        const uint64_t t = e.ticket;
        it = pending_.erase(it);
        finish(t, s, now);
        continue;
      }
      p.state = P_BUILDING;
      p.refs = 1;
      e.holds = true;
      p.charged = e.footprint;
      charge(e.footprint);
      lru_.push_front(e.key);
      p.lru = lru_.begin();
      plans_.emplace(e.key, p);
      building_++;
      st_.builds++;
      e.built = 1;
      ++it;       // routed to the ready queue once the build completes
    }
  }

  void dispatch(double now) {
    while (!ready_.empty() && (int)inflight_.size() < opt_.max_inflight) {
      std::vector<Item> items;
      Batch b;
      while (!ready_.empty() && (int)items.size() < opt_.max_group) {
        const uint64_t t = ready_.front();
        ready_.pop_front();
        Entry& e = entries_[t];
        Plan& p = plans_[e.key];
        items.push_back(Item{&e.req, p.h});
        b.tickets.push_back(t);
        e.state = R_RUNNING;
        e.t_dispatch = now;
      }
      const int s = be_->apply(items, &b.h);
      if (s != 0) {
        for (uint64_t t : b.tickets) {
          auto pit = plans_.find(entries_[t].key);
          if (pit != plans_.end()) pit->second.refs--;
          finish(t, s, now);
        }
        continue;
      }
      st_.batches++;
      st_.items += items.size();
      st_.running += items.size();
      inflight_.push_back(b);
    }
  }

  Backend* be_;
  Options opt_;
  Stats st_;
  uint64_t next_ticket_ = 1;
  int building_ = 0;
  std::unordered_map<uint64_t, Entry> entries_;
  std::list<uint64_t> pending_;
  std::deque<uint64_t> ready_;
  std::unordered_map<uint64_t, Plan> plans_;
  std::unordered_map<uint64_t, int> fail_code_;
  std::list<uint64_t> lru_;
  std::vector<Batch> inflight_;
  std::deque<Completion> done_;
};

}  // namespace pinv_sched
