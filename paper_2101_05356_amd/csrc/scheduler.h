// Continuous-batching scheduler of reconstruction requests (host only, no HIP).
//
// Requests (one face reconstruction each: a target image, initial
// parameters, a number of Adam steps) arrive at any time.  Between steps the
// scheduler
//   1. admits queued requests in arrival order while a slot is free, the
//      request's device bytes fit the remaining HBM budget and its work per
//      step (nominal rays) fits the remaining work cap (strict FIFO: a
//      request that does not fit blocks the ones behind it, so none starves;
//      the head request is always admitted when nothing runs, whatever its
//      work).  The work cap keeps a round near the size that already fills
//      the device: past it, stepping more requests together only slows every
//      one of them down (processor sharing) without raising the rate at
//      which requests complete;
//   2. advances every active request by k steps in one batched call, with k
//      the smallest number of steps any active request still needs (capped by
//      a quantum, so new arrivals wait at most `quantum` steps);
//   3. fails any request whose last loss is not finite;
//   4. retires the requests that reached their step count, reading their
//      results and freeing their slot and bytes.
// The executor does the device work; it is a template parameter so that the
// policy can be exercised against a simulated executor on the host.
//
// Exec must provide:
//   using Req = ...;                         request payload (movable)
//   size_t bytes(const Req&);                device bytes one active request holds
//   double work(const Req&);                 work of one step of the request (any unit)
//   int add(Req&, int32_t* handle);          FR_OK or an error code
//   int remove(int32_t handle);
//   int step(int n);                         advance every active request n steps
//   int last_losses(std::vector<std::pair<int32_t, float>>&);  latest loss per handle
//   int read(int32_t handle, std::vector<float>& params, std::vector<float>& losses);
//   double now();                            seconds, monotonic
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <deque>
#include <map>
#include <utility>
#include <vector>

namespace fr {

enum ReqState { REQ_QUEUED = 0, REQ_RUNNING = 1, REQ_DONE = 2, REQ_FAILED = 3, REQ_CANCELLED = 4 };

// Status codes shared with the C ABI.
enum { SCHED_OK = 0, SCHED_ERR_INVALID_ARG = 1, SCHED_ERR_BUDGET = 4, SCHED_ERR_NONFINITE = 6, SCHED_ERR_NOT_FOUND = 8 };

struct SchedStats {
  int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, rejected = 0;
  int32_t queued = 0, active = 0, peak_active = 0;
  size_t bytes_in_use = 0, peak_bytes = 0;
  double p50 = 0, p99 = 0, mean = 0, recons_per_s = 0, busy_s = 0;
  int64_t steps = 0, ticks = 0;
};

// Nearest-rank percentile of an ascending sample (q in (0, 1]).
inline double percentile_sorted(const std::vector<double>& v, double q) {
  if (v.empty()) return 0.0;
  size_t r = (size_t)std::ceil(q * (double)v.size());
  r = std::min(std::max<size_t>(r, 1), v.size());
  return v[r - 1];
}

template <class Exec>
class Scheduler {
 public:
  using Req = typename Exec::Req;

  struct Entry {
    uint64_t id = 0;
    Req req{};
    int state = REQ_QUEUED, status = SCHED_OK;
    int steps_total = 0, steps_done = 0;
    int32_t handle = -1;
    size_t bytes = 0;
    double work = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    float final_loss = NAN;
    bool cancel = false;
    std::vector<float> params, losses;
  };

  // work_cap <= 0: no cap.
  Scheduler(Exec& ex, size_t budget, int max_slots, int quantum, double work_cap = 0.0)
      : ex_(ex), budget_(budget), max_slots_(std::max(max_slots, 1)), quantum_(std::max(quantum, 1)),
        work_cap_(work_cap > 0.0 ? work_cap : 0.0) {}

  // Queue request `id` (unique, chosen by the caller; t_submit: arrival time
  // on the executor's clock).
  int submit(uint64_t nid, Req&& r, int n_steps, double t_submit) {
    if (n_steps <= 0 || all_.count(nid)) return SCHED_ERR_INVALID_ARG;
    const size_t b = ex_.bytes(r);
    if (stats_.submitted == 0 || t_submit < first_submit_) first_submit_ = t_submit;
    Entry& e = all_[nid];
    e.id = nid;
    e.steps_total = n_steps;
    e.bytes = b;
    e.work = ex_.work(r);
    e.t_submit = t_submit;
    ++stats_.submitted;
    if (b == 0 || b > budget_) {   // could never be admitted
      e.state = REQ_FAILED;
      e.status = SCHED_ERR_BUDGET;
      e.t_done = t_submit;
      ++stats_.rejected;
      ++stats_.failed;
      return SCHED_ERR_BUDGET;
    }
    e.req = std::move(r);
    queue_.push_back(nid);
    return SCHED_OK;
  }

  // Cancel: a queued request leaves at once, an active one at the next step boundary.
  int cancel(uint64_t id) {
    auto it = all_.find(id);
    if (it == all_.end()) return SCHED_ERR_NOT_FOUND;
    Entry& e = it->second;
    if (e.state == REQ_QUEUED) {
      queue_.erase(std::remove(queue_.begin(), queue_.end(), id), queue_.end());
      finish(e, REQ_CANCELLED, SCHED_OK);
    } else if (e.state == REQ_RUNNING) {
      e.cancel = true;
    }
    return SCHED_OK;
  }

  bool idle() const { return queue_.empty() && active_.empty(); }

  // One scheduling round; returns the ids whose state changed.
  std::vector<uint64_t> tick() {
    std::vector<uint64_t> changed;
    // drop cancelled active requests
    for (size_t i = 0; i < active_.size();) {
      Entry& e = all_[active_[i]];
      if (e.cancel) {
        release(i);
        finish(e, REQ_CANCELLED, SCHED_OK);
        changed.push_back(e.id);
      } else {
        ++i;
      }
    }
    // admit in arrival order
    while (!queue_.empty() && (int)active_.size() < max_slots_) {
      Entry& e = all_[queue_.front()];
      if (used_ + e.bytes > budget_) break;
      if (work_cap_ > 0.0 && !active_.empty() && work_ + e.work > work_cap_) break;
      queue_.pop_front();
      int32_t h = -1;
      const int rc = ex_.add(e.req, &h);
      e.req = Req{};   // the executor has copied the inputs
      if (rc != SCHED_OK) {
        finish(e, REQ_FAILED, rc);
        changed.push_back(e.id);
        continue;
      }
      e.handle = h;
      e.state = REQ_RUNNING;
      e.t_admit = ex_.now();
      used_ += e.bytes;
      work_ += e.work;
      active_.push_back(e.id);
      changed.push_back(e.id);
    }
    stats_.peak_active = std::max<int32_t>(stats_.peak_active, (int32_t)active_.size());
    stats_.peak_bytes = std::max(stats_.peak_bytes, used_);
    peak_work_ = std::max(peak_work_, work_);
    if (active_.empty()) return changed;
    // advance
    int k = quantum_;
    for (uint64_t id : active_) k = std::min(k, all_[id].steps_total - all_[id].steps_done);
    const double t0 = ex_.now();
    const int rc = ex_.step(k);
    stats_.busy_s += ex_.now() - t0;
    ++stats_.ticks;
    if (rc != SCHED_OK) {   // a failed batched step fails every active request
      while (!active_.empty()) {
        Entry& e = all_[active_.back()];
        release(active_.size() - 1);
        finish(e, REQ_FAILED, rc);
        changed.push_back(e.id);
      }
      return changed;
    }
    stats_.steps += k;
    for (uint64_t id : active_) all_[id].steps_done += k;
    // failure detection: a non-finite loss ends the request
    losses_.clear();
    ex_.last_losses(losses_);
    std::map<int32_t, float> last(losses_.begin(), losses_.end());
    for (size_t i = 0; i < active_.size();) {
      Entry& e = all_[active_[i]];
      auto it = last.find(e.handle);
      const float l = it == last.end() ? NAN : it->second;
      e.final_loss = l;
      if (!std::isfinite(l)) {
        (void)ex_.read(e.handle, e.params, e.losses);
        release(i);
        finish(e, REQ_FAILED, SCHED_ERR_NONFINITE);
        changed.push_back(e.id);
      } else if (e.steps_done >= e.steps_total) {
        const int rr = ex_.read(e.handle, e.params, e.losses);
        release(i);
        finish(e, rr == SCHED_OK ? REQ_DONE : REQ_FAILED, rr);
        changed.push_back(e.id);
      } else {
        ++i;
      }
    }
    return changed;
  }

  // Remove every active request from the executor and drop the queue (on
  // shutdown; the requests end cancelled).
  void drop_all() {
    while (!active_.empty()) {
      Entry& e = all_[active_.back()];
      release(active_.size() - 1);
      finish(e, REQ_CANCELLED, SCHED_OK);
    }
    for (uint64_t id : queue_) finish(all_[id], REQ_CANCELLED, SCHED_OK);
    queue_.clear();
  }

  // Largest work admitted together so far.
  double peak_work() const { return peak_work_; }

  const Entry* find(uint64_t id) const {
    auto it = all_.find(id);
    return it == all_.end() ? nullptr : &it->second;
  }

  // Drop a finished request's record (its result has been read).
  int forget(uint64_t id) {
    auto it = all_.find(id);
    if (it == all_.end()) return SCHED_ERR_NOT_FOUND;
    if (it->second.state == REQ_QUEUED || it->second.state == REQ_RUNNING) return SCHED_ERR_INVALID_ARG;
    all_.erase(it);
    return SCHED_OK;
  }

  SchedStats stats() const {
    SchedStats s = stats_;
    s.queued = (int32_t)queue_.size();
    s.active = (int32_t)active_.size();
    s.bytes_in_use = used_;
    std::vector<double> lat = lat_;
    std::sort(lat.begin(), lat.end());
    double sum = 0;
    for (double x : lat) sum += x;
    s.p50 = percentile_sorted(lat, 0.50);
    s.p99 = percentile_sorted(lat, 0.99);
    s.mean = lat.empty() ? 0.0 : sum / (double)lat.size();
    s.recons_per_s = (lat.empty() || last_done_ <= first_submit_) ? 0.0 : (double)lat.size() / (last_done_ - first_submit_);
    return s;
  }

 private:
  void release(size_t i) {
    Entry& e = all_[active_[i]];
    ex_.remove(e.handle);
    used_ -= e.bytes;
    work_ = active_.size() > 1 ? std::max(0.0, work_ - e.work) : 0.0;
    active_.erase(active_.begin() + (long)i);
  }

  void finish(Entry& e, int state, int status) {
    e.state = state;
    e.status = status;
    e.t_done = ex_.now();
    e.req = Req{};
    if (state == REQ_DONE) {
      ++stats_.completed;
      lat_.push_back(e.t_done - e.t_submit);
      last_done_ = std::max(last_done_, e.t_done);
    }
    else if (state == REQ_FAILED) ++stats_.failed;
    else if (state == REQ_CANCELLED) ++stats_.cancelled;
  }

  Exec& ex_;
  size_t budget_;
  int max_slots_, quantum_;
  double work_cap_;
  size_t used_ = 0;
  double work_ = 0, peak_work_ = 0;
  std::deque<uint64_t> queue_;
  std::vector<uint64_t> active_;
  std::map<uint64_t, Entry> all_;
  std::vector<std::pair<int32_t, float>> losses_;
  std::vector<double> lat_;   // arrival-to-done seconds of completed requests
  double first_submit_ = 0, last_done_ = 0;
  SchedStats stats_;
};

}  // namespace fr
