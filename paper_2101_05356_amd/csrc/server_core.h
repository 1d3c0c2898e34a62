// Threaded front of the continuous-batching scheduler (host only, no HIP).
//
// One worker thread owns the executor and the Scheduler: it drains the inbox
// of submitted requests and cancellations, runs scheduling rounds while
// anything is queued or active, and publishes every request's state.  Client
// threads only touch the inbox, the cancellation list and the published
// records, all under one mutex; the device work of a round runs with the
// mutex released.  The executor is a template parameter so that the same code
// runs against a simulated executor on the host (and under the thread and
// address sanitizers there).
//
// Exec must provide, beside what Scheduler<Exec> asks:
//   int init();       on the worker thread before the first round (FR_OK or an error)
//   void shutdown();  on the worker thread after the last round
#pragma once

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "scheduler.h"

namespace fr {

struct PublishedReq {
  int32_t state = REQ_QUEUED, status = SCHED_OK;
  int32_t steps_done = 0, n_steps = 0;
  float final_loss = NAN;
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::vector<float> params, losses;
};

template <class Exec>
class ServerCore {
 public:
  using Req = typename Exec::Req;

  ServerCore(Exec& ex, size_t budget, int max_slots, int quantum, double work_cap)
      : ex_(ex), budget_(budget), sched_(ex, budget, max_slots, quantum, work_cap) {}
  ~ServerCore() { stop(); }

  // Start the worker; returns the executor's init status (the worker has
  // ended already when it is not SCHED_OK).
  int start() {
    worker_ = std::thread([this] { run(); });
    std::unique_lock<std::mutex> lk(mu_);
    cv_idle_.wait(lk, [&] { return started_; });
    const int rc = init_status_;
    lk.unlock();
    if (rc != SCHED_OK) worker_.join();
    return rc;
  }

  // Stop the worker (requests still queued or running are dropped).
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    if (worker_.joinable()) worker_.join();
  }

  // Queue a request; SCHED_ERR_BUDGET if it alone exceeds the budget.
  int submit(Req&& r, int n_steps, uint64_t* id) {
    if (n_steps <= 0) return SCHED_ERR_INVALID_ARG;
    const size_t b = ex_.bytes(r);
    if (b == 0 || b > budget_) return SCHED_ERR_BUDGET;
    {
      std::lock_guard<std::mutex> lk(mu_);
      *id = next_id_++;
      PublishedReq& p = pub_[*id];
      p.n_steps = n_steps;
      p.t_submit = ex_.now();
      inbox_.push_back({*id, std::move(r), n_steps, p.t_submit});
      idle_ = false;
    }
    cv_.notify_all();
    return SCHED_OK;
  }

  // Copy of a request's published record.
  int poll(uint64_t id, PublishedReq* out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = pub_.find(id);
    if (it == pub_.end()) return SCHED_ERR_NOT_FOUND;
    *out = it->second;
    return SCHED_OK;
  }

  // Hand a request's record to `f` under the lock (no copy of its vectors).
  template <class F>
  int with_record(uint64_t id, F&& f) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = pub_.find(id);
    if (it == pub_.end()) return SCHED_ERR_NOT_FOUND;
    f(it->second);
    return SCHED_OK;
  }

  int cancel(uint64_t id) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (!pub_.count(id)) return SCHED_ERR_NOT_FOUND;
      cancels_.push_back(id);
      idle_ = false;
    }
    cv_.notify_all();
    return SCHED_OK;
  }

  // Drop the record of a finished request.
  int forget(uint64_t id) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = pub_.find(id);
    if (it == pub_.end()) return SCHED_ERR_NOT_FOUND;
    if (it->second.state == REQ_QUEUED || it->second.state == REQ_RUNNING) return SCHED_ERR_INVALID_ARG;
    pub_.erase(it);
    return SCHED_OK;
  }

  // Scheduler statistics of the last round; `submitted` counts every
  // accepted submission and `queued` includes the inbox.
  SchedStats stats() {
    std::lock_guard<std::mutex> lk(mu_);
    SchedStats s = stats_;
    s.submitted = (int64_t)next_id_ - 1;
    s.queued += (int32_t)inbox_.size();
    return s;
  }

  // Block until nothing is queued or running; false after timeout_s.
  bool wait(double timeout_s) {
    std::unique_lock<std::mutex> lk(mu_);
    return cv_idle_.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return idle_; });
  }

 private:
  struct Incoming {
    uint64_t id;
    Req req;
    int n_steps;
    double t;
  };

  // Called with the lock held, on the worker thread.
  void publish(uint64_t id) {
    const auto* e = sched_.find(id);
    if (!e) return;
    auto it = pub_.find(id);
    if (it == pub_.end()) return;   // forgotten meanwhile
    PublishedReq& p = it->second;
    p.state = e->state;
    p.status = e->status;
    p.steps_done = e->steps_done;
    p.n_steps = e->steps_total;
    p.final_loss = e->final_loss;
    p.t_submit = e->t_submit;
    p.t_admit = e->t_admit;
    p.t_done = e->t_done;
    if (e->state == REQ_DONE || e->state == REQ_FAILED) {
      p.params = e->params;
      p.losses = e->losses;
    }
  }

  void run() {
    const int rc = ex_.init();
    {
      std::lock_guard<std::mutex> lk(mu_);
      init_status_ = rc;
      started_ = true;
    }
    cv_idle_.notify_all();
    if (rc != SCHED_OK) return;
    std::vector<uint64_t> running;
    for (;;) {
      std::vector<uint64_t> touched;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || !inbox_.empty() || !cancels_.empty() || !sched_.idle(); });
        if (stop_) break;
        while (!inbox_.empty()) {
          Incoming in = std::move(inbox_.front());
          inbox_.pop_front();
          (void)sched_.submit(in.id, std::move(in.req), in.n_steps, in.t);
          touched.push_back(in.id);
        }
        for (uint64_t id : cancels_) {
          (void)sched_.cancel(id);
          touched.push_back(id);
        }
        cancels_.clear();
        for (uint64_t id : touched) publish(id);
      }
      std::vector<uint64_t> changed = sched_.tick();   // device work, lock not held
      {
        std::lock_guard<std::mutex> lk(mu_);
        for (uint64_t id : changed) publish(id);
        // running requests: refresh their step counts
        running.clear();
        for (auto& kv : pub_)
          if (kv.second.state == REQ_RUNNING) running.push_back(kv.first);
        for (uint64_t id : running) publish(id);
        stats_ = sched_.stats();
        idle_ = sched_.idle() && inbox_.empty() && cancels_.empty();
        if (idle_) cv_idle_.notify_all();
      }
    }
    sched_.drop_all();
    ex_.shutdown();
  }

  Exec& ex_;
  size_t budget_;
  Scheduler<Exec> sched_;
  std::thread worker_;
  std::mutex mu_;
  std::condition_variable cv_, cv_idle_;
  bool stop_ = false, idle_ = true, started_ = false;
  int init_status_ = SCHED_OK;
  uint64_t next_id_ = 1;
  std::deque<Incoming> inbox_;
  std::vector<uint64_t> cancels_;
  std::map<uint64_t, PublishedReq> pub_;
  SchedStats stats_{};
};

}  // namespace fr
