// Host-only driver of the continuous-batching scheduler against a simulated
// executor with a virtual clock: every scenario prints one JSON object that
// tests/test_scheduler_host.py checks.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../paper_2101_05356_amd/csrc/scheduler.h"

struct SimExec {
  struct Req {
    size_t bytes = 0;
    double cost = 0.0;   // seconds per step while active
    int nan_at = -1;     // loss turns NaN once this many steps are done
    int fail_add = 0;    // add() fails with this code
    int tag = 0;
    double work = 0.0;   // work per step, checked against the work cap
  };
  struct Job {
    Req r;
    int t = 0;
  };
  std::map<int32_t, Job> jobs;
  int32_t next = 1;
  double clock = 0.0, overhead = 0.001;
  double floor = 0.0;   // a step costs at least this much (a device that is not yet full)
  int max_active = 0;
  double max_work = 0.0;   // largest summed work stepped together
  size_t bytes(const Req& r) { return r.bytes; }
  double work(const Req& r) { return r.work; }
  double active_work() const {
    double w = 0;
    for (auto& kv : jobs) w += kv.second.r.work;
    return w;
  }
  int add(Req& r, int32_t* h) {
    if (r.fail_add) return r.fail_add;
    *h = next++;
    jobs[*h] = Job{r, 0};
    max_active = std::max(max_active, (int)jobs.size());
    return 0;
  }
  int remove(int32_t h) { return jobs.erase(h) ? 0 : 8; }
  int step(int n) {
    max_work = std::max(max_work, active_work());
    double c = 0.0;
    for (auto& kv : jobs) { c += kv.second.r.cost; kv.second.t += n; }
    clock += n * (overhead + std::max(c, floor));
    return 0;
  }
  int last_losses(std::vector<std::pair<int32_t, float>>& out) {
    for (auto& kv : jobs) {
      const Job& j = kv.second;
      out.emplace_back(kv.first, (j.r.nan_at >= 0 && j.t >= j.r.nan_at) ? NAN : 1.0f / (1.0f + j.t));
    }
    return 0;
  }
  int read(int32_t h, std::vector<float>& params, std::vector<float>& losses) {
    const Job& j = jobs.at(h);
    params = {(float)j.r.tag, (float)j.t};
    losses.assign(j.t, 0.0f);
    return 0;
  }
  double now() { return clock; }
};

struct Arrival {
  double t;
  SimExec::Req r;
  int steps;
  uint64_t id;
};

struct Run {
  SimExec ex;
  fr::Scheduler<SimExec> s;
  std::map<uint64_t, int> submit_rc;
  std::vector<uint64_t> done_order;
  Run(size_t budget, int slots, int quantum, double work_cap = 0.0) : s(ex, budget, slots, quantum, work_cap) {}

  // Feed arrivals in time order; between arrivals run scheduling rounds.
  void drive(std::vector<Arrival> arr, const std::map<int, std::vector<uint64_t>>& cancel_at_tick = {}) {
    size_t next = 0;
    int tick = 0;
    while (next < arr.size() || !s.idle()) {
      while (next < arr.size() && arr[next].t <= ex.clock) {
        submit_rc[arr[next].id] = s.submit(arr[next].id, SimExec::Req(arr[next].r), arr[next].steps, arr[next].t);
        ++next;
      }
      auto it = cancel_at_tick.find(tick);
      if (it != cancel_at_tick.end())
        for (uint64_t id : it->second) s.cancel(id);
      if (s.idle()) {   // nothing to do until the next arrival
        ex.clock = arr[next].t;
        continue;
      }
      for (uint64_t id : s.tick())
        if (s.find(id)->state >= fr::REQ_DONE &&
            std::find(done_order.begin(), done_order.end(), id) == done_order.end())
          done_order.push_back(id);
      ++tick;
    }
  }

  void print(const char* name) {
    printf("{\"scenario\": \"%s\", \"max_active\": %d, \"max_work\": %.6f, \"peak_work\": %.6f, \"reqs\": {", name,
           ex.max_active, ex.max_work, s.peak_work());
    bool first = true;
    for (auto& kv : submit_rc) {
      const auto* e = s.find(kv.first);
      printf("%s\"%llu\": {\"rc\": %d, \"state\": %d, \"status\": %d, \"steps_done\": %d, \"t_submit\": %.6f, "
             "\"t_admit\": %.6f, \"t_done\": %.6f, \"n_losses\": %zu}",
             first ? "" : ", ", (unsigned long long)kv.first, kv.second, e->state, e->status, e->steps_done,
             e->t_submit, e->t_admit, e->t_done, e->losses.size());
      first = false;
    }
    printf("}, \"done_order\": [");
    for (size_t i = 0; i < done_order.size(); ++i) printf("%s%llu", i ? ", " : "", (unsigned long long)done_order[i]);
    const fr::SchedStats st = s.stats();
    printf("], \"stats\": {\"completed\": %lld, \"failed\": %lld, \"cancelled\": %lld, \"rejected\": %lld, "
           "\"peak_active\": %d, \"peak_bytes\": %zu, \"bytes_in_use\": %zu, \"p50\": %.6f, \"p99\": %.6f, "
           "\"mean\": %.6f, \"recons_per_s\": %.6f, \"steps\": %lld, \"ticks\": %lld}}\n",
           (long long)st.completed, (long long)st.failed, (long long)st.cancelled, (long long)st.rejected,
           st.peak_active, st.peak_bytes, st.bytes_in_use, st.p50, st.p99, st.mean, st.recons_per_s,
           (long long)st.steps, (long long)st.ticks);
  }
};

static SimExec::Req req(size_t bytes, double cost = 0.01, int nan_at = -1, int fail_add = 0, double work = 0.0) {
  SimExec::Req r;
  r.bytes = bytes; r.cost = cost; r.nan_at = nan_at; r.fail_add = fail_add; r.work = work;
  return r;
}

int main(int argc, char** argv) {
  const std::string sc = argc > 1 ? argv[1] : "";
  if (sc == "fifo_budget") {         // budget admits two of the 4-byte requests at a time
    Run r(10, 8, 4);
    std::vector<Arrival> a;
    for (int i = 1; i <= 6; ++i) a.push_back({0.0, req(4), 5, (uint64_t)i});
    r.drive(a);
    r.print("fifo_budget");
  } else if (sc == "slots") {        // slots bound concurrency
    Run r(1000, 3, 4);
    std::vector<Arrival> a;
    for (int i = 1; i <= 7; ++i) a.push_back({0.0, req(1), 3 + i, (uint64_t)i});
    r.drive(a);
    r.print("slots");
  } else if (sc == "reject") {       // a request larger than the budget never enters
    Run r(10, 4, 4);
    r.drive({{0.0, req(20), 5, 1}, {0.0, req(5), 5, 2}});
    r.print("reject");
  } else if (sc == "mixed_steps") {  // each request runs exactly its step count
    Run r(1000, 8, 4);
    r.drive({{0.0, req(1), 3, 1}, {0.0, req(1), 7, 2}, {0.0, req(1), 12, 3}, {0.05, req(1), 2, 4}});
    r.print("mixed_steps");
  } else if (sc == "cancel") {       // cancel while queued and while running
    Run r(1000, 1, 2);
    r.drive({{0.0, req(1), 10, 1}, {0.0, req(1), 10, 2}, {0.0, req(1), 4, 3}}, {{0, {2}}, {1, {1}}});
    r.print("cancel");
  } else if (sc == "nan") {          // a non-finite loss fails that request only
    Run r(1000, 8, 4);
    r.drive({{0.0, req(1), 10, 1}, {0.0, req(1, 0.01, 3), 10, 2}, {0.0, req(1), 10, 3}});
    r.print("nan");
  } else if (sc == "add_fail") {     // a failed allocation does not leak budget
    Run r(10, 8, 4);
    r.drive({{0.0, req(10, 0.01, -1, 3), 5, 1}, {0.0, req(10), 5, 2}});
    r.print("add_fail");
  } else if (sc == "hol") {          // strict FIFO: a small request waits behind a big one
    Run r(10, 8, 5);
    r.drive({{0.0, req(8), 10, 1}, {0.0, req(8), 10, 2}, {0.0, req(1), 1, 3}});
    r.print("hol");
  } else if (sc == "latency") {      // serial service: known completion times
    Run r(1000, 1, 10);
    std::vector<Arrival> a;
    for (int i = 1; i <= 4; ++i) a.push_back({0.0, req(1, 0.099), 10, (uint64_t)i});
    r.drive(a);
    r.print("latency");
  } else if (sc == "arrivals") {     // arrivals over time, idle gaps
    Run r(1000, 4, 3);
    r.drive({{0.0, req(1), 6, 1}, {10.0, req(1), 6, 2}, {10.0, req(1), 3, 3}, {30.0, req(1), 1, 4}});
    r.print("arrivals");
  } else if (sc == "work_cap") {     // the work cap bounds what is stepped together, in FIFO order
    Run r(1000, 8, 4, 10.0);
    // works 4, 4, 4, 12 (above the cap: runs alone), 1, 1
    const double w[6] = {4, 4, 4, 12, 1, 1};
    std::vector<Arrival> a;
    for (int i = 1; i <= 6; ++i) a.push_back({0.0, req(1, 0.01, -1, 0, w[i - 1]), 4 + i, (uint64_t)i});
    r.drive(a);
    r.print("work_cap");
  } else if (sc == "cap_latency_uncapped" || sc == "cap_latency_capped") {
    // batch arrival of eight equal requests on a device that one request
    // keeps half busy: a step of k requests costs max(2, k) * 0.05
    Run r(1000, 16, 10, sc == "cap_latency_capped" ? 2.0 : 0.0);
    r.ex.overhead = 0.0;
    r.ex.floor = 0.1;
    std::vector<Arrival> a;
    for (int i = 1; i <= 8; ++i) a.push_back({0.0, req(1, 0.05, -1, 0, 1.0), 20, (uint64_t)i});
    r.drive(a);
    r.print(sc.c_str());
  } else {
    fprintf(stderr, "unknown scenario\n");
    return 2;
  }
  return 0;
}
