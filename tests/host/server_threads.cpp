// Host-only driver of the threaded server front (server_core.h) against a
// simulated executor on the real clock: several client threads submit, poll,
// cancel, forget and read statistics while the worker runs rounds.  Built
// plain and under the thread and address/undefined-behaviour sanitizers by
// tests/test_host_sanitizers.py; prints one JSON object.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_2101_05356_amd/csrc/server_core.h"

struct ThreadExec {
  struct Req {
    size_t bytes = 0;
    double work = 0.0;
    int tag = 0;
  };
  struct Job {
    Req r;
    int t = 0;
  };
  std::map<int32_t, Job> jobs;   // touched by the worker thread only
  int32_t next = 1;
  int max_active = 0;
  bool inited = false, shut = false;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  int init() { inited = true; return 0; }
  void shutdown() { shut = true; jobs.clear(); }
  size_t bytes(const Req& r) { return r.bytes; }
  double work(const Req& r) { return r.work; }
  int add(Req& r, int32_t* h) {
    *h = next++;
    jobs[*h] = Job{r, 0};
    if ((int)jobs.size() > max_active) max_active = (int)jobs.size();
    return 0;
  }
  int remove(int32_t h) { return jobs.erase(h) ? 0 : 8; }
  int step(int n) {
    for (auto& kv : jobs) kv.second.t += n;
    std::this_thread::sleep_for(std::chrono::microseconds(50 * n));
    return 0;
  }
  int last_losses(std::vector<std::pair<int32_t, float>>& out) {
    for (auto& kv : jobs) out.emplace_back(kv.first, 1.0f / (1.0f + kv.second.t));
    return 0;
  }
  int read(int32_t h, std::vector<float>& params, std::vector<float>& losses) {
    const Job& j = jobs.at(h);
    params = {(float)j.r.tag, (float)j.t};
    losses.assign(j.t, 0.5f);
    return 0;
  }
  double now() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

int main() {
  ThreadExec ex;
  std::atomic<int> bad{0};
  int done = 0, cancelled = 0, forgotten = 0, steps_ok = 0, total = 0, max_active = 0;
  bool waited = false;
  long long stats_completed = 0, stats_submitted = 0;
  {
    fr::ServerCore<ThreadExec> srv(ex, 100, 6, 3, 40.0);
    if (srv.start() != 0) return 1;
    const int n_clients = 4, per_client = 24;
    struct Sub { uint64_t id; int steps, tag; };
    std::vector<std::vector<Sub>> ids(n_clients);
    std::atomic<bool> running{true};
    std::vector<std::thread> th;
    for (int c = 0; c < n_clients; ++c) {
      th.emplace_back([&, c] {
        std::mt19937 rng(17 + c);
        for (int i = 0; i < per_client; ++i) {
          ThreadExec::Req r;
          r.bytes = 5 + rng() % 30;
          r.work = 5.0 + (double)(rng() % 20);
          r.tag = c * 1000 + i;
          const int steps = 1 + (int)(rng() % 12);
          uint64_t id = 0;
          if (srv.submit(std::move(r), steps, &id) != 0) { ++bad; continue; }
          ids[c].push_back({id, steps, c * 1000 + i});
          fr::PublishedReq p;
          if (srv.poll(id, &p) != 0) ++bad;
          if (i % 7 == 3) srv.cancel(id);
          std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
        }
      });
    }
    std::thread watcher([&] {   // statistics and polls of unknown ids meanwhile
      while (running.load()) {
        const fr::SchedStats s = srv.stats();
        if (s.bytes_in_use > 100 || s.active > 6) ++bad;
        fr::PublishedReq p;
        if (srv.poll(999999, &p) != fr::SCHED_ERR_NOT_FOUND) ++bad;
        std::this_thread::sleep_for(std::chrono::microseconds(200));
      }
    });
    for (auto& t : th) t.join();
    waited = srv.wait(60.0);
    running = false;
    watcher.join();
    for (int c = 0; c < n_clients; ++c)
      for (const Sub& sb : ids[c]) {
        const uint64_t id = sb.id;
        const int steps = sb.steps;
        ++total;
        fr::PublishedReq p;
        if (srv.poll(id, &p) != 0) { ++bad; continue; }
        if (p.state == fr::REQ_DONE) {
          ++done;
          if (p.steps_done == steps && (int)p.losses.size() == steps && p.params.size() == 2 &&
              (int)p.params[0] == sb.tag && (int)p.params[1] == steps)
            ++steps_ok;
        } else if (p.state == fr::REQ_CANCELLED) {
          ++cancelled;
        } else {
          ++bad;
        }
        if (srv.forget(id) == 0) ++forgotten;
      }
    const fr::SchedStats s = srv.stats();
    stats_completed = s.completed;
    stats_submitted = s.submitted;
    srv.stop();
  }
  max_active = ex.max_active;
  printf("{\"total\": %d, \"done\": %d, \"cancelled\": %d, \"steps_ok\": %d, \"forgotten\": %d, \"bad\": %d, "
         "\"waited\": %s, \"max_active\": %d, \"stats_completed\": %lld, \"stats_submitted\": %lld, "
         "\"inited\": %s, \"shut\": %s, \"jobs_left\": %zu}\n",
         total, done, cancelled, steps_ok, forgotten, bad.load(), waited ? "true" : "false", max_active,
         stats_completed, stats_submitted, ex.inited ? "true" : "false", ex.shut ? "true" : "false", ex.jobs.size());
  return 0;
}
