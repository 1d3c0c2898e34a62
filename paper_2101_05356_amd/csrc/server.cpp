// Reconstruction server: a worker thread that owns one HIP stream and one
// batch of jobs, and schedules submitted requests onto it with the
// continuous-batching policy of scheduler.h.  The device work goes through
// the batch entry points of the C ABI.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/fr.h"
#include "scheduler.h"

namespace fr {
int model_device(const fr_model* m);   // defined with the model object
}

namespace {

using Clock = std::chrono::steady_clock;

// Executor over one fr_batch on the worker's stream.
struct BatchExec {
  struct Req {
    fr_job_desc desc{};
    std::vector<float> cam, p0, e1, e2, target, params, lr;
    std::vector<int32_t> shape;
    // point the description at this request's own copies
    void bind() {
      desc.cam = cam.data(); desc.light_p0 = p0.data(); desc.light_e1 = e1.data(); desc.light_e2 = e2.data();
      desc.light_shape = shape.data(); desc.target = target.data(); desc.params = params.data(); desc.lr = lr.data();
    }
  };

  fr_model* model = nullptr;
  fr_batch* batch = nullptr;
  hipStream_t st = nullptr;
  bool use_graph = true;
  Clock::time_point t0;
  std::vector<int32_t> ids;
  std::vector<float> tmp;

  size_t bytes(const Req& r) { return fr_job_bytes(model, &r.desc); }
  int add(Req& r, int32_t* h) {
    r.bind();
    return fr_batch_add(batch, &r.desc, h, reinterpret_cast<fr_stream>(st));
  }
  int remove(int32_t h) { return fr_batch_remove(batch, h); }
  int step(int n) {
    const int rc = fr_batch_step(batch, n, use_graph ? 1 : 0, reinterpret_cast<fr_stream>(st));
    if (rc != FR_OK) return rc;
    return hipStreamSynchronize(st) == hipSuccess ? FR_OK : FR_ERR_DEVICE;
  }
  int last_losses(std::vector<std::pair<int32_t, float>>& out) {
    const int n = fr_batch_size(batch);
    ids.assign(std::max(n, 1), 0);
    tmp.assign(std::max(n, 1), 0.0f);
    const int got = fr_batch_losses(batch, n, ids.data(), tmp.data(), reinterpret_cast<fr_stream>(st));
    if (got < 0) return FR_ERR_DEVICE;
    for (int i = 0; i < got; ++i) out.emplace_back(ids[i], tmp[i]);
    return FR_OK;
  }
  int read(int32_t h, std::vector<float>& params, std::vector<float>& losses) {
    int32_t t = 0, np = 0, cap = 0;
    if (fr_batch_job_info(batch, h, &np, &cap, nullptr) != FR_OK) return FR_ERR_NOT_FOUND;
    params.assign(np, 0.0f);
    std::vector<float> hist(cap, 0.0f);
    const int rc = fr_batch_read(batch, h, params.data(), nullptr, hist.data(), nullptr, &t,
                                 reinterpret_cast<fr_stream>(st));
    if (rc != FR_OK) return rc;
    hist.resize(std::min<size_t>(hist.size(), (size_t)std::max(t, 0)));
    losses.swap(hist);
    return FR_OK;
  }
  double now() { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

struct Published {
  fr_result r{};
  std::vector<float> params, losses;
};

}  // namespace

struct fr_server {
  fr_model* model = nullptr;
  fr_server_opts opts{};
  BatchExec ex;
  fr::Scheduler<BatchExec>* sched = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv, cv_idle;
  bool stop = false, idle = true, started = false;
  int init_status = FR_OK;
  uint64_t next_id = 1;
  struct Incoming {
    uint64_t id;
    BatchExec::Req req;
    int n_steps;
    double t;
  };
  std::deque<Incoming> inbox;
  std::vector<uint64_t> cancels;
  std::map<uint64_t, Published> pub;
  fr::SchedStats stats{};

  void publish(uint64_t id) {
    const auto* e = sched->find(id);
    if (!e) return;
    Published& p = pub[id];
    p.r.state = e->state;
    p.r.status = e->status;
    p.r.steps_done = e->steps_done;
    p.r.n_steps = e->steps_total;
    p.r.final_loss = e->final_loss;
    p.r.t_submit = e->t_submit;
    p.r.t_admit = e->t_admit;
    p.r.t_done = e->t_done;
    if (e->state == fr::REQ_DONE || e->state == fr::REQ_FAILED) {
      p.params = e->params;
      p.losses = e->losses;
    }
  }

  void run() {
    if (hipSetDevice(fr::model_device(model)) != hipSuccess ||
        hipStreamCreateWithFlags(&ex.st, hipStreamNonBlocking) != hipSuccess) {
      std::lock_guard<std::mutex> lk(mu);
      init_status = FR_ERR_DEVICE;
      started = true;
      cv_idle.notify_all();
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      started = true;
      cv_idle.notify_all();
    }
    for (;;) {
      std::vector<uint64_t> touched;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || !inbox.empty() || !cancels.empty() || !sched->idle(); });
        if (stop) break;
        while (!inbox.empty()) {
          Incoming in = std::move(inbox.front());
          inbox.pop_front();
          (void)sched->submit(in.id, std::move(in.req), in.n_steps, in.t);
          touched.push_back(in.id);
        }
        for (uint64_t id : cancels) {
          (void)sched->cancel(id);
          touched.push_back(id);
        }
        cancels.clear();
        for (uint64_t id : touched) publish(id);
      }
      std::vector<uint64_t> changed = sched->tick();   // device work, lock not held
      {
        std::lock_guard<std::mutex> lk(mu);
        for (uint64_t id : changed) publish(id);
        // running requests: refresh their step counts
        for (auto& kv : pub)
          if (kv.second.r.state == fr::REQ_RUNNING) publish(kv.first);
        stats = sched->stats();
        idle = sched->idle() && inbox.empty() && cancels.empty();
        if (idle) cv_idle.notify_all();
      }
    }
    // shut down: release every job still held
    delete sched;
    sched = nullptr;
    fr_batch_destroy(ex.batch);
    ex.batch = nullptr;
    (void)hipStreamDestroy(ex.st);
  }
};

namespace {
template <class T>
bool copy_in(std::vector<T>& dst, const T* src, size_t n) {
  if (!src) return false;
  dst.assign(src, src + n);
  return true;
}
}  // namespace

extern "C" {

int fr_server_create(fr_model* model, const fr_server_opts* o, fr_server** out) {
  if (!model || !o || !out || o->max_slots <= 0 || o->quantum <= 0 || o->hbm_budget == 0) return FR_ERR_INVALID_ARG;
  fr_server* s = new fr_server();
  s->model = model;
  s->opts = *o;
  if (fr_batch_create(model, &s->ex.batch) != FR_OK) {
    delete s;
    return FR_ERR_INVALID_ARG;
  }
  s->ex.model = model;
  s->ex.use_graph = o->use_graph != 0;
  s->ex.t0 = Clock::now();
  s->sched = new fr::Scheduler<BatchExec>(s->ex, o->hbm_budget, o->max_slots, o->quantum);
  s->worker = std::thread([s] { s->run(); });
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_idle.wait(lk, [&] { return s->started; });
  if (s->init_status != FR_OK) {
    const int rc = s->init_status;
    lk.unlock();
    s->worker.join();
    delete s->sched;
    fr_batch_destroy(s->ex.batch);
    delete s;
    return rc;
  }
  *out = s;
  return FR_OK;
}

int fr_server_destroy(fr_server* s) {
  if (!s) return FR_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  s->worker.join();
  delete s;
  return FR_OK;
}

int fr_server_submit(fr_server* s, const fr_request* rq, uint64_t* id) {
  if (!s || !rq || !id) return FR_ERR_INVALID_ARG;
  const fr_job_desc& d = rq->job;
  if (rq->n_steps <= 0 || d.width <= 0 || d.height <= 0 || d.n_lights <= 0 || d.spp <= 0 || d.hist_cap < 0)
    return FR_ERR_INVALID_ARG;
  const int L = d.n_lights;
  const int np = fr_model_n_param(s->model, L);
  BatchExec::Req r;
  r.desc = d;
  const size_t px3 = 3 * (size_t)d.width * d.height;
  if (!copy_in(r.cam, d.cam, 12) || !copy_in(r.p0, d.light_p0, 3 * L) || !copy_in(r.e1, d.light_e1, 3 * L) ||
      !copy_in(r.e2, d.light_e2, 3 * L) || !copy_in(r.shape, d.light_shape, L) || !copy_in(r.target, d.target, px3) ||
      !copy_in(r.params, d.params, np) || !copy_in(r.lr, d.lr, np))
    return FR_ERR_INVALID_ARG;
  r.bind();
  const size_t bytes = fr_job_bytes(s->model, &r.desc);
  if (bytes == 0 || bytes > s->opts.hbm_budget) return FR_ERR_BUDGET;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    *id = s->next_id++;
    Published& p = s->pub[*id];
    p.r.state = fr::REQ_QUEUED;
    p.r.status = FR_OK;
    p.r.n_steps = rq->n_steps;
    p.r.final_loss = NAN;
    p.r.t_submit = s->ex.now();
    s->inbox.push_back({*id, std::move(r), rq->n_steps, p.r.t_submit});
    s->idle = false;
  }
  s->cv.notify_all();
  return FR_OK;
}

int fr_server_poll(fr_server* s, uint64_t id, fr_result* out, float* h_params, float* h_losses) {
  if (!s || !out) return FR_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->pub.find(id);
  if (it == s->pub.end()) return FR_ERR_NOT_FOUND;
  *out = it->second.r;
  if (h_params && !it->second.params.empty())
    std::memcpy(h_params, it->second.params.data(), 4 * it->second.params.size());
  if (h_losses && !it->second.losses.empty())
    std::memcpy(h_losses, it->second.losses.data(), 4 * it->second.losses.size());
  out->n_losses = (int32_t)it->second.losses.size();
  return FR_OK;
}

int fr_server_cancel(fr_server* s, uint64_t id) {
  if (!s) return FR_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->pub.count(id)) return FR_ERR_NOT_FOUND;
    s->cancels.push_back(id);
    s->idle = false;
  }
  s->cv.notify_all();
  return FR_OK;
}

int fr_server_forget(fr_server* s, uint64_t id) {
  if (!s) return FR_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->pub.find(id);
  if (it == s->pub.end()) return FR_ERR_NOT_FOUND;
  const int st = it->second.r.state;
  if (st == fr::REQ_QUEUED || st == fr::REQ_RUNNING) return FR_ERR_INVALID_ARG;
  s->pub.erase(it);
  return FR_OK;   // the scheduler's own record goes with the server
}

int fr_server_stats(fr_server* s, fr_stats* out) {
  if (!s || !out) return FR_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  const fr::SchedStats& t = s->stats;
  *out = fr_stats{};
  out->submitted = (int64_t)s->next_id - 1;
  out->completed = t.completed; out->failed = t.failed; out->cancelled = t.cancelled; out->rejected = t.rejected;
  out->queued = t.queued + (int32_t)s->inbox.size(); out->active = t.active; out->peak_active = t.peak_active;
  out->bytes_in_use = t.bytes_in_use; out->peak_bytes = t.peak_bytes;
  out->p50_s = t.p50; out->p99_s = t.p99; out->mean_s = t.mean; out->recons_per_s = t.recons_per_s;
  out->busy_s = t.busy_s; out->steps = t.steps; out->ticks = t.ticks;
  return FR_OK;
}

int fr_server_wait(fr_server* s, double timeout_s) {
  if (!s) return FR_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  const bool ok = s->cv_idle.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return s->idle; });
  return ok ? FR_OK : FR_ERR_LIMIT;
}

double fr_server_clock(fr_server* s) { return s ? s->ex.now() : -1.0; }

}  // extern "C"
