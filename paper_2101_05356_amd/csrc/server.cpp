// Reconstruction server: a worker thread that owns one HIP stream and one
// batch of jobs, and schedules submitted requests onto it with the
// continuous-batching policy of scheduler.h.  The device work goes through
// the batch entry points of the C ABI.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <vector>

#include "../../include/fr.h"
#include "server_core.h"

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
  double work(const Req& r) {
    const fr_job_desc& d = r.desc;
    return (double)d.width * (double)d.height * (double)d.spp * (1.0 + (double)d.n_lights);
  }
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
  // worker-thread set-up and tear-down
  int init() {
    if (hipSetDevice(fr::model_device(model)) != hipSuccess ||
        hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
      return FR_ERR_DEVICE;
    return FR_OK;
  }
  void shutdown() {
    fr_batch_destroy(batch);
    batch = nullptr;
    if (st) (void)hipStreamDestroy(st);
    st = nullptr;
  }
};

}  // namespace

struct fr_server {
  fr_model* model = nullptr;
  fr_server_opts opts{};
  BatchExec ex;
  fr::ServerCore<BatchExec>* core = nullptr;
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
  s->core = new fr::ServerCore<BatchExec>(s->ex, o->hbm_budget, o->max_slots, o->quantum, o->work_cap);
  const int rc = s->core->start();
  if (rc != FR_OK) {
    delete s->core;
    s->ex.shutdown();
    delete s;
    return rc;
  }
  *out = s;
  return FR_OK;
}

int fr_server_destroy(fr_server* s) {
  if (!s) return FR_OK;
  s->core->stop();   // the worker releases the batch and its stream
  delete s->core;
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
  return s->core->submit(std::move(r), rq->n_steps, id);
}

int fr_server_poll(fr_server* s, uint64_t id, fr_result* out, float* h_params, float* h_losses) {
  if (!s || !out) return FR_ERR_INVALID_ARG;
  return s->core->with_record(id, [&](const fr::PublishedReq& p) {
    *out = fr_result{};
    out->state = p.state; out->status = p.status; out->steps_done = p.steps_done; out->n_steps = p.n_steps;
    out->final_loss = p.final_loss; out->t_submit = p.t_submit; out->t_admit = p.t_admit; out->t_done = p.t_done;
    out->n_losses = (int32_t)p.losses.size();
    if (h_params && !p.params.empty()) std::memcpy(h_params, p.params.data(), 4 * p.params.size());
    if (h_losses && !p.losses.empty()) std::memcpy(h_losses, p.losses.data(), 4 * p.losses.size());
  });
}

int fr_server_cancel(fr_server* s, uint64_t id) {
  if (!s) return FR_ERR_INVALID_ARG;
  return s->core->cancel(id);
}

int fr_server_forget(fr_server* s, uint64_t id) {
  if (!s) return FR_ERR_INVALID_ARG;
  return s->core->forget(id);   // the scheduler's own record goes with the server
}

int fr_server_stats(fr_server* s, fr_stats* out) {
  if (!s || !out) return FR_ERR_INVALID_ARG;
  const fr::SchedStats t = s->core->stats();
  *out = fr_stats{};
  out->submitted = t.submitted;
  out->completed = t.completed; out->failed = t.failed; out->cancelled = t.cancelled; out->rejected = t.rejected;
  out->queued = t.queued; out->active = t.active; out->peak_active = t.peak_active;
  out->bytes_in_use = t.bytes_in_use; out->peak_bytes = t.peak_bytes;
  out->p50_s = t.p50; out->p99_s = t.p99; out->mean_s = t.mean; out->recons_per_s = t.recons_per_s;
  out->busy_s = t.busy_s; out->steps = t.steps; out->ticks = t.ticks;
  return FR_OK;
}

int fr_server_wait(fr_server* s, double timeout_s) {
  if (!s) return FR_ERR_INVALID_ARG;
  return s->core->wait(timeout_s) ? FR_OK : FR_ERR_LIMIT;
}

double fr_server_clock(fr_server* s) { return s ? s->ex.now() : -1.0; }

}  // extern "C"
