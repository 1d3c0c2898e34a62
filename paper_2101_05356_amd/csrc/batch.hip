// Batched optimisation step over many reconstructions ("jobs") at once.
//
// Every job is one face being reconstructed: its coefficients, pose and light
// radiances are optimised by Adam against its own target image (Sec. 4
// "Optimization strategy", Sec. 5 learning rates), with its own image size,
// samples per pixel and lights.  A step of ALL active jobs is one launch per
// stage: the grid of a stage is the concatenation of every job's blocks, and a
// block finds its job through a per-stage prefix table; job descriptors live
// in a device table.  The sequence of stage launches is captured once per job
// mix into a hipGraph and replayed every step; the step counters (Philox
// counter word 4 and Adam's t) advance on the device, so a replay needs no
// host work.
#include "fr_all.hip"
#include "batch.h"

namespace fr {

// ---------------------------------------------------------------------------
// Job table lookups
// ---------------------------------------------------------------------------
// Job of global block b: the last j with prefix[j] <= b (prefix[0] = 0).
__device__ __forceinline__ int job_of(const int* __restrict__ prefix, int njobs, int b, int& local) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
  }
  local = b - prefix[lo];
  return lo;
}

#define FR_JOB_PROLOGUE                                     \
  int lb;                                                   \
  const int jb = job_of(prefix, njobs, blockIdx.x, lb);    \
  if (lb >= prefix[jb + 1] - prefix[jb]) return;            \
  const JobDev& J = jobs[jb];

#define FR_BATCH_KERNEL(name, threads) \
  __global__ __launch_bounds__(threads) void name(const JobDev* __restrict__ jobs, const int* __restrict__ prefix, int njobs)

FR_BATCH_KERNEL(kb_blend_geo, 256) { FR_JOB_PROLOGUE blend_block(J.mean_geo, J.basis_geo, J.param, J.K_geo, J.M, J.v_obj, lb); }
FR_BATCH_KERNEL(kb_blend_alb, 256) {
  FR_JOB_PROLOGUE blend_block(J.mean_alb, J.basis_alb, J.param + J.off_alb, J.K_alb, J.M, J.diffuse, lb);
}
FR_BATCH_KERNEL(kb_pose, 256) { FR_JOB_PROLOGUE pose_block(J.v_obj, J.N, J.param + J.off_pose, J.v_w, lb); }
FR_BATCH_KERNEL(kb_normals, 256) {
  FR_JOB_PROLOGUE normals_block(J.v_w, J.tris, J.vf_off, J.vf_idx, J.N, J.normals, J.nlen, lb);
}
FR_BATCH_KERNEL(kb_refit, kRefitTile) {
  FR_JOB_PROLOGUE refit_local_block(J.v_w, J.tris, J.order, J.F, J.nodes, J.node_parent, J.leaf_parent, J.recs,
                                    kBoxPad, lb);
}
FR_BATCH_KERNEL(kb_refit_top, 1024) {
  FR_JOB_PROLOGUE refit_top_block(J.nodes, J.node_parent, J.top_nodes, J.top_level_off, J.n_top_levels);
}
FR_BATCH_KERNEL(kb_gather4, 256) { FR_JOB_PROLOGUE gather4_block(J.nodes, J.n4_src, J.n4, J.nodes4, lb); }
FR_BATCH_KERNEL(kb_light_setup, 256) {
  FR_JOB_PROLOGUE light_setup_block(J.lp0, J.le1, J.le2, J.param + J.off_rad, J.lshape, J.ra.L, J.lights, lb);
}
__attribute__((amdgpu_waves_per_eu(8))) FR_BATCH_KERNEL(kb_primary, 256) { FR_JOB_PROLOGUE primary_block<false>(J.ra, lb); }
__attribute__((amdgpu_waves_per_eu(8))) FR_BATCH_KERNEL(kb_render_fwd, 256) {
  FR_JOB_PROLOGUE render_fwd_block<false, false>(J.ra, J.ra.n_lchunks > 1 ? nullptr : J.image, lb);
}
FR_BATCH_KERNEL(kb_sum_chunks, 256) {
  FR_JOB_PROLOGUE sum_chunks_block(J.ra.partial, 3 * J.ra.W * J.ra.H, J.ra.n_lchunks, J.image, lb);
}
FR_BATCH_KERNEL(kb_loss, 256) {
  FR_JOB_PROLOGUE loss_block(J.image, J.target, J.ra.W, J.ra.H, J.smooth, J.taps, J.smooth ? J.gsign : J.dEdp,
                             J.loss_part, lb);
}
FR_BATCH_KERNEL(kb_loss_final, 256) {
  FR_JOB_PROLOGUE loss_final_block(J.loss_part, cdiv_d(J.ra.W * J.ra.H, 256), J.loss, lb);
  __syncthreads();
  if (threadIdx.x == 0 && J.t < J.hist_cap) J.loss_hist[J.t] = J.loss[0];
}
FR_BATCH_KERNEL(kb_smooth_adjoint, 256) {
  FR_JOB_PROLOGUE if (J.smooth) smooth_adjoint_block(J.gsign, J.ra.W, J.ra.H, J.taps, J.dEdp, lb);
}
// zero the gradient buffers: grad, g_vobj, the fixed-point accumulators, light slots
FR_BATCH_KERNEL(kb_zero_grads, 256) {
  FR_JOB_PROLOGUE
  const int i = lb * 256 + threadIdx.x;
  const int n9 = 9 * J.N;
  const int nslot = kSlots * (12 * J.ra.L + 12);
  if (i < J.n_param) J.grad[i] = 0.0f;
  if (i < 3 * J.N) J.g_vobj[i] = 0.0f;
  for (int k = i; k < n9; k += J.zero_stride) J.acc[k] = 0;
  for (int k = i; k < nslot; k += J.zero_stride) J.lslots[k] = 0;
}
// The adjoint takes the forward's shadow masks (J.rb.vis_in).
__attribute__((amdgpu_waves_per_eu(4))) FR_BATCH_KERNEL(kb_render_bwd, 256) {
  FR_JOB_PROLOGUE
  const FixGrads g = {J.acc, J.acc + 3 * J.N, J.acc + 6 * J.N, nullptr, nullptr};
  render_bwd_block<false, true>(J.rb, J.dEdp, g, J.lslots, lb);
}
// fixed-point vertex and diffuse gradients -> float
FR_BATCH_KERNEL(kb_fix_finalize, 256) {
  FR_JOB_PROLOGUE
  const int i = lb * 256 + threadIdx.x;
  if (i >= 3 * J.N) return;
  const double s = (double)grad_scale(J.gmax);
  J.g_verts[i] = (float)(from_fix(J.acc[i]) / s);
  J.g_diffuse[i] = (float)(from_fix(J.acc[6 * J.N + i]) / s);
}
FR_BATCH_KERNEL(kb_slots_reduce, 256) {
  FR_JOB_PROLOGUE slots_reduce_block(J.lslots, 12 * J.ra.L + 12, J.ra.L, nullptr, J.grad + J.off_rad, nullptr, nullptr,
                                     lb, J.gmax);
}
FR_BATCH_KERNEL(kb_normals_bwd_project, 256) {
  FR_JOB_PROLOGUE normals_bwd_project_block(J.v_w, J.tris, J.vf_off, J.vf_idx, J.N, J.acc + 3 * J.N, J.gnorm, lb);
}
FR_BATCH_KERNEL(kb_normals_bwd_gather, 256) {
  FR_JOB_PROLOGUE normals_bwd_gather_block(J.v_w, J.tris, J.vf_off, J.vf_idx, J.N, J.gnorm, J.acc, lb);
}
FR_BATCH_KERNEL(kb_face_front, 256) { FR_JOB_PROLOGUE face_front_block(J.v_w, J.tris, J.F, J.ra.cam, J.face_front, lb); }
FR_BATCH_KERNEL(kb_edge_len, 256) {
  FR_JOB_PROLOGUE edge_len_block(J.v_w, J.ea.edges, J.edge_faces, J.ea.E, J.face_front, J.ra.cam, J.ea.th,
                                 J.ea.aspect, J.ra.W, J.ra.H, J.edge_len, lb);
}
FR_BATCH_KERNEL(kb_edge_scan, 256) { FR_JOB_PROLOGUE edge_scan_local_block(J.edge_len, J.ea.E, J.edge_cdf, J.scan_part, lb); }
FR_BATCH_KERNEL(kb_edge_scan_add, 256) { FR_JOB_PROLOGUE edge_scan_add_block(J.edge_cdf, J.ea.E, J.scan_part, lb); }
__attribute__((amdgpu_waves_per_eu(8))) FR_BATCH_KERNEL(kb_edge_samples, 256) { FR_JOB_PROLOGUE edge_samples_block<false, false>(J.rb, J.ea, lb); }
// shadow-edge term into the vertex accumulators (its jumps' light points are
// shaded with the step's light records; the camera rays are traced again)
FR_BATCH_KERNEL(kb_shadow_edges, 256) {
  FR_JOB_PROLOGUE shadow_edge_sample<false, false>(J.rb, J.se, lb * 256 + (int)threadIdx.x);
}
FR_BATCH_KERNEL(kb_pose_bwd_v, 256) { FR_JOB_PROLOGUE pose_bwd_v_block(J.N, J.param + J.off_pose, J.g_verts, J.g_vobj, lb); }
FR_BATCH_KERNEL(kb_pose_bwd_p, 1024) {
  FR_JOB_PROLOGUE pose_bwd_p_block(J.v_obj, J.N, J.param + J.off_pose, J.g_verts, J.grad + J.off_pose, lb);
}
FR_BATCH_KERNEL(kb_blend_bwd_geo, 1024) { FR_JOB_PROLOGUE blend_bwd_block(J.basis_geo, J.g_vobj, J.M, J.grad, lb); }
FR_BATCH_KERNEL(kb_blend_bwd_alb, 1024) {
  FR_JOB_PROLOGUE blend_bwd_block(J.basis_alb, J.g_diffuse, J.M, J.grad + J.off_alb, lb);
}
FR_BATCH_KERNEL(kb_adam, 256) {
  FR_JOB_PROLOGUE
  const int t = J.t + 1;
  const float c1 = adam_bias(0.9f, t), c2 = adam_bias(0.999f, t);
  adam_block(J.param, J.grad, J.adam_m, J.adam_v, J.lr, J.n_param, 0.9f, 0.999f, 1e-8f, c1, c2, lb);
}
// Advance the step counters of every job.  Step k (1-based) renders with
// Philox counter word 4 = k and takes Adam's bias correction at t = k; J.t
// counts the completed steps.
__global__ void kb_advance(JobDev* jobs, int njobs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= njobs) return;
  jobs[j].t += 1;
  jobs[j].ra.step = (uint32_t)(jobs[j].t + 1);
  jobs[j].rb.step = (uint32_t)(jobs[j].t + 1);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
enum Stage {
  S_BLEND_GEO, S_BLEND_ALB, S_POSE, S_NORMALS, S_REFIT, S_REFIT_TOP, S_GATHER4, S_LIGHTS, S_PRIM, S_FWD, S_SUM, S_LOSS,
  S_LOSS_FINAL, S_SMOOTH_ADJ, S_ZERO_GRADS, S_BWD, S_SLOTS, S_NBWD_P, S_NBWD_G, S_FACE_FRONT, S_EDGE_LEN, S_EDGE_SCAN, S_EDGE_SCAN_ADD,
  S_EDGE_SAMPLES, S_SHADOW_EDGES, S_FIX_FINALIZE, S_POSE_BWD_V, S_POSE_BWD_P, S_BLEND_BWD_GEO, S_BLEND_BWD_ALB, S_ADAM, S_COUNT
};

static int stage_blocks(const JobDev& J, int s) {
  const int N = J.N, F = J.F, px = J.ra.W * J.ra.H;
  switch (s) {
    case S_BLEND_GEO: case S_BLEND_ALB: return cdiv(J.M, 256);
    case S_POSE: case S_POSE_BWD_V: return cdiv(N, 256);
    case S_NORMALS: case S_NBWD_P: case S_NBWD_G: return normals_blocks(N);
    case S_FIX_FINALIZE: return cdiv(3 * N, 256);
    case S_REFIT: return cdiv(F, kRefitTile);
    case S_REFIT_TOP: return J.n_top_levels > 0 ? 1 : 0;
    case S_FACE_FRONT: return cdiv(F, 256);
    case S_GATHER4: return cdiv(4 * J.n4, 256);
    case S_LIGHTS: return cdiv(J.ra.L, 256);
    case S_PRIM: return wave_blocks_items(J.ra, 1);
    case S_FWD: return wave_blocks_items(J.ra);
    case S_SUM: return J.ra.n_lchunks > 1 ? cdiv(3 * px, 256) : 0;
    case S_LOSS: case S_SMOOTH_ADJ: return cdiv(px, 256);
    case S_LOSS_FINAL: return 1;
    case S_ZERO_GRADS: return cdiv(std::max(J.n_param, 3 * N), 256);
    case S_BWD: return tile_blocks(J.rb);
    case S_SLOTS: return 12 * J.ra.L + 12;
    case S_EDGE_LEN: return J.ea.n_samples > 0 ? cdiv(J.ea.E, 256) : 0;
    case S_EDGE_SCAN: case S_EDGE_SCAN_ADD: return J.ea.n_samples > 0 ? cdiv(J.ea.E, kScanTile) : 0;
    case S_EDGE_SAMPLES: return J.ea.n_samples > 0 ? J.ea.bx * J.ea.n_groups : 0;
    case S_SHADOW_EDGES: return J.se.n_samples > 0 ? cdiv(J.se.n_samples, 256) : 0;
    case S_POSE_BWD_P: return 1;
    case S_BLEND_BWD_GEO: return J.K_geo;
    case S_BLEND_BWD_ALB: return J.K_alb;
    case S_ADAM: return cdiv(J.n_param, 256);
  }
  return 0;
}

Batch::~Batch() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (d_jobs) (void)hipFree(d_jobs);
  if (d_prefix) (void)hipFree(d_prefix);
  if (aux) (void)hipStreamDestroy(aux);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
}

// The step's second stream and its fork/join events (default priority); left
// null (the step then runs serially) if any cannot be made.
void Batch::make_aux() {
  if (aux) return;
  hipStream_t x = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) == hipSuccess &&
      hipEventCreateWithFlags(&e0, hipEventDisableTiming) == hipSuccess &&
      hipEventCreateWithFlags(&e1, hipEventDisableTiming) == hipSuccess) {
    aux = x; ev_fork = e0; ev_join = e1;
    return;
  }
  if (x) (void)hipStreamDestroy(x);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipGetLastError();
}

int Batch::upload(hipStream_t st) {
  const int nj = (int)jobs.size();
  if (exec) { (void)hipGraphExecDestroy(exec); exec = nullptr; }
  if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
  if (nj == 0) return FR_OK;
  if (nj > cap) {
    if (d_jobs) (void)hipFree(d_jobs);
    if (d_prefix) (void)hipFree(d_prefix);
    d_jobs = nullptr; d_prefix = nullptr;
    cap = std::max(nj, 2 * cap);
    if (hipMalloc(&d_jobs, sizeof(JobDev) * cap) != hipSuccess) return FR_ERR_OOM;
    if (hipMalloc(&d_prefix, sizeof(int) * S_COUNT * (cap + 1)) != hipSuccess) return FR_ERR_OOM;
  }
  std::vector<int> prefix((size_t)S_COUNT * (nj + 1), 0);
  total.assign(S_COUNT, 0);
  for (int s = 0; s < S_COUNT; ++s) {
    int acc = 0;
    for (int j = 0; j < nj; ++j) {
      prefix[(size_t)s * (nj + 1) + j] = acc;
      // keep each job's first block on XCD 0 so the render's XCD-aware mapping holds per job
      const int b = stage_blocks(jobs[j], s);
      acc += (s == S_PRIM || s == S_FWD || s == S_BWD) ? cdiv(b, 8) * 8 : b;
    }
    prefix[(size_t)s * (nj + 1) + nj] = acc;
    total[s] = acc;
  }
  max_nl = 0;
  for (auto& J : jobs) max_nl = std::max(max_nl, 12 * J.ra.L + 12);
  if (hipMemcpyAsync(d_jobs, jobs.data(), sizeof(JobDev) * nj, hipMemcpyHostToDevice, st) != hipSuccess)
    return FR_ERR_DEVICE;
  if (hipMemcpyAsync(d_prefix, prefix.data(), sizeof(int) * prefix.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return FR_ERR_DEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return FR_ERR_DEVICE;
  njobs_dev = nj;
  return FR_OK;
}

void Batch::launch_step(hipStream_t st) {
  const int nj = njobs_dev;
  auto P = [&](int s) { return d_prefix + (size_t)s * (nj + 1); };
  // Independent stages go to the second stream, forked from and joined back
  // to the step's stream by events (in a captured graph: parallel branches).
  // The same two events serve every fork/join pair: a wait binds to the
  // record enqueued before it.
  const hipStream_t main_st = st;
  const auto fork = [&]() {
    const bool f = aux && hipEventRecord(ev_fork, main_st) == hipSuccess &&
                   hipStreamWaitEvent(aux, ev_fork, 0) == hipSuccess;
    st = f ? aux : main_st;
    return f;
  };
  const auto join = [&](bool f) {
    if (f) {
      (void)hipEventRecord(ev_join, aux);
      (void)hipStreamWaitEvent(main_st, ev_join, 0);
    }
    st = main_st;
  };
#define FR_LAUNCH(kernel, stage, threads, lds)                                                      \
  if (total[stage] > 0)                                                                              \
    hipLaunchKernelGGL(kernel, dim3(total[stage]), dim3(threads), lds, st, d_jobs, P(stage), nj);
  // beside the geometry chain: the albedo blend, the light records and the
  // zeroing of this step's gradient accumulators (nothing reads them before
  // the adjoint)
  bool f = fork();
  FR_LAUNCH(kb_blend_alb, S_BLEND_ALB, 256, 0);
  FR_LAUNCH(kb_light_setup, S_LIGHTS, 256, 0);
  FR_LAUNCH(kb_zero_grads, S_ZERO_GRADS, 256, 0);
  st = main_st;
  FR_LAUNCH(kb_blend_geo, S_BLEND_GEO, 256, 0);
  FR_LAUNCH(kb_pose, S_POSE, 256, 0);
  FR_LAUNCH(kb_normals, S_NORMALS, 256, 0);
  FR_LAUNCH(kb_refit, S_REFIT, kRefitTile, 0);
  FR_LAUNCH(kb_refit_top, S_REFIT_TOP, 1024, 0);
  FR_LAUNCH(kb_gather4, S_GATHER4, 256, 0);
  join(f);
  // camera-ray hits of every sample, read by the forward and again by the
  // adjoint (nothing between them moves the geometry or the counters)
  FR_LAUNCH(kb_primary, S_PRIM, 256, 0);
  FR_LAUNCH(kb_render_fwd, S_FWD, 256, 0);
  FR_LAUNCH(kb_sum_chunks, S_SUM, 256, 0);
  FR_LAUNCH(kb_loss, S_LOSS, 256, 0);
  FR_LAUNCH(kb_loss_final, S_LOSS_FINAL, 256, 0);
  FR_LAUNCH(kb_smooth_adjoint, S_SMOOTH_ADJ, 256, 0);
  // the boundary terms beside the interior adjoint: both need only the zeroed
  // accumulators, the geometry and dE/dp, and add into the vertex
  // accumulators with integer atomics (order-free sums)
  f = fork();
  FR_LAUNCH(kb_face_front, S_FACE_FRONT, 256, 0);
  FR_LAUNCH(kb_edge_len, S_EDGE_LEN, 256, 0);
  FR_LAUNCH(kb_edge_scan, S_EDGE_SCAN, 256, 0);
  FR_LAUNCH(kb_edge_scan_add, S_EDGE_SCAN_ADD, 256, 0);
  FR_LAUNCH(kb_edge_samples, S_EDGE_SAMPLES, 256, 0);
  FR_LAUNCH(kb_shadow_edges, S_SHADOW_EDGES, 256, 0);
  st = main_st;
  FR_LAUNCH(kb_render_bwd, S_BWD, 256, max_nl * sizeof(fix_t) + kBwdPartBytes);
  FR_LAUNCH(kb_slots_reduce, S_SLOTS, 256, 0);
  FR_LAUNCH(kb_normals_bwd_project, S_NBWD_P, 256, 0);
  FR_LAUNCH(kb_normals_bwd_gather, S_NBWD_G, 256, 0);
  join(f);
  // (each cross-stream wait costs ~10 us even when already met, so the short
  // stages after the adjoint stay in one chain)
  FR_LAUNCH(kb_fix_finalize, S_FIX_FINALIZE, 256, 0);
  FR_LAUNCH(kb_pose_bwd_v, S_POSE_BWD_V, 256, 0);
  FR_LAUNCH(kb_pose_bwd_p, S_POSE_BWD_P, 1024, 0);
  FR_LAUNCH(kb_blend_bwd_geo, S_BLEND_BWD_GEO, 1024, 0);
  FR_LAUNCH(kb_blend_bwd_alb, S_BLEND_BWD_ALB, 1024, 0);
  FR_LAUNCH(kb_adam, S_ADAM, 256, 0);
#undef FR_LAUNCH
  hipLaunchKernelGGL(kb_advance, dim3(cdiv(nj, 256)), dim3(256), 0, st, d_jobs, nj);
}

int Batch::step(hipStream_t st, int n, bool use_graph) {
  if (njobs_dev == 0) return FR_OK;
  make_aux();
  if (!use_graph) {
    for (int i = 0; i < n; ++i) launch_step(st);
    return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
  }
  if (!exec) {
    // capture on a private stream so that the caller's stream is never in capture mode
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return FR_ERR_DEVICE;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return FR_ERR_DEVICE;
    }
    launch_step(cs);
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) return FR_ERR_DEVICE;
  }
  for (int i = 0; i < n; ++i)
    if (hipGraphLaunch(exec, st) != hipSuccess) return FR_ERR_DEVICE;
  return FR_OK;
}

}  // namespace fr
