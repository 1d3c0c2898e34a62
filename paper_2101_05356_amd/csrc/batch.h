// Device descriptor of one reconstruction job and the host-side batch that
// steps many jobs with one launch per stage.
#pragma once

#include <vector>

#include "fr_kernels.h"

namespace fr {

// Everything a batched stage kernel needs about one job (device-resident).
struct JobDev {
  RenderArgs ra;            // forward view (light chunks for the forward)
  RenderArgs rb;            // backward view (light chunks for the backward)
  EdgeArgs ea;              // boundary term
  ShadowEdgeArgs se;        // shadow-edge boundary term (n_samples 0: off)
  const float* mean_geo; const float* basis_geo; const float* mean_alb; const float* basis_alb;
  int K_geo, K_alb, N, F, M;
  float* v_obj; float* v_w; float* diffuse;
  float* image; const float* target; float* dEdp; float* gsign; double* loss_part; float* loss;
  float* loss_hist; int hist_cap;
  float* g_verts; float* g_diffuse; float* g_vobj; float* gnorm; fix_t* lslots; int zero_stride;
  fix_t* acc;               // fixed-point accumulators: verts [3N], normals [3N], diffuse [3N]
  uint32_t* gmax;           // the sums' scale: bits of max |dE/dp| / spp = 1 / spp (grad_scale)
  float* param; float* grad; float* adam_m; float* adam_v; const float* lr;
  int n_param, off_alb, off_pose, off_rad;
  const int32_t* tris; const int32_t* vf_off; const int32_t* vf_idx; float* normals; float* nlen;
  BvhNode* nodes; Bvh4Node* nodes4; const int32_t* n4_src; int n4; TriRec* recs; const int32_t* order; const int32_t* node_parent; const int32_t* leaf_parent;
  uint32_t* flags;
  const int32_t* top_nodes; const int32_t* top_level_off; int n_top_levels;
  const int32_t* edge_faces; uint8_t* face_front; double* edge_len; double* edge_cdf; double* scan_part;
  const float* lp0; const float* le1; const float* le2; const int32_t* lshape; LightRec* lights;
  int smooth; Taps taps;
  int t;                    // completed steps; step t + 1 renders with counter word 4 = t + 1
};

// A set of jobs stepped together.  The host keeps a copy of the table; after
// adding or removing jobs, upload() refreshes the device table and drops the
// captured graph.
struct Batch {
  std::vector<JobDev> jobs;
  JobDev* d_jobs = nullptr;
  int* d_prefix = nullptr;
  int cap = 0, njobs_dev = 0, max_nl = 0;
  std::vector<int> total;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // second stream of the step: the boundary terms beside the interior adjoint
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  ~Batch();
  void make_aux();
  int upload(hipStream_t st);
  void launch_step(hipStream_t st);
  int step(hipStream_t st, int n, bool use_graph);
};

}  // namespace fr
