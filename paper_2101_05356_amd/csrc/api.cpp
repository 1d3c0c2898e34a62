// C ABI of the face renderer: argument checks, object lifetimes, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "fr_kernels.h"

struct fr_ctx {
  int device = 0;
  std::string last_error;
};

struct fr_mesh {
  fr_ctx* ctx = nullptr;
  fr::MeshDev d;
  std::vector<int32_t> h_edges, h_edge_faces;
  double* loss_scratch = nullptr;   // per-block loss partials
  float* loss_gtmp = nullptr;       // sign image before the adjoint smoothing
  int loss_cap = 0;
};

namespace {

int fail(fr_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

#define FR_HIP(ctx, expr)                                                             \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail((ctx), FR_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
hipError_t dalloc(T** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(n, 1) * sizeof(T));
}

bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int build_args(fr_mesh* m, const fr_scene* s, const fr_render_opts* o, fr::RenderArgs& a) {
  fr_ctx* ctx = m->ctx;
  if (!s || !o) return fail(ctx, FR_ERR_INVALID_ARG, "scene and opts are required");
  if (s->width <= 0 || s->height <= 0 || s->n_lights < 0)
    return fail(ctx, FR_ERR_INVALID_ARG, "image size must be positive and n_lights >= 0");
  if (!pow2(s->spp) || s->spp > 1024) return fail(ctx, FR_ERR_LIMIT, "spp must be a power of two in [1, 1024]");
  if ((long long)s->width * s->height > (1ll << 26)) return fail(ctx, FR_ERR_LIMIT, "image larger than 2^26 pixels");
  if (!s->verts || !s->diffuse || !s->specular || !s->roughness || !s->cam)
    return fail(ctx, FR_ERR_INVALID_ARG, "null scene pointer");
  if (s->n_lights > 0 && (!s->light_p0 || !s->light_e1 || !s->light_e2 || !s->light_rad || !s->light_shape))
    return fail(ctx, FR_ERR_INVALID_ARG, "null light pointer");
  if (!(s->fov_y > 0.0f && s->fov_y < 3.1f)) return fail(ctx, FR_ERR_INVALID_ARG, "fov_y must be in (0, 3.1)");
  if (o->brdf_variant != FR_BRDF_PRINTED && o->brdf_variant != FR_BRDF_NORMALIZED)
    return fail(ctx, FR_ERR_INVALID_ARG, "bad brdf_variant");
  if (m->d.built == 0) return fail(ctx, FR_ERR_INVALID_ARG, "fr_mesh_update(FR_REBUILD) must run first");
  const fr::MeshDev& d = m->d;
  a.nodes = d.nodes; a.recs = d.recs; a.tris = d.tris; a.verts = s->verts; a.normals = d.normals;
  a.diffuse = s->diffuse; a.specular = s->specular; a.roughness = s->roughness;
  a.lights = d.lights; a.cam = s->cam;
  a.N = d.N; a.F = d.F; a.L = s->n_lights;
  a.W = s->width; a.H = s->height; a.S = s->spp;
  a.lanes_per_pixel = std::min(a.S, 64);
  a.chunks = a.S > 64 ? a.S / 64 : 1;
  const int P = 64 / a.lanes_per_pixel;
  int lg = 0;
  while ((1 << lg) < P) ++lg;
  a.tile_w = 1 << ((lg + 1) / 2);
  a.tile_h = P / a.tile_w;
  a.tiles_x = (a.W + a.tile_w - 1) / a.tile_w;
  a.tiles_y = (a.H + a.tile_h - 1) / a.tile_h;
  a.n_tiles = a.tiles_x * a.tiles_y;
  a.tan_half = (float)std::tan(0.5 * (double)s->fov_y);
  a.aspect = (float)((double)a.W / (double)a.H);
  a.k0 = (uint32_t)(s->seed & 0xffffffffull);
  a.k1 = (uint32_t)(s->seed >> 32);
  a.step = s->step;
  a.variant = o->brdf_variant;
  a.components = o->components;
  a.dbg_hit = o->dbg_hit; a.dbg_pflag = o->dbg_pflag; a.dbg_vis = o->dbg_vis; a.dbg_stats = o->dbg_stats;
  return FR_OK;
}

int ensure_lights(fr_mesh* m, int L) {
  if (L <= m->d.light_cap) return FR_OK;
  if (m->d.lights) (void)hipFree(m->d.lights);
  if (m->d.ltmp) (void)hipFree(m->d.ltmp);
  m->d.lights = nullptr;
  m->d.ltmp = nullptr;
  const int cap = std::max(L, 128);
  if (dalloc(&m->d.lights, cap) != hipSuccess || dalloc(&m->d.ltmp, (size_t)cap * 12) != hipSuccess)
    return fail(m->ctx, FR_ERR_OOM, "light table allocation failed");
  m->d.light_cap = cap;
  return FR_OK;
}

}  // namespace

extern "C" {

const char* fr_status_string(int status) {
  switch (status) {
    case FR_OK: return "ok";
    case FR_ERR_INVALID_ARG: return "invalid argument";
    case FR_ERR_SHAPE: return "inconsistent shapes";
    case FR_ERR_OOM: return "device out of memory";
    case FR_ERR_BUDGET: return "request exceeds the HBM budget";
    case FR_ERR_DEVICE: return "HIP runtime error";
    case FR_ERR_NONFINITE: return "non-finite value";
    case FR_ERR_LIMIT: return "implementation limit exceeded";
    case FR_ERR_NOT_FOUND: return "unknown request";
    default: return "unknown status";
  }
}

const char* fr_last_error(const fr_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

int fr_ctx_create(int hip_device, fr_ctx** out) {
  if (!out) return FR_ERR_INVALID_ARG;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return FR_ERR_DEVICE;
  if (hipSetDevice(hip_device) != hipSuccess) return FR_ERR_DEVICE;
  fr_ctx* c = new fr_ctx();
  c->device = hip_device;
  *out = c;
  return FR_OK;
}

int fr_ctx_destroy(fr_ctx* ctx) {
  delete ctx;
  return FR_OK;
}

int fr_mesh_create(fr_ctx* ctx, int32_t n_verts, int32_t n_tris, const int32_t* h_tris, fr_mesh** out) {
  if (!ctx || !out || !h_tris) return fail(ctx, FR_ERR_INVALID_ARG, "null argument");
  if (n_verts < 3 || n_tris < 1) return fail(ctx, FR_ERR_INVALID_ARG, "need >= 3 vertices and >= 1 triangle");
  if (n_tris > (1 << 26)) return fail(ctx, FR_ERR_LIMIT, "more than 2^26 triangles");
  for (int64_t i = 0; i < 3ll * n_tris; ++i)
    if (h_tris[i] < 0 || h_tris[i] >= n_verts) return fail(ctx, FR_ERR_SHAPE, "triangle index out of range");
  FR_HIP(ctx, hipSetDevice(ctx->device));
  fr_mesh* m = new fr_mesh();
  m->ctx = ctx;
  fr::MeshDev& d = m->d;
  d.N = n_verts;
  d.F = n_tris;
  // vertex -> faces CSR (faces in increasing order)
  std::vector<int32_t> off(n_verts + 1, 0), idx(3 * (size_t)n_tris);
  for (int64_t i = 0; i < 3ll * n_tris; ++i) off[h_tris[i] + 1]++;
  for (int i = 0; i < n_verts; ++i) off[i + 1] += off[i];
  std::vector<int32_t> fill(off.begin(), off.end() - 1);
  for (int f = 0; f < n_tris; ++f)
    for (int k = 0; k < 3; ++k) idx[fill[h_tris[3 * f + k]]++] = f;
  // unique edges (lower vertex id first, sorted) and their faces
  std::map<std::pair<int, int>, std::pair<int, int>> em;
  for (int f = 0; f < n_tris; ++f)
    for (int k = 0; k < 3; ++k) {
      int a = h_tris[3 * f + k], b = h_tris[3 * f + (k + 1) % 3];
      if (a > b) std::swap(a, b);
      auto it = em.find({a, b});
      if (it == em.end()) em[{a, b}] = {f, -1};
      else if (it->second.second < 0) it->second.second = f;
    }
  d.E = (int)em.size();
  for (auto& kv : em) {
    m->h_edges.push_back(kv.first.first); m->h_edges.push_back(kv.first.second);
    m->h_edge_faces.push_back(kv.second.first); m->h_edge_faces.push_back(kv.second.second);
  }
  const int F = n_tris, NI = std::max(F - 1, 1), nb = (F + 1023) / 1024;
  bool ok = dalloc(&d.tris, 3 * (size_t)F) == hipSuccess && dalloc(&d.vf_off, n_verts + 1) == hipSuccess &&
            dalloc(&d.vf_idx, 3 * (size_t)F) == hipSuccess && dalloc(&d.normals, 3 * (size_t)n_verts) == hipSuccess &&
            dalloc(&d.nlen, n_verts) == hipSuccess && dalloc(&d.gnorm, 3 * (size_t)n_verts) == hipSuccess &&
            dalloc(&d.edges, 2 * (size_t)d.E) == hipSuccess && dalloc(&d.edge_faces, 2 * (size_t)d.E) == hipSuccess &&
            dalloc(&d.nodes, NI) == hipSuccess && dalloc(&d.recs, F) == hipSuccess && dalloc(&d.order, F) == hipSuccess &&
            dalloc(&d.node_parent, NI) == hipSuccess && dalloc(&d.leaf_parent, F) == hipSuccess &&
            dalloc(&d.flags, NI) == hipSuccess && dalloc(&d.keys[0], F) == hipSuccess &&
            dalloc(&d.keys[1], F) == hipSuccess && dalloc(&d.vals[0], F) == hipSuccess &&
            dalloc(&d.vals[1], F) == hipSuccess && dalloc(&d.hist, 256 * (size_t)nb) == hipSuccess &&
            dalloc(&d.partial, 64 * 6) == hipSuccess && dalloc(&d.scene_box, 6) == hipSuccess &&
            dalloc(&d.depth, 2) == hipSuccess && dalloc(&d.edge_len, d.E) == hipSuccess &&
            dalloc(&d.edge_cdf, d.E) == hipSuccess && dalloc(&d.face_front, F) == hipSuccess &&
            dalloc(&d.scan_part, 1024) == hipSuccess;
  if (!ok) { fr_mesh_destroy(m); return fail(ctx, FR_ERR_OOM, "mesh allocation failed"); }
  ok = hipMemcpy(d.tris, h_tris, sizeof(int32_t) * 3 * F, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(d.vf_off, off.data(), sizeof(int32_t) * (n_verts + 1), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(d.vf_idx, idx.data(), sizeof(int32_t) * 3 * F, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(d.edges, m->h_edges.data(), sizeof(int32_t) * 2 * d.E, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(d.edge_faces, m->h_edge_faces.data(), sizeof(int32_t) * 2 * d.E, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) { fr_mesh_destroy(m); return fail(ctx, FR_ERR_DEVICE, "mesh upload failed"); }
  *out = m;
  return FR_OK;
}

int fr_mesh_destroy(fr_mesh* m) {
  if (!m) return FR_OK;
  fr::MeshDev& d = m->d;
  void* ptrs[] = {d.tris, d.vf_off, d.vf_idx, d.normals, d.nlen, d.gnorm, d.edges, d.edge_faces, d.nodes, d.recs,
                  d.order, d.node_parent, d.leaf_parent, d.flags, d.keys[0], d.keys[1], d.vals[0], d.vals[1],
                  d.hist, d.partial, d.scene_box, d.depth, d.lights, d.ltmp, d.edge_len, d.edge_cdf, d.face_front,
                  d.scan_part, m->loss_scratch, m->loss_gtmp};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete m;
  return FR_OK;
}

int fr_mesh_update(fr_mesh* m, const float* d_verts, int mode, fr_stream stream) {
  if (!m || !d_verts) return FR_ERR_INVALID_ARG;
  fr_ctx* ctx = m->ctx;
  if (mode != FR_REFIT && mode != FR_REBUILD) return fail(ctx, FR_ERR_INVALID_ARG, "bad mode");
  if (mode == FR_REFIT && !m->d.built) return fail(ctx, FR_ERR_INVALID_ARG, "refit before the first build");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  fr::launch_normals(m->d, d_verts, st);
  if (mode == FR_REBUILD) {
    int depth = 0;
    const int rc = fr::bvh_build(m->d, d_verts, st, &depth);
    if (rc != FR_OK) { m->d.built = 0; return fail(ctx, rc, "BVH build failed (device error or invalid topology)"); }
    m->d.bvh_depth = depth;
    if (depth > fr::kStackDepth) {
      m->d.built = 0;
      return fail(ctx, FR_ERR_LIMIT, "BVH depth " + std::to_string(depth) + " exceeds the traversal stack");
    }
    m->d.built = 1;
  } else {
    fr::bvh_refit(m->d, d_verts, st);
  }
  FR_HIP(ctx, hipGetLastError());
  return FR_OK;
}

const float* fr_mesh_normals(const fr_mesh* m) { return m ? m->d.normals : nullptr; }

int32_t fr_mesh_edges(const fr_mesh* m, int32_t* h_edges, int32_t* h_faces) {
  if (!m) return -1;
  if (h_edges) std::memcpy(h_edges, m->h_edges.data(), sizeof(int32_t) * m->h_edges.size());
  if (h_faces) std::memcpy(h_faces, m->h_edge_faces.data(), sizeof(int32_t) * m->h_edge_faces.size());
  return m->d.E;
}

int32_t fr_mesh_bvh_depth(const fr_mesh* m) { return m ? m->d.bvh_depth : -1; }

int fr_render_forward(fr_mesh* m, const fr_scene* s, const fr_render_opts* o, float* d_image, fr_stream stream) {
  if (!m || !d_image) return FR_ERR_INVALID_ARG;
  fr::RenderArgs a;
  int rc = build_args(m, s, o, a);
  if (rc != FR_OK) return rc;
  const bool any_dbg = o->dbg_hit || o->dbg_pflag || o->dbg_vis || o->dbg_stats;
  if (any_dbg && !(o->dbg_hit && o->dbg_pflag && o->dbg_vis))
    return fail(m->ctx, FR_ERR_INVALID_ARG, "the forward dump needs dbg_hit, dbg_pflag and dbg_vis");
  if ((rc = ensure_lights(m, s->n_lights)) != FR_OK) return rc;
  a.lights = m->d.lights;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (s->n_lights > 0) fr::launch_light_setup(*s, m->d.lights, st);
  fr::launch_render_forward(a, d_image, st);
  FR_HIP(m->ctx, hipGetLastError());
  return FR_OK;
}

int fr_loss(const float* d_image, const float* d_target, int32_t W, int32_t H, int32_t smooth, float* d_loss,
            float* d_dEdp, fr_stream stream) {
  if (!d_image || !d_target || !d_loss || W <= 0 || H <= 0) return FR_ERR_INVALID_ARG;
  // scratch: per-block partial sums and the sign image (allocated per call size class)
  static thread_local double* scratch = nullptr;
  static thread_local float* gtmp = nullptr;
  static thread_local size_t cap = 0;
  const size_t npx = (size_t)W * H;
  if (npx > cap) {
    if (scratch) (void)hipFree(scratch);
    if (gtmp) (void)hipFree(gtmp);
    scratch = nullptr; gtmp = nullptr; cap = 0;
    if (dalloc(&scratch, (npx + 255) / 256) != hipSuccess || dalloc(&gtmp, 3 * npx) != hipSuccess)
      return FR_ERR_OOM;
    cap = npx;
  }
  fr::launch_loss(d_image, d_target, W, H, smooth, d_loss, d_dEdp, scratch, gtmp,
                  reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_render_backward(fr_mesh* m, const fr_scene* s, const fr_render_opts* o, const float* d_dEdp, fr_grads* g,
                       fr_stream stream) {
  if (!m || !d_dEdp || !g) return FR_ERR_INVALID_ARG;
  fr::RenderArgs a;
  int rc = build_args(m, s, o, a);
  if (rc != FR_OK) return rc;
  if (o->dbg_vis || (!o->dbg_hit) != (!o->dbg_pflag))
    return fail(m->ctx, FR_ERR_INVALID_ARG, "the backward dump takes dbg_hit and dbg_pflag only");
  a.dbg_hit = nullptr; a.dbg_pflag = nullptr; a.dbg_vis = nullptr; a.dbg_stats = nullptr;
  if ((rc = ensure_lights(m, s->n_lights)) != FR_OK) return rc;
  a.lights = m->d.lights;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (s->n_lights > 0) fr::launch_light_setup(*s, m->d.lights, st);
  fr::launch_zero(m->d.gnorm, 3 * m->d.N, st);
  fr::launch_render_backward(a, d_dEdp, *g, m->d.gnorm, st);
  if (g->normals) fr::launch_axpy(g->normals, m->d.gnorm, 3 * m->d.N, st);   // before the in-place projection
  if (g->verts) fr::launch_normals_backward(m->d, s->verts, m->d.gnorm, g->verts, st);
  const int ns = o->edge_samples < 0 ? s->width * s->height : o->edge_samples;
  if (ns > 0 && (g->verts || g->cam || o->dbg_hit))
    fr::launch_edges(m->d, a, d_dEdp, ns, *g, o->dbg_hit, o->dbg_pflag, std::tan(0.5 * (double)s->fov_y), st);
  FR_HIP(m->ctx, hipGetLastError());
  return FR_OK;
}

int fr_blend(const float* d_mean, const float* d_basis, const float* d_coef, int32_t K, int32_t M, float* d_out,
             fr_stream stream) {
  if (!d_mean || !d_basis || !d_coef || !d_out || K < 0 || M <= 0) return FR_ERR_INVALID_ARG;
  fr::launch_blend(d_mean, d_basis, d_coef, K, M, d_out, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_blend_backward(const float* d_basis, const float* d_gout, int32_t K, int32_t M, float* d_gcoef,
                      fr_stream stream) {
  if (!d_basis || !d_gout || !d_gcoef || K <= 0 || M <= 0) return FR_ERR_INVALID_ARG;
  fr::launch_blend_backward(d_basis, d_gout, K, M, d_gcoef, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_pose_forward(const float* d_v, int32_t n, const float* d_pose, float* d_vw, fr_stream stream) {
  if (!d_v || !d_pose || !d_vw || n <= 0) return FR_ERR_INVALID_ARG;
  fr::launch_pose(d_v, n, d_pose, d_vw, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_pose_backward(const float* d_v, int32_t n, const float* d_pose, const float* d_gw, float* d_gv, float* d_gpose,
                     fr_stream stream) {
  if (!d_v || !d_pose || !d_gw || n <= 0) return FR_ERR_INVALID_ARG;
  fr::launch_pose_backward(d_v, n, d_pose, d_gw, d_gv, d_gpose, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_adam_step(float* d_param, const float* d_grad, float* d_m, float* d_v, const float* d_lr, int32_t n, int32_t t,
                 float beta1, float beta2, float eps, fr_stream stream) {
  if (!d_param || !d_grad || !d_m || !d_v || !d_lr || n <= 0 || t < 1) return FR_ERR_INVALID_ARG;
  fr::launch_adam(d_param, d_grad, d_m, d_v, d_lr, n, t, beta1, beta2, eps, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

}  // extern "C"
