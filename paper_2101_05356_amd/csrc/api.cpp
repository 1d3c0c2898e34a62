// C ABI of the face renderer: argument checks, object lifetimes, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "fr_kernels.h"

struct fr_ctx {
  int device = 0;
  std::string last_error;
};

// What the mesh's primary-hit buffer currently holds: the camera-ray hits of
// the render call with these inputs (valid = false: nothing usable); and
// whether its shadow-mask buffer holds that call's decisions for the lights
// below (kept by a forward asked to keep them).
struct LightKey {
  bool valid = false;
  int32_t L = 0, lc = 0;
  const float* p0 = nullptr;
  const float* e1 = nullptr;
  const float* e2 = nullptr;
  const int32_t* shape = nullptr;
  const void* buf = nullptr;
};

struct PrimKey {
  bool valid = false;
  int32_t W = 0, H = 0, S = 0;
  uint64_t seed = 0;
  uint32_t step = 0;
  float fov = 0.0f;
  const float* verts = nullptr;
  const float* cam = nullptr;
  const void* buf = nullptr;
  uint64_t version = 0;
  bool operator==(const PrimKey& o) const {
    return valid && o.valid && W == o.W && H == o.H && S == o.S && seed == o.seed && step == o.step &&
           std::memcmp(&fov, &o.fov, sizeof(float)) == 0 && verts == o.verts && cam == o.cam && buf == o.buf &&
           version == o.version;
  }
};

// What a caller's workspace holds from the last render call that used it:
// the camera-ray hits of the call with key `prim` (at the workspace's start)
// and, when a forward kept them, its shadow masks for the lights of `vis`
// (vis_bytes at offset vis_off).
struct WsState {
  PrimKey prim;
  LightKey vis;
  size_t vis_off = 0, vis_bytes = 0;
};

struct fr_mesh {
  fr_ctx* ctx = nullptr;
  fr::MeshDev d;
  uint64_t version = 0;   // bumped by every fr_mesh_update
  std::mutex mu;          // guards ws
  std::map<const void*, WsState> ws;   // keyed by workspace address
  std::vector<int32_t> h_edges, h_edge_faces;
  // the backward's second stream: the boundary term runs there beside the
  // interior adjoint (created by the first backward; default priority)
  std::mutex fork_mu;     // one backward's fork/join enqueue at a time
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
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

// Carves typed sub-buffers out of one allocation (256-byte aligned).
struct Carver {
  size_t off = 0;
  char* base = nullptr;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += sizeof(T) * std::max<size_t>(n, 1);
    return p;
  }
};

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// A render call's workspace: [camera-ray hits | light table | kept shadow
// masks | call region].  The hits and the masks carry a forward's decisions
// to the backward that takes them; the call region holds one call's scratch
// and nothing in it outlives the call.
size_t ws_prim_bytes(const fr_scene* s) {
  return al256((size_t)s->width * s->height * s->spp * sizeof(fr::PrimHit));
}
// the light records, then the device copies of the call's kernel arguments
size_t ws_light_rec_bytes(const fr_scene* s) { return al256((size_t)std::max(s->n_lights, 1) * sizeof(fr::LightRec)); }
size_t ws_light_bytes(const fr_scene* s) {
  return ws_light_rec_bytes(s) + al256(fr::kRenderArgSlots * sizeof(fr::RenderArgs));
}
fr::RenderArgs* ws_args(const fr_scene* s, char* base) {
  return reinterpret_cast<fr::RenderArgs*>(base + ws_prim_bytes(s) + ws_light_rec_bytes(s));
}
int fwd_chunk(const fr_render_opts* o) { return o->light_chunk > 0 ? o->light_chunk : fr::kLightChunkFwd; }
size_t ws_vis_bytes(const fr_scene* s, int lc) {
  return s->n_lights > 0 ? al256((size_t)fr::cdiv(s->n_lights, lc) * s->width * s->height * s->spp * 4) : 0;
}
// forward: the per-light-chunk partial images
size_t ws_fwd_region(const fr_scene* s, int lc) {
  const size_t nch = std::max(1, fr::cdiv(s->n_lights, lc));
  return nch > 1 ? al256(nch * 3 * (size_t)s->width * s->height * sizeof(float)) : 0;
}
// backward: fixed-point accumulators, the normals' adjoint, the light/camera
// slots, texel sums and the boundary term's silhouette CDF
struct BwdScratch {
  fr::fix_t* acc;        // [13N + 12]: verts, normals, diffuse, specular (3N each), roughness (N), camera (12)
  float* gnorm;          // [3N]
  fr::fix_t* slots;      // [kSlots (12 Lg + 12 + 3 B^2)]
  fr::fix_t* tex;        // [7 M^2]
  double* edge_len;      // [E]
  double* edge_cdf;      // [E]
  uint8_t* face_front;   // [F]
  double* scan_part;     // [ceil(E / 1024)]
};
size_t carve_bwd(const fr::MeshDev& d, const fr_scene* s, char* base, BwdScratch* out) {
  Carver c;
  c.base = base;
  BwdScratch b;
  const size_t N = d.N, Lg = std::min(s->n_lights, fr::kBwdMaxLights), B = std::max(s->sh_bands, 0);
  const size_t MM = (size_t)std::max(s->tex_size, 0) * std::max(s->tex_size, 0);
  b.acc = c.take<fr::fix_t>(13 * N + 13);   // the last word holds max |dE/dp| (float bits)
  b.gnorm = c.take<float>(3 * N);
  b.slots = c.take<fr::fix_t>((size_t)fr::kSlots * (12 * Lg + 12 + 3 * B * B));
  b.tex = MM > 0 ? c.take<fr::fix_t>(7 * MM) : nullptr;
  b.edge_len = c.take<double>(d.E);
  b.edge_cdf = c.take<double>(d.E);
  b.face_front = c.take<uint8_t>(d.F);
  b.scan_part = c.take<double>(std::max(1, (d.E + 1023) / 1024));
  if (out) *out = b;
  return al256(c.off);
}
// shadow-edge term: fixed-point sums of verts, light geometry, camera
// and one word for max |dE/dp|
size_t ws_se_region(const fr::MeshDev& d, const fr_scene* s) {
  return al256((3 * (size_t)d.N + 9 * (size_t)std::max(s->n_lights, 0) + 13) * sizeof(fr::fix_t));
}

// Constants of the SH lighting: A_l, the clamped cosine's SH coefficients
// (pi, 2 pi / 3, then 0 for odd l and 2 pi (-1)^(l/2+1) C(l, l/2) /
// (2^l (l + 2)(l - 1)) for even l), and the real-SH normalisation
// sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), times sqrt 2 for m > 0.
void sh_tables(fr::RenderArgs& a) {
  const double pi = 3.14159265358979323846;
  for (int l = 0; l < fr::kMaxShBands; ++l) {
    double A;
    if (l == 0) A = pi;
    else if (l == 1) A = 2.0 * pi / 3.0;
    else if (l & 1) A = 0.0;
    else {
      double binom = 1.0;                      // C(l, l/2)
      for (int k = 1; k <= l / 2; ++k) binom = binom * (l / 2 + k) / k;
      A = 2.0 * pi * ((l / 2) % 2 ? 1.0 : -1.0) * binom / (std::pow(2.0, l) * (l + 2.0) * (l - 1.0));
    }
    a.sh_ash[l] = (float)A;
    for (int m = 0; m <= l; ++m) {
      double r = 1.0;                          // (l-m)! / (l+m)!
      for (int k = l - m + 1; k <= l + m; ++k) r /= k;
      a.sh_norm[l * (l + 1) / 2 + m] = (float)(std::sqrt((2.0 * l + 1.0) / (4.0 * pi) * r) * (m > 0 ? std::sqrt(2.0) : 1.0));
    }
  }
}

int build_args(fr_mesh* m, const fr_scene* s, const fr_render_opts* o, fr::RenderArgs& a, int default_chunk) {
  fr_ctx* ctx = m->ctx;
  if (!s || !o) return fail(ctx, FR_ERR_INVALID_ARG, "scene and opts are required");
  if (s->width <= 0 || s->height <= 0 || s->n_lights < 0)
    return fail(ctx, FR_ERR_INVALID_ARG, "image size must be positive and n_lights >= 0");
  if (!pow2(s->spp) || s->spp > 1024) return fail(ctx, FR_ERR_LIMIT, "spp must be a power of two in [1, 1024]");
  if ((long long)s->width * s->height > (1ll << 26)) return fail(ctx, FR_ERR_LIMIT, "image larger than 2^26 pixels");
  if (s->tex_size < 0 || s->tex_size > 16384) return fail(ctx, FR_ERR_LIMIT, "tex_size must be in [0, 16384]");
  if (o->shadow_traversal != 0 && o->shadow_traversal != 1)
    return fail(ctx, FR_ERR_INVALID_ARG, "shadow_traversal must be 0 (wave packet) or 1 (per lane)");
  const bool maps = s->tex_size > 0;
  if (!s->verts || !s->cam || (!maps && (!s->diffuse || !s->specular || !s->roughness)))
    return fail(ctx, FR_ERR_INVALID_ARG, "null scene pointer");
  if (maps && (!s->tex_uv || !s->tex_diffuse || !s->tex_specular || !s->tex_roughness))
    return fail(ctx, FR_ERR_INVALID_ARG, "null reflectance-map pointer");
  if (s->n_lights > 0 && (!s->light_p0 || !s->light_e1 || !s->light_e2 || !s->light_rad || !s->light_shape))
    return fail(ctx, FR_ERR_INVALID_ARG, "null light pointer");
  if (!(s->fov_y > 0.0f && s->fov_y < 3.1f)) return fail(ctx, FR_ERR_INVALID_ARG, "fov_y must be in (0, 3.1)");
  if (o->brdf_variant != FR_BRDF_PRINTED && o->brdf_variant != FR_BRDF_NORMALIZED)
    return fail(ctx, FR_ERR_INVALID_ARG, "bad brdf_variant");
  if (m->d.built == 0) return fail(ctx, FR_ERR_INVALID_ARG, "fr_mesh_update(FR_REBUILD) must run first");
  const fr::MeshDev& d = m->d;
  a.nodes = d.nodes4; a.recs = d.recs; a.tris = d.tris; a.verts = s->verts; a.normals = d.normals;
  a.diffuse = s->diffuse; a.specular = s->specular; a.roughness = s->roughness;
  a.lights = nullptr; a.cam = s->cam;   // the light table: set by the caller
  a.M = maps ? s->tex_size : 0;
  a.uv = maps ? s->tex_uv : nullptr;
  a.tex_c = maps ? s->tex_diffuse : nullptr;
  a.tex_s = maps ? s->tex_specular : nullptr;
  a.tex_r = maps ? s->tex_roughness : nullptr;
  a.N = d.N; a.F = d.F; a.L = s->n_lights;
  a.W = s->width; a.H = s->height; a.S = s->spp;
  a.lanes_per_pixel = std::min(a.S, 64);
  a.chunks = a.S > 64 ? a.S / 64 : 1;
  const int P = 64 / a.lanes_per_pixel;
  int lg = 0;
  while ((1 << lg) < P) ++lg;
  a.tile_w = 1 << ((lg + 1) / 2);
  a.tile_h = P / a.tile_w;
  if (o->light_chunk < 0 || o->light_chunk > 32)
    return fail(ctx, FR_ERR_INVALID_ARG, "light_chunk must be in [0, 32]");
  a.lc = o->light_chunk > 0 ? o->light_chunk : default_chunk;
  a.shadow_traversal = o->shadow_traversal;
  a.gmax = nullptr;
  a.n_lchunks = std::max(1, (s->n_lights + a.lc - 1) / a.lc);
  a.partial = nullptr;
  a.prim = nullptr;   // set by the caller (from its workspace, or a job's own buffer)
  a.vis_out = nullptr; a.vis_in = nullptr; a.vis_lc = 0;
  a.light0 = 0;
  if (s->sh_bands < 0 || s->sh_bands > fr::kMaxShBands || (s->sh_bands > 0 && !s->sh))
    return fail(ctx, FR_ERR_INVALID_ARG, "sh_bands must be in [0, 11] with sh given");
  a.sh = s->sh_bands > 0 ? s->sh : nullptr;
  a.sh_bands = s->sh_bands;
  sh_tables(a);
  a.tiles_x = (a.W + a.tile_w - 1) / a.tile_w;
  a.tiles_y = (a.H + a.tile_h - 1) / a.tile_h;
  a.n_tiles = a.tiles_x * a.tiles_y;
  a.tan_half_d = std::tan(0.5 * (double)s->fov_y);
  a.aspect_d = (double)a.W / (double)a.H;
  a.tan_half = (float)a.tan_half_d;
  a.aspect = (float)a.aspect_d;
  a.k0 = (uint32_t)(s->seed & 0xffffffffull);
  a.k1 = (uint32_t)(s->seed >> 32);
  a.step = s->step;
  a.variant = o->brdf_variant;
  a.components = o->components;
  a.dbg_hit = o->dbg_hit; a.dbg_pflag = o->dbg_pflag; a.dbg_vis = o->dbg_vis; a.dbg_stats = o->dbg_stats;
  return FR_OK;
}

// Host-side topology of a mesh: triangles, vertex->face CSR (faces in
// increasing order), unique edges (lower id first, sorted) and their faces.
struct HostTopo {
  int N = 0, F = 0;
  std::vector<int32_t> tris, off, idx, edges, edge_faces;
};

int build_topology(fr_ctx* ctx, int32_t n_verts, int32_t n_tris, const int32_t* h_tris, HostTopo& t) {
  if (n_verts < 3 || n_tris < 1) return fail(ctx, FR_ERR_INVALID_ARG, "need >= 3 vertices and >= 1 triangle");
  if (n_tris > (1 << 26)) return fail(ctx, FR_ERR_LIMIT, "more than 2^26 triangles");
  for (int64_t i = 0; i < 3ll * n_tris; ++i)
    if (h_tris[i] < 0 || h_tris[i] >= n_verts) return fail(ctx, FR_ERR_SHAPE, "triangle index out of range");
  t.N = n_verts;
  t.F = n_tris;
  t.tris.assign(h_tris, h_tris + 3ll * n_tris);
  t.off.assign(n_verts + 1, 0);
  t.idx.assign(3 * (size_t)n_tris, 0);
  for (int64_t i = 0; i < 3ll * n_tris; ++i) t.off[h_tris[i] + 1]++;
  for (int i = 0; i < n_verts; ++i) t.off[i + 1] += t.off[i];
  std::vector<int32_t> fill(t.off.begin(), t.off.end() - 1);
  for (int f = 0; f < n_tris; ++f)
    for (int k = 0; k < 3; ++k) t.idx[fill[h_tris[3 * f + k]]++] = f;
  std::map<std::pair<int, int>, std::pair<int, int>> em;
  for (int f = 0; f < n_tris; ++f)
    for (int k = 0; k < 3; ++k) {
      int a = h_tris[3 * f + k], b = h_tris[3 * f + (k + 1) % 3];
      if (a > b) std::swap(a, b);
      auto it = em.find({a, b});
      if (it == em.end()) em[{a, b}] = {f, -1};
      else if (it->second.second < 0) it->second.second = f;
    }
  for (auto& kv : em) {
    t.edges.push_back(kv.first.first); t.edges.push_back(kv.first.second);
    t.edge_faces.push_back(kv.second.first); t.edge_faces.push_back(kv.second.second);
  }
  return FR_OK;
}

// with_scratch: the mesh also holds the per-call buffers of the adjoint
// (fixed-point sums, the normals' adjoint, the silhouette CDF), which a batch
// job's step uses in place of a caller's workspace.
int mesh_from_topology(fr_ctx* ctx, const HostTopo& t, bool with_scratch, fr_mesh** out) {
  FR_HIP(ctx, hipSetDevice(ctx->device));
  fr_mesh* m = new fr_mesh();
  m->ctx = ctx;
  fr::MeshDev& d = m->d;
  d.N = t.N;
  d.F = t.F;
  d.E = (int)(t.edges.size() / 2);
  m->h_edges = t.edges;
  m->h_edge_faces = t.edge_faces;
  const int F = t.F, NI = std::max(F - 1, 1), nb = (F + 1023) / 1024, n_verts = t.N;
  bool ok = dalloc(&d.tris, 3 * (size_t)F) == hipSuccess && dalloc(&d.vf_off, n_verts + 1) == hipSuccess &&
            dalloc(&d.vf_idx, 3 * (size_t)F) == hipSuccess && dalloc(&d.normals, 3 * (size_t)n_verts) == hipSuccess &&
            dalloc(&d.nlen, n_verts) == hipSuccess &&
            dalloc(&d.edges, 2 * (size_t)d.E) == hipSuccess && dalloc(&d.edge_faces, 2 * (size_t)d.E) == hipSuccess &&
            dalloc(&d.nodes, NI) == hipSuccess && dalloc(&d.recs, F + 1) == hipSuccess &&
            dalloc(&d.order, F) == hipSuccess && dalloc(&d.node_parent, NI) == hipSuccess &&
            dalloc(&d.leaf_parent, F) == hipSuccess && dalloc(&d.flags, NI) == hipSuccess &&
            dalloc(&d.keys[0], F) == hipSuccess && dalloc(&d.keys[1], F) == hipSuccess &&
            dalloc(&d.vals[0], F) == hipSuccess && dalloc(&d.vals[1], F) == hipSuccess &&
            dalloc(&d.hist, 256 * (size_t)nb) == hipSuccess && dalloc(&d.partial, 64 * 6) == hipSuccess &&
            dalloc(&d.scene_box, 6) == hipSuccess && dalloc(&d.depth, 2) == hipSuccess;
  if (ok && with_scratch)
    ok = dalloc(&d.gnorm, 3 * (size_t)n_verts) == hipSuccess && dalloc(&d.edge_len, d.E) == hipSuccess &&
         dalloc(&d.edge_cdf, d.E) == hipSuccess && dalloc(&d.face_front, F) == hipSuccess &&
         dalloc(&d.scan_part, (size_t)std::max(1, (d.E + 1023) / 1024)) == hipSuccess &&
         dalloc(&d.acc, 13 * (size_t)n_verts + 12) == hipSuccess;
  if (!ok) { fr_mesh_destroy(m); return fail(ctx, FR_ERR_OOM, "mesh allocation failed"); }
  ok = hipMemcpy(d.tris, t.tris.data(), sizeof(int32_t) * 3 * F, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(d.vf_off, t.off.data(), sizeof(int32_t) * (n_verts + 1), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(d.vf_idx, t.idx.data(), sizeof(int32_t) * 3 * F, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(d.edges, t.edges.data(), sizeof(int32_t) * 2 * d.E, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(d.edge_faces, t.edge_faces.data(), sizeof(int32_t) * 2 * d.E, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) { fr_mesh_destroy(m); return fail(ctx, FR_ERR_DEVICE, "mesh upload failed"); }
  // face across each edge of each face (the shadow-edge term's adjacency)
  std::vector<int32_t> nbr(3 * (size_t)F, -1);
  for (size_t e = 0; e < t.edges.size() / 2; ++e) {
    const int a = t.edges[2 * e], b = t.edges[2 * e + 1];
    const int fs[2] = {t.edge_faces[2 * e], t.edge_faces[2 * e + 1]};
    for (int q = 0; q < 2; ++q) {
      const int f = fs[q];
      if (f < 0) continue;
      for (int k = 0; k < 3; ++k) {
        const int i = t.tris[3 * (size_t)f + k], j = t.tris[3 * (size_t)f + (k + 1) % 3];
        if ((i == a && j == b) || (i == b && j == a)) nbr[3 * (size_t)f + k] = fs[1 - q];
      }
    }
  }
  if (dalloc(&d.face_nbr, 3 * (size_t)F) != hipSuccess ||
      hipMemcpy(d.face_nbr, nbr.data(), sizeof(int32_t) * 3 * F, hipMemcpyHostToDevice) != hipSuccess) {
    fr_mesh_destroy(m);
    return fail(ctx, FR_ERR_DEVICE, "mesh upload failed");
  }
  *out = m;
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
  // the static scratch of fr_loss_noalloc on this device
  if (!fr::noalloc_scratch(hip_device)) return FR_ERR_DEVICE;
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
  HostTopo topo;
  int rc = build_topology(ctx, n_verts, n_tris, h_tris, topo);
  if (rc != FR_OK) return rc;
  return mesh_from_topology(ctx, topo, false, out);
}

int fr_mesh_destroy(fr_mesh* m) {
  if (!m) return FR_OK;
  fr::MeshDev& d = m->d;
  void* ptrs[] = {d.tris, d.vf_off, d.vf_idx, d.normals, d.nlen, d.gnorm, d.edges, d.edge_faces, d.face_nbr, d.nodes, d.recs,
                  d.order, d.node_parent, d.leaf_parent, d.flags, d.keys[0], d.keys[1], d.vals[0], d.vals[1],
                  d.hist, d.partial, d.scene_box, d.depth, d.edge_len, d.edge_cdf, d.face_front,
                  d.scan_part, d.acc, d.nodes4, d.n4_src, d.top_nodes, d.top_level_off};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (m->aux) (void)hipStreamDestroy(m->aux);   // released once its work is done
  if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
  if (m->ev_join) (void)hipEventDestroy(m->ev_join);
  delete m;
  return FR_OK;
}

int fr_mesh_update(fr_mesh* m, const float* d_verts, int mode, fr_stream stream) {
  if (!m || !d_verts) return FR_ERR_INVALID_ARG;
  fr_ctx* ctx = m->ctx;
  if (mode != FR_REFIT && mode != FR_REBUILD && mode != FR_REBUILD_SAH)
    return fail(ctx, FR_ERR_INVALID_ARG, "bad mode");
  if (mode == FR_REFIT && !m->d.built) return fail(ctx, FR_ERR_INVALID_ARG, "refit before the first build");
  ++m->version;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  fr::launch_normals(m->d, d_verts, st);
  if (mode != FR_REFIT) {
    int depth = 0;
    const int rc = fr::bvh_build(m->d, d_verts, st, mode == FR_REBUILD_SAH, &depth);
    if (rc != FR_OK) { m->d.built = 0; return fail(ctx, rc, "BVH build failed (device error or invalid topology)"); }
    m->d.bvh_depth = depth;
    // the 4-wide traversal pushes at most three entries per level
    if (depth > fr::kStackDepth || 3 * m->d.depth4 > fr::kStackDepth) {
      m->d.built = 0;
      return fail(ctx, FR_ERR_LIMIT, "BVH depth " + std::to_string(depth) + " (4-wide " +
                                         std::to_string(m->d.depth4) + ") exceeds the traversal stack");
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

// The backward's light chunks: the four waves of a block take a tile's
// chunks of one light group (at most 128 lights), so lc >= ceil(L_group / 4)
// (at most 32 lights per chunk).  The adjoint launcher recomputes them per
// group; a batch job (at most 128 lights) has one group.
int bwd_chunks(fr_mesh* m, fr::RenderArgs& a) {
  const int Lg = std::min(a.L, fr::kBwdMaxLights);
  a.lc = std::max(a.lc, std::max(1, fr::cdiv(Lg, 4)));
  if (a.lc > 32) return fail(m->ctx, FR_ERR_LIMIT, "light_chunk must be <= 32");
  a.n_lchunks = std::max(1, fr::cdiv(Lg, a.lc));
  return FR_OK;
}

PrimKey prim_key_of(const fr_mesh* m, const fr_scene* s, const void* ws) {
  PrimKey k;
  k.valid = true;
  k.W = s->width; k.H = s->height; k.S = s->spp;
  k.seed = s->seed; k.step = s->step; k.fov = s->fov_y;
  k.verts = s->verts; k.cam = s->cam;
  k.buf = ws;
  k.version = m->version;
  return k;
}

LightKey light_key_of(const fr_scene* s, int lc, const void* ws) {
  LightKey k;
  k.valid = true;
  k.L = s->n_lights; k.lc = lc;
  k.p0 = s->light_p0; k.e1 = s->light_e1; k.e2 = s->light_e2; k.shape = s->light_shape;
  k.buf = ws;
  return k;
}

bool same_lights(const LightKey& a, const LightKey& b) {
  return a.valid && b.valid && a.L == b.L && a.p0 == b.p0 && a.e1 == b.e1 && a.e2 == b.e2 && a.shape == b.shape &&
         a.buf == b.buf;
}

// The caller's workspace of a render call: its base, and what it holds from
// the last call that used it.  Kept shadow masks count only where this call's
// layout puts them (right after its light table); a call whose hits or light
// table would cover them forgets them.
int ws_open(fr_mesh* m, const fr_scene* s, const fr_render_opts* o, char** base, WsState* st) {
  if (!o->workspace)
    return fail(m->ctx, FR_ERR_INVALID_ARG, "opts->workspace is required (size from fr_render_workspace_size)");
  if (reinterpret_cast<uintptr_t>(o->workspace) & 255)
    return fail(m->ctx, FR_ERR_INVALID_ARG, "opts->workspace must be 256-byte aligned");
  *base = static_cast<char*>(o->workspace);
  std::lock_guard<std::mutex> lk(m->mu);
  *st = m->ws[o->workspace];
  if (st->vis.valid && st->vis_off != ws_prim_bytes(s) + ws_light_bytes(s)) st->vis = LightKey{};
  if (!st->vis.valid) st->vis_off = st->vis_bytes = 0;
  return FR_OK;
}

int ws_need(fr_mesh* m, const fr_render_opts* o, size_t need) {
  if (o->workspace_bytes < need)
    return fail(m->ctx, FR_ERR_SHAPE, "workspace of " + std::to_string(o->workspace_bytes) + " bytes; this call needs " +
                                          std::to_string(need));
  return FR_OK;
}

void ws_store(fr_mesh* m, const void* base, const WsState& st) {
  std::lock_guard<std::mutex> lk(m->mu);
  m->ws[base] = st;
}

int fr_render_workspace_size(const fr_mesh* m, const fr_scene* s, const fr_render_opts* o, size_t* bytes) {
  if (!m || !s || !o || !bytes) return FR_ERR_INVALID_ARG;
  if (s->width <= 0 || s->height <= 0 || s->spp <= 0 || s->n_lights < 0 || s->tex_size < 0 || s->sh_bands < 0 ||
      o->light_chunk < 0 || o->light_chunk > 32)
    return FR_ERR_INVALID_ARG;
  const int lc = fwd_chunk(o);
  const size_t region = std::max({ws_fwd_region(s, lc), carve_bwd(m->d, s, nullptr, nullptr), ws_se_region(m->d, s)});
  *bytes = ws_prim_bytes(s) + ws_light_bytes(s) + (o->keep_shadows ? ws_vis_bytes(s, lc) : 0) + region;
  return FR_OK;
}

int fr_render_forward(fr_mesh* m, const fr_scene* s, const fr_render_opts* o, float* d_image, fr_stream stream) {
  if (!m || !d_image) return FR_ERR_INVALID_ARG;
  fr::RenderArgs a;
  int rc = build_args(m, s, o, a, fr::kLightChunkFwd);
  if (rc != FR_OK) return rc;
  const bool any_dbg = o->dbg_hit || o->dbg_pflag || o->dbg_vis || o->dbg_stats;
  if (any_dbg && !(o->dbg_hit && o->dbg_pflag && o->dbg_vis))
    return fail(m->ctx, FR_ERR_INVALID_ARG, "the forward dump needs dbg_hit, dbg_pflag and dbg_vis");
  char* base = nullptr;
  WsState st;
  if ((rc = ws_open(m, s, o, &base, &st)) != FR_OK) return rc;
  const bool keep = o->keep_shadows && s->n_lights > 0;
  const size_t pb = ws_prim_bytes(s), lb = ws_light_bytes(s), vb = keep ? ws_vis_bytes(s, a.lc) : 0;
  if ((rc = ws_need(m, o, pb + lb + vb + ws_fwd_region(s, a.lc))) != FR_OK) return rc;
  a.prim = reinterpret_cast<fr::PrimHit*>(base);
  fr::LightRec* lights = reinterpret_cast<fr::LightRec*>(base + pb);
  a.lights = lights;
  if (keep) {
    a.vis_out = reinterpret_cast<uint32_t*>(base + pb + lb);
    a.vis_lc = a.lc;
  }
  if (a.n_lchunks > 1) a.partial = reinterpret_cast<float*>(base + pb + lb + vb);
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  if (s->n_lights > 0) fr::launch_light_setup(*s, lights, hs);
  fr::launch_render_forward(a, ws_args(s, base), d_image, hs, static_cast<hipEvent_t>(o->ev_kernel_begin),
                            static_cast<hipEvent_t>(o->ev_kernel_end));
  FR_HIP(m->ctx, hipGetLastError());
  WsState now;
  now.prim = prim_key_of(m, s, base);
  if (keep) {
    now.vis = light_key_of(s, a.lc, base);
    now.vis_off = pb + lb;
    now.vis_bytes = vb;
  }
  ws_store(m, base, now);
  return FR_OK;
}

size_t fr_loss_workspace_size(int32_t W, int32_t H, int32_t smooth) {
  return W > 0 && H > 0 ? fr::loss_scratch_bytes(W, H, smooth != 0) : 0;
}

int fr_loss(const float* d_image, const float* d_target, int32_t W, int32_t H, int32_t smooth, float* d_loss,
            float* d_dEdp, void* d_work, size_t work_bytes, fr_stream stream) {
  if (!d_image || !d_target || !d_loss || !d_work || W <= 0 || H <= 0) return FR_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(d_work) & 255) return FR_ERR_INVALID_ARG;
  if (work_bytes < fr::loss_scratch_bytes(W, H, smooth != 0)) return FR_ERR_SHAPE;
  Carver c;
  c.base = static_cast<char*>(d_work);
  double* part = c.take<double>(((size_t)W * H + 255) / 256);
  float* gtmp = smooth ? c.take<float>(3 * (size_t)W * H) : nullptr;
  fr::launch_loss(d_image, d_target, W, H, smooth, d_loss, d_dEdp, part, gtmp, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_landmark_loss(const float* d_verts, const int32_t* d_idx, int32_t n, const float* d_cam, float fov_y, int32_t W,
                     int32_t H, const float* d_z, float* d_loss, float* d_gverts, float* d_gcam, fr_stream stream) {
  if (!d_verts || !d_idx || !d_cam || !d_z || !d_loss || n < 0 || W <= 0 || H <= 0 || !(fov_y > 0.0f && fov_y < 3.1f))
    return FR_ERR_INVALID_ARG;
  fr::launch_landmarks(d_verts, d_idx, n, d_cam, std::tan(0.5f * fov_y), W, H, d_z, d_loss, d_gverts, d_gcam,
                       reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_prior(const float* d_x, const float* d_sigma, int32_t n, int32_t kind, float weight, float* d_loss, float* d_g,
             fr_stream stream) {
  if (!d_x || !d_loss || n < 0 || kind < FR_PRIOR_STATISTICAL || kind > FR_PRIOR_LIGHT_CHROMA ||
      (kind == FR_PRIOR_STATISTICAL && !d_sigma) || (kind == FR_PRIOR_LIGHT_CHROMA && n % 3))
    return FR_ERR_INVALID_ARG;
  fr::launch_prior(d_x, d_sigma, n, kind, weight, d_loss, d_g, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

size_t fr_map_regularizers_workspace_size(int32_t M) { return M > 0 ? fr::map_reg_scratch_bytes(M) : 0; }

int fr_map_regularizers(const float* d_c, const float* d_s, const float* d_r, const float* d_c0, const float* d_s0,
                        int32_t M, const fr_map_reg_weights* w, float* d_loss, float* d_gc, float* d_gs, float* d_gr,
                        void* d_work, size_t work_bytes, fr_stream stream) {
  if (!d_c || !d_s || !d_r || !d_c0 || !d_s0 || !w || !d_loss || !d_work || M <= 0 || M > 16384)
    return FR_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(d_work) & 255) return FR_ERR_INVALID_ARG;
  if (work_bytes < fr::map_reg_scratch_bytes(M)) return FR_ERR_SHAPE;
  const fr::MapRegWeights mw{w->w_sym, w->w_chroma, w->w_smooth, w->w_box};
  fr::launch_map_regularizers(d_c, d_s, d_r, d_c0, d_s0, M, mw, d_loss, d_gc, d_gs, d_gr, static_cast<double*>(d_work),
                              reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_render_backward(fr_mesh* m, const fr_scene* s, const fr_render_opts* o, const float* d_dEdp, fr_grads* g,
                       fr_stream stream) {
  if (!m || !d_dEdp || !g) return FR_ERR_INVALID_ARG;
  fr::RenderArgs a;
  int rc = build_args(m, s, o, a, 1);
  if (rc != FR_OK) return rc;
  if (o->dbg_vis || (!o->dbg_hit) != (!o->dbg_pflag))
    return fail(m->ctx, FR_ERR_INVALID_ARG, "the backward dump takes dbg_hit and dbg_pflag only");
  if ((rc = bwd_chunks(m, a)) != FR_OK) return rc;
  a.dbg_hit = nullptr; a.dbg_pflag = nullptr; a.dbg_vis = nullptr; a.dbg_stats = nullptr;
  char* base = nullptr;
  WsState st;
  if ((rc = ws_open(m, s, o, &base, &st)) != FR_OK) return rc;
  const size_t pb = ws_prim_bytes(s), lb = ws_light_bytes(s);
  // the call's scratch goes after any kept shadow masks, used here or not
  const size_t roff = pb + lb + st.vis_bytes;
  BwdScratch w;
  if ((rc = ws_need(m, o, roff + carve_bwd(m->d, s, base + roff, &w))) != FR_OK) return rc;
  a.prim = reinterpret_cast<fr::PrimHit*>(base);
  fr::LightRec* lights = reinterpret_cast<fr::LightRec*>(base + pb);
  a.lights = lights;
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  // the mesh's buffers, with the per-call ones from the workspace
  fr::MeshDev d = m->d;
  d.acc = w.acc; d.gnorm = w.gnorm; d.edge_len = w.edge_len; d.edge_cdf = w.edge_cdf; d.face_front = w.face_front;
  d.scan_part = w.scan_part;
  // fixed-point accumulators: verts, normals, diffuse, specular (3N each), roughness (N), camera (12)
  const size_t N = d.N;
  fr::fix_t* acc_v = d.acc;
  fr::fix_t* acc_n = d.acc + 3 * N;
  fr::fix_t* acc_c = d.acc + 6 * N;
  fr::fix_t* acc_s = d.acc + 9 * N;
  fr::fix_t* acc_r = d.acc + 12 * N;
  fr::fix_t* acc_cam = d.acc + 13 * N;
  // max |dE/dp| / spp (the largest per-sample seed) sets the power-of-two
  // scale of the fixed-point sums
  uint32_t* gmax = reinterpret_cast<uint32_t*>(d.acc + 13 * N + 12);
  fr::launch_zero_fix(d.acc, 13 * N + 13, hs);
  fr::launch_abs_max(d_dEdp, 3 * a.W * a.H, a.S, gmax, hs);
  a.gmax = gmax;
  // texel accumulators [7 M^2]: diffuse, specular (3 M^2 each), roughness (M^2)
  const size_t MM = (size_t)a.M * a.M;
  const bool want_tex = a.M > 0 && (g->tex_diffuse || g->tex_specular || g->tex_roughness);
  if (want_tex) fr::launch_zero_fix(w.tex, 7 * MM, hs);
  if (s->n_lights > 0) fr::launch_light_setup(*s, lights, hs);
  const bool want_n = g->normals || g->verts;
  const bool vtx_refl = a.M == 0;
  fr::FixGrads fg = {g->verts ? acc_v : nullptr, want_n ? acc_n : nullptr,
                     vtx_refl && g->diffuse ? acc_c : nullptr, vtx_refl && g->specular ? acc_s : nullptr,
                     vtx_refl && g->roughness ? acc_r : nullptr, nullptr, nullptr, nullptr};
  if (want_tex) {
    fg.tex_c = g->tex_diffuse ? w.tex : nullptr;
    fg.tex_s = g->tex_specular ? w.tex + 3 * MM : nullptr;
    fg.tex_r = g->tex_roughness ? w.tex + 6 * MM : nullptr;
  }
  const PrimKey key = prim_key_of(m, s, base);
  const bool reuse = o->reuse_forward && st.prim == key;
  const bool use_vis = reuse && s->n_lights > 0 && same_lights(st.vis, light_key_of(s, st.vis.lc, base));
  if (use_vis) {
    a.vis_in = reinterpret_cast<const uint32_t*>(base + st.vis_off);
    a.vis_lc = st.vis.lc;
  }
  // The primary-visibility term (Sec. 4 "Edge Sampling") needs only the zeroed
  // accumulators, the geometry and dE/dp: it runs on the mesh's second stream
  // beside the interior adjoint, both adding into the vertex accumulators with
  // integer atomics (the sums do not depend on the order).  Serial on the
  // caller's stream if that stream cannot be made.
  const int ns = o->edge_samples < 0 ? s->width * s->height : o->edge_samples;
  const bool with_edges = ns > 0 && (g->verts || g->cam || o->dbg_hit);
  const auto edges_on = [&](hipStream_t es) {
    fr::launch_edges(d, a, d_dEdp, ns, g->verts ? acc_v : nullptr, g->cam ? acc_cam : nullptr, o->dbg_hit,
                     o->dbg_pflag, std::tan(0.5 * (double)s->fov_y), es);
  };
  std::unique_lock<std::mutex> fork(m->fork_mu, std::defer_lock);
  bool forked = false;
  if (with_edges) {
    fork.lock();
    if (!m->aux) {
      hipStream_t x = nullptr;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) == hipSuccess &&
          hipEventCreateWithFlags(&e0, hipEventDisableTiming) == hipSuccess &&
          hipEventCreateWithFlags(&e1, hipEventDisableTiming) == hipSuccess) {
        m->aux = x; m->ev_fork = e0; m->ev_join = e1;
      } else {
        if (x) (void)hipStreamDestroy(x);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipGetLastError();
      }
    }
    if (m->aux) {
      FR_HIP(m->ctx, hipEventRecord(m->ev_fork, hs));
      FR_HIP(m->ctx, hipStreamWaitEvent(m->aux, m->ev_fork, 0));
      edges_on(m->aux);
      FR_HIP(m->ctx, hipEventRecord(m->ev_join, m->aux));
      forked = true;
    }
  }
  fr::launch_render_backward(a, ws_args(s, base), d_dEdp, fg, w.slots, *g, hs,
                             static_cast<hipEvent_t>(o->ev_kernel_begin), static_cast<hipEvent_t>(o->ev_kernel_end),
                             !reuse);
  FR_HIP(m->ctx, hipGetLastError());
  // the hits now belong to this call; the masks stay only if they were this call's
  WsState now;
  now.prim = key;
  if (use_vis) { now.vis = st.vis; now.vis_off = st.vis_off; now.vis_bytes = st.vis_bytes; }
  ws_store(m, base, now);
  if (g->normals) fr::launch_fix_to_float(acc_n, g->normals, 3 * d.N, hs, gmax);
  if (g->verts) fr::launch_normals_backward(d, s->verts, acc_n, d.gnorm, acc_v, hs);
  if (with_edges && !forked) edges_on(hs);
  if (forked) FR_HIP(m->ctx, hipStreamWaitEvent(hs, m->ev_join, 0));
  if (fork.owns_lock()) fork.unlock();
  if (g->verts) fr::launch_fix_to_float(acc_v, g->verts, 3 * d.N, hs, gmax);
  if (fg.diffuse) fr::launch_fix_to_float(acc_c, g->diffuse, 3 * d.N, hs, gmax);
  if (fg.specular) fr::launch_fix_to_float(acc_s, g->specular, 3 * d.N, hs, gmax);
  if (fg.roughness) fr::launch_fix_to_float(acc_r, g->roughness, d.N, hs, gmax);
  if (fg.tex_c) fr::launch_fix_to_float(fg.tex_c, g->tex_diffuse, (int)(3 * MM), hs, gmax);
  if (fg.tex_s) fr::launch_fix_to_float(fg.tex_s, g->tex_specular, (int)(3 * MM), hs, gmax);
  if (fg.tex_r) fr::launch_fix_to_float(fg.tex_r, g->tex_roughness, (int)MM, hs, gmax);
  if (g->cam) fr::launch_fix_to_float(acc_cam, g->cam, 12, hs, gmax);
  FR_HIP(m->ctx, hipGetLastError());
  return FR_OK;
}

int fr_shadow_edges(fr_mesh* m, const fr_scene* s, const fr_render_opts* o, const float* d_dEdp, int32_t n_samples,
                    fr_grads* g, int32_t* d_rec, uint8_t* d_flag, fr_stream stream) {
  if (!m || !d_dEdp || !g || n_samples < 0) return FR_ERR_INVALID_ARG;
  if ((!d_rec) != (!d_flag)) return fail(m->ctx, FR_ERR_INVALID_ARG, "the shadow-edge dump takes d_rec and d_flag together");
  fr::RenderArgs a;
  int rc = build_args(m, s, o, a, 1);
  if (rc != FR_OK) return rc;
  if ((long long)s->width * s->height * s->spp >= (1ll << 31))
    return fail(m->ctx, FR_ERR_LIMIT, "the shadow-edge term needs W*H*spp < 2^31");
  a.dbg_hit = nullptr; a.dbg_pflag = nullptr; a.dbg_vis = nullptr; a.dbg_stats = nullptr;
  char* base = nullptr;
  WsState st;
  if ((rc = ws_open(m, s, o, &base, &st)) != FR_OK) return rc;
  const size_t pb = ws_prim_bytes(s), lb = ws_light_bytes(s), roff = pb + lb + st.vis_bytes;
  const size_t N = m->d.N, L = s->n_lights, nacc = 3 * N + 9 * L + 13;
  if ((rc = ws_need(m, o, roff + ws_se_region(m->d, s))) != FR_OK) return rc;
  // the hits and any kept masks stay as they are (this call traces its own camera rays)
  ws_store(m, base, st);
  if (n_samples == 0 || L == 0) return FR_OK;
  fr::LightRec* lights = reinterpret_cast<fr::LightRec*>(base + pb);
  a.lights = lights;
  fr::fix_t* acc = reinterpret_cast<fr::fix_t*>(base + roff);
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  uint32_t* gmax = reinterpret_cast<uint32_t*>(acc + nacc - 1);   // max |dE/dp| / spp: the sums' scale
  fr::launch_zero_fix(acc, nacc, hs);
  fr::launch_abs_max(d_dEdp, 3 * s->width * s->height, s->spp, gmax, hs);
  fr::launch_light_setup(*s, lights, hs);
  fr::ShadowEdgeArgs e;
  e.nbr = m->d.face_nbr;
  e.n_samples = n_samples;
  e.dEdp = d_dEdp;
  e.gverts = g->verts ? acc : nullptr;
  e.glight = g->light_geom ? acc + 3 * N : nullptr;
  e.gcam = g->cam ? acc + 3 * N + 9 * L : nullptr;
  e.dbg_rec = d_rec;
  e.dbg_flag = d_flag;
  e.gmax = gmax;
  fr::launch_shadow_edges(a, e, hs);
  FR_HIP(m->ctx, hipGetLastError());
  if (g->verts) fr::launch_fix_to_float(acc, g->verts, (int)(3 * N), hs, gmax);
  if (g->light_geom) fr::launch_fix_to_float(acc + 3 * N, g->light_geom, (int)(9 * L), hs, gmax);
  if (g->cam) fr::launch_fix_to_float(acc + 3 * N + 9 * L, g->cam, 12, hs, gmax);
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

int fr_light_stage(const float* d_faces, const float* d_params, int32_t n, float* d_p0, float* d_e1, float* d_e2,
                   float* d_rad, int32_t* d_shape, fr_stream stream) {
  if (!d_faces || !d_params || n < 0) return FR_ERR_INVALID_ARG;
  if (n > 0) fr::launch_light_stage(d_faces, d_params, n, d_p0, d_e1, d_e2, d_rad, d_shape,
                                    reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_light_stage_backward(const float* d_faces, const float* d_params, int32_t n, const float* d_g_geom,
                            const float* d_g_rad, float* d_gparams, fr_stream stream) {
  if (!d_faces || !d_params || !d_gparams || n < 0) return FR_ERR_INVALID_ARG;
  if (n > 0) fr::launch_light_stage_backward(d_faces, d_params, n, d_g_geom, d_g_rad, d_gparams,
                                             reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_pose_backward(const float* d_v, int32_t n, const float* d_pose, const float* d_gw, float* d_gv, float* d_gpose,
                     fr_stream stream) {
  if (!d_v || !d_pose || !d_gw || n <= 0) return FR_ERR_INVALID_ARG;
  fr::launch_pose_backward(d_v, n, d_pose, d_gw, d_gv, d_gpose, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_bake_vertex_map(const int32_t* d_tris, const float* d_uv, int32_t n_tris, const float* d_attr, int32_t channels,
                       int32_t M, float* d_map, fr_stream stream) {
  if (!d_tris || !d_uv || !d_attr || !d_map || n_tris < 0 || channels < 1 || channels > 4 || M <= 0 || M > 16384)
    return FR_ERR_INVALID_ARG;
  fr::launch_bake_map(d_tris, d_uv, n_tris, d_attr, channels, M, d_map, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_axpy(float* d_y, const float* d_x, float a, const float* d_s, int32_t n, fr_stream stream) {
  if (!d_y || !d_x || n < 0) return FR_ERR_INVALID_ARG;
  fr::launch_axpy(d_y, d_x, a, d_s, n, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_adam_step(float* d_param, const float* d_grad, float* d_m, float* d_v, const float* d_lr, int32_t n, int32_t t,
                 float beta1, float beta2, float eps, fr_stream stream) {
  if (!d_param || !d_grad || !d_m || !d_v || !d_lr || n <= 0 || t < 1) return FR_ERR_INVALID_ARG;
  fr::launch_adam(d_param, d_grad, d_m, d_v, d_lr, n, t, beta1, beta2, eps, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

}  // extern "C"

// ===========================================================================
// Batched reconstruction jobs
// ===========================================================================
#include "batch.h"

struct fr_model {
  fr_ctx* ctx = nullptr;
  HostTopo topo;
  const float* mean_geo = nullptr; const float* basis_geo = nullptr; int K_geo = 0;
  const float* mean_alb = nullptr; const float* basis_alb = nullptr; int K_alb = 0;
  const float* specular = nullptr; const float* roughness = nullptr;
};

namespace {

struct JobHost {
  fr_mesh* mesh = nullptr;
  char* arena = nullptr;
  size_t bytes = 0;
  int n_param = 0, W = 0, H = 0, hist_cap = 0;
  fr::JobDev dev{};
};

// Lays out (base == nullptr: only sizes) the device buffers of one job.
void layout_job(Carver& c, const fr_model* md, const fr_job_desc* d, fr::JobDev& J, int n_lchunks) {
  const size_t N3 = 3 * (size_t)md->topo.N, px3 = 3 * (size_t)d->width * d->height;
  const int L = d->n_lights;
  const int n_param = md->K_geo + md->K_alb + 6 + 3 * L;
  J.v_obj = c.take<float>(N3); J.v_w = c.take<float>(N3); J.diffuse = c.take<float>(N3);
  J.g_verts = c.take<float>(N3); J.g_diffuse = c.take<float>(N3); J.g_vobj = c.take<float>(N3);
  J.image = c.take<float>(px3); J.dEdp = c.take<float>(px3); J.gsign = c.take<float>(px3);
  J.target = c.take<float>(px3);
  J.ra.partial = n_lchunks > 1 ? c.take<float>(px3 * n_lchunks) : nullptr;
  J.ra.prim = c.take<fr::PrimHit>((size_t)d->width * d->height * d->spp);
  J.ra.vis_out = L > 0 ? c.take<uint32_t>((size_t)n_lchunks * d->width * d->height * d->spp) : nullptr;
  J.loss_part = c.take<double>(fr::cdiv(d->width * d->height, 256));
  J.loss = c.take<float>(1);
  J.loss_hist = c.take<float>(std::max(d->hist_cap, 1));
  J.lslots = c.take<fr::fix_t>((size_t)fr::kSlots * (12 * L + 12));
  J.param = c.take<float>(n_param); J.grad = c.take<float>(n_param);
  J.adam_m = c.take<float>(n_param); J.adam_v = c.take<float>(n_param); J.lr = c.take<float>(n_param);
  J.lights = c.take<fr::LightRec>(L);
  J.lp0 = c.take<float>(3 * L); J.le1 = c.take<float>(3 * L); J.le2 = c.take<float>(3 * L);
  J.lshape = c.take<int32_t>(L);
  J.ra.cam = c.take<float>(12);
  J.gmax = c.take<uint32_t>(1);
}

int validate_job(fr_model* md, const fr_job_desc* d) {
  fr_ctx* ctx = md->ctx;
  if (!d) return fail(ctx, FR_ERR_INVALID_ARG, "null job description");
  if (d->width <= 0 || d->height <= 0 || d->n_lights <= 0) return fail(ctx, FR_ERR_INVALID_ARG, "bad job sizes");
  if (d->n_lights > fr::kBwdMaxLights) return fail(ctx, FR_ERR_LIMIT, "a job takes at most 128 lights");
  if (!pow2(d->spp) || d->spp > 1024) return fail(ctx, FR_ERR_LIMIT, "spp must be a power of two in [1, 1024]");
  if (!d->cam || !d->light_p0 || !d->light_e1 || !d->light_e2 || !d->light_shape || !d->target || !d->params ||
      !d->lr)
    return fail(ctx, FR_ERR_INVALID_ARG, "null job pointer");
  if (!(d->fov_y > 0.0f && d->fov_y < 3.1f)) return fail(ctx, FR_ERR_INVALID_ARG, "fov_y must be in (0, 3.1)");
  if (d->edge_samples < -1 || d->shadow_edge_samples < -1)
    return fail(ctx, FR_ERR_INVALID_ARG, "edge sample counts must be -1 (W*H) or >= 0");
  return FR_OK;
}

}  // namespace

namespace fr {
int model_device(const fr_model* m) { return m->ctx->device; }
}  // namespace fr

struct fr_batch {
  fr_model* model = nullptr;
  fr::Batch b;
  std::map<int32_t, JobHost*> jobs;
  int32_t next_id = 1;
  bool dirty = false;
};

extern "C" {

int fr_model_create(fr_ctx* ctx, int32_t n_verts, int32_t n_tris, const int32_t* h_tris, const float* d_mean_geo,
                    const float* d_basis_geo, int32_t K_geo, const float* d_mean_alb, const float* d_basis_alb,
                    int32_t K_alb, const float* d_specular, const float* d_roughness, fr_model** out) {
  if (!ctx || !out || !h_tris || !d_mean_geo || !d_mean_alb || !d_specular || !d_roughness || K_geo < 0 ||
      K_alb < 0 || (K_geo > 0 && !d_basis_geo) || (K_alb > 0 && !d_basis_alb))
    return fail(ctx, FR_ERR_INVALID_ARG, "bad model arguments");
  fr_model* m = new fr_model();
  m->ctx = ctx;
  const int rc = build_topology(ctx, n_verts, n_tris, h_tris, m->topo);
  if (rc != FR_OK) { delete m; return rc; }
  m->mean_geo = d_mean_geo; m->basis_geo = d_basis_geo; m->K_geo = K_geo;
  m->mean_alb = d_mean_alb; m->basis_alb = d_basis_alb; m->K_alb = K_alb;
  m->specular = d_specular; m->roughness = d_roughness;
  *out = m;
  return FR_OK;
}

int fr_model_destroy(fr_model* m) {
  delete m;
  return FR_OK;
}

int32_t fr_model_n_param(const fr_model* m, int32_t n_lights) {
  return m ? m->K_geo + m->K_alb + 6 + 3 * n_lights : -1;
}

size_t fr_job_bytes(const fr_model* m, const fr_job_desc* d) {
  if (!m || !d || d->n_lights <= 0 || d->width <= 0 || d->height <= 0) return 0;
  fr::JobDev J{};
  Carver c;
  layout_job(c, m, d, J, std::max(1, fr::cdiv(d->n_lights, fr::kLightChunkFwd)));
  const size_t F = m->topo.F, N = m->topo.N, E = m->topo.edges.size() / 2;
  // mesh: topology, normals, BVH (64-byte binary nodes, 4-wide nodes for about
  // half of them, 48-byte records), sort buffers, edge tables, accumulators
  const size_t mesh = F * (12 + 12 + 64 + 80 + 48 + 4 * 8 + 1) + N * (4 + 4 * 7 + 13 * 8) + E * (16 + 16);
  return c.off + mesh;
}

int fr_batch_create(fr_model* model, fr_batch** out) {
  if (!model || !out) return FR_ERR_INVALID_ARG;
  fr_batch* b = new fr_batch();
  b->model = model;
  *out = b;
  return FR_OK;
}

int fr_batch_destroy(fr_batch* b) {
  if (!b) return FR_OK;
  for (auto& kv : b->jobs) {
    fr_mesh_destroy(kv.second->mesh);
    if (kv.second->arena) (void)hipFree(kv.second->arena);
    delete kv.second;
  }
  delete b;
  return FR_OK;
}

int fr_batch_add(fr_batch* b, const fr_job_desc* d, int32_t* job_id, fr_stream stream) {
  if (!b || !job_id) return FR_ERR_INVALID_ARG;
  fr_model* md = b->model;
  fr_ctx* ctx = md->ctx;
  int rc = validate_job(md, d);
  if (rc != FR_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  JobHost* jh = new JobHost();
  rc = mesh_from_topology(ctx, md->topo, true, &jh->mesh);
  if (rc != FR_OK) { delete jh; return rc; }
  fr::JobDev& J = jh->dev;
  const int L = d->n_lights;
  const int nch_f = std::max(1, fr::cdiv(L, fr::kLightChunkFwd));
  Carver sizing;
  layout_job(sizing, md, d, J, nch_f);
  if (hipMalloc(reinterpret_cast<void**>(&jh->arena), sizing.off) != hipSuccess) {
    fr_mesh_destroy(jh->mesh);
    delete jh;
    return fail(ctx, FR_ERR_OOM, "job allocation failed");
  }
  jh->bytes = sizing.off;
  Carver c;
  c.base = jh->arena;
  layout_job(c, md, d, J, nch_f);
  const int n_param = md->K_geo + md->K_alb + 6 + 3 * L;
  jh->n_param = n_param; jh->W = d->width; jh->H = d->height; jh->hist_cap = std::max(d->hist_cap, 1);
  const size_t px3 = 3 * (size_t)d->width * d->height;
  auto cp = [&](const void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(const_cast<void*>(dst), src, bytes, hipMemcpyDefault, st) == hipSuccess;
  };
  // the sums' scale as a per-call backward takes it when max |dE/dp| = 1
  // (the batch's dE/dp is the photometric loss's smoothed sign image): the
  // bits of 1 / spp, copied from static storage so that no error path can
  // free the source of the asynchronous copy
  static const float kInvSpp[11] = {1.0f,       0.5f,        0.25f,        0.125f,        0.0625f,      0.03125f,
                                    0.015625f,  0.0078125f,  0.00390625f,  0.001953125f,  0.0009765625f};
  int log2_spp = 0;
  while ((1 << log2_spp) < d->spp) ++log2_spp;   // spp: a power of two in [1, 1024] (validate_job)
  bool ok = cp(J.gmax, &kInvSpp[log2_spp], 4) &&
            cp(J.param, d->params, 4 * n_param) && cp(J.lr, d->lr, 4 * n_param) && cp(J.target, d->target, 4 * px3) &&
            cp(J.lp0, d->light_p0, 12 * L) && cp(J.le1, d->light_e1, 12 * L) && cp(J.le2, d->light_e2, 12 * L) &&
            cp(J.lshape, d->light_shape, 4 * L) && cp(J.ra.cam, d->cam, 48);
  ok = ok && hipMemsetAsync(J.adam_m, 0, 4 * n_param, st) == hipSuccess &&
       hipMemsetAsync(J.adam_v, 0, 4 * n_param, st) == hipSuccess &&
       hipMemsetAsync(J.loss_hist, 0, 4 * jh->hist_cap, st) == hipSuccess;
  if (!ok) { fr_mesh_destroy(jh->mesh); (void)hipFree(jh->arena); delete jh; return fail(ctx, FR_ERR_DEVICE, "job upload"); }
  // initial geometry and BVH
  const int N = md->topo.N, M = 3 * N;
  fr::launch_blend(md->mean_geo, md->basis_geo, J.param, md->K_geo, M, J.v_obj, st);
  fr::launch_blend(md->mean_alb, md->basis_alb, J.param + md->K_geo, md->K_alb, M, J.diffuse, st);
  fr::launch_pose(J.v_obj, N, J.param + md->K_geo + md->K_alb, J.v_w, st);
  rc = fr_mesh_update(jh->mesh, J.v_w, FR_REBUILD_SAH, stream);
  if (rc != FR_OK) { fr_mesh_destroy(jh->mesh); (void)hipFree(jh->arena); delete jh; return rc; }
  // render views
  fr_scene sc{};
  sc.width = d->width; sc.height = d->height; sc.spp = d->spp; sc.n_lights = L;
  sc.verts = J.v_w; sc.diffuse = J.diffuse; sc.specular = md->specular; sc.roughness = md->roughness;
  sc.light_p0 = J.lp0; sc.light_e1 = J.le1; sc.light_e2 = J.le2; sc.light_rad = J.param + n_param - 3 * L;
  sc.light_shape = J.lshape; sc.cam = J.ra.cam; sc.fov_y = d->fov_y; sc.step = 0; sc.seed = d->seed;
  fr_render_opts o{};
  o.brdf_variant = d->brdf_variant;
  o.components = 3;
  float* partial = J.ra.partial;
  fr::PrimHit* prim = J.ra.prim;
  uint32_t* vis = J.ra.vis_out;
  const float* cam = J.ra.cam;
  if ((rc = build_args(jh->mesh, &sc, &o, J.ra, fr::kLightChunkFwd)) != FR_OK ||
      (rc = build_args(jh->mesh, &sc, &o, J.rb, 1)) != FR_OK || (rc = bwd_chunks(jh->mesh, J.rb)) != FR_OK) {
    fr_mesh_destroy(jh->mesh); (void)hipFree(jh->arena); delete jh; return rc;
  }
  J.ra.partial = partial; J.rb.partial = nullptr;
  J.ra.prim = prim; J.rb.prim = prim;
  // the adjoint reads the forward's shadow decisions (same step, geometry and lights)
  J.ra.vis_out = vis; J.ra.vis_lc = J.ra.lc;
  J.rb.vis_in = vis; J.rb.vis_lc = J.ra.lc;
  J.ra.lights = J.lights; J.rb.lights = J.lights;
  J.ra.cam = cam; J.rb.cam = cam;
  J.rb.gmax = J.gmax;   // the interior adjoint's seeds dE/dp / spp under the job's scale
  const fr::MeshDev& md_ = jh->mesh->d;
  J.ea.edges = md_.edges; J.ea.cdf = md_.edge_cdf; J.ea.E = md_.E;
  J.ea.n_samples = d->edge_samples < 0 ? d->width * d->height : d->edge_samples;
  fr::edge_groups(L, J.ea.n_samples, J.ea);
  J.ea.th = std::tan(0.5 * (double)d->fov_y);
  J.ea.aspect = (double)d->width / (double)d->height;
  J.ea.dEdp = J.dEdp; J.ea.gverts = md_.acc; J.ea.gcam = nullptr; J.ea.dbg_rec = nullptr; J.ea.dbg_flag = nullptr;
  J.ea.gmax = J.gmax;
  // shadow-edge term: vertex gradients only (the batch optimises no light geometry or camera)
  J.se = fr::ShadowEdgeArgs{};
  J.se.nbr = md_.face_nbr;
  J.se.n_samples = d->shadow_edge_samples < 0 ? d->width * d->height : d->shadow_edge_samples;
  J.se.dEdp = J.dEdp; J.se.gverts = md_.acc; J.se.gmax = J.gmax;
  J.mean_geo = md->mean_geo; J.basis_geo = md->basis_geo; J.mean_alb = md->mean_alb; J.basis_alb = md->basis_alb;
  J.K_geo = md->K_geo; J.K_alb = md->K_alb; J.N = N; J.F = md->topo.F; J.M = M;
  J.hist_cap = jh->hist_cap;
  J.gnorm = md_.gnorm;
  J.acc = md_.acc;
  J.zero_stride = fr::cdiv(std::max(n_param, 3 * N), 256) * 256;
  J.n_param = n_param; J.off_alb = md->K_geo; J.off_pose = md->K_geo + md->K_alb; J.off_rad = n_param - 3 * L;
  J.tris = md_.tris; J.vf_off = md_.vf_off; J.vf_idx = md_.vf_idx; J.normals = md_.normals; J.nlen = md_.nlen;
  J.top_nodes = md_.top_nodes; J.top_level_off = md_.top_level_off; J.n_top_levels = md_.n_top_levels;
  J.nodes = md_.nodes; J.nodes4 = md_.nodes4; J.n4_src = md_.n4_src; J.n4 = md_.n4; J.recs = md_.recs; J.order = md_.order; J.node_parent = md_.node_parent;
  J.leaf_parent = md_.leaf_parent; J.flags = md_.flags;
  J.edge_faces = md_.edge_faces; J.face_front = md_.face_front; J.edge_len = md_.edge_len; J.edge_cdf = md_.edge_cdf;
  J.scan_part = md_.scan_part;
  J.smooth = d->smooth ? 1 : 0;
  const double e = 0.60653065971263342, z = (1.0 + 2.0 * e) * (1.0 + 2.0 * e);
  J.taps = fr::Taps{(float)(1.0 / z), (float)(e / z), (float)(e * e / z)};
  J.t = 0;
  J.ra.step = J.rb.step = 1;
  const int32_t id = b->next_id++;
  b->jobs[id] = jh;
  b->b.jobs.push_back(J);
  b->dirty = true;
  *job_id = id;
  return hipStreamSynchronize(st) == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}

int fr_batch_remove(fr_batch* b, int32_t job_id) {
  if (!b) return FR_ERR_INVALID_ARG;
  auto it = b->jobs.find(job_id);
  if (it == b->jobs.end()) return FR_ERR_NOT_FOUND;
  JobHost* jh = it->second;
  // table entries are kept in job-id order, so the position is the rank of the id
  int pos = 0;
  for (auto& kv : b->jobs) { if (kv.first == job_id) break; ++pos; }
  if (hipDeviceSynchronize() != hipSuccess) return FR_ERR_DEVICE;
  b->b.jobs.erase(b->b.jobs.begin() + pos);
  b->jobs.erase(it);
  fr_mesh_destroy(jh->mesh);
  if (jh->arena) (void)hipFree(jh->arena);
  delete jh;
  b->dirty = true;
  return FR_OK;
}

int32_t fr_batch_size(const fr_batch* b) { return b ? (int32_t)b->jobs.size() : -1; }

int fr_batch_step(fr_batch* b, int32_t n_steps, int32_t use_graph, fr_stream stream) {
  if (!b || n_steps < 0) return FR_ERR_INVALID_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (b->dirty) {
    const int rc = b->b.upload(st);
    if (rc != FR_OK) return fail(b->model->ctx, rc, "batch table upload failed");
    b->dirty = false;
  }
  const int rc = b->b.step(st, n_steps, use_graph != 0);
  if (rc != FR_OK) return fail(b->model->ctx, rc, "batch step failed");
  for (auto& J : b->b.jobs) {   // host mirror of the device step counters
    J.t += n_steps;
    J.ra.step = (uint32_t)(J.t + 1);
    J.rb.step = (uint32_t)(J.t + 1);
  }
  return FR_OK;
}

int fr_batch_job_info(const fr_batch* b, int32_t job_id, int32_t* n_param, int32_t* hist_cap, int32_t* steps_done) {
  if (!b) return FR_ERR_INVALID_ARG;
  auto it = b->jobs.find(job_id);
  if (it == b->jobs.end()) return FR_ERR_NOT_FOUND;
  int pos = 0;
  for (auto& kv : b->jobs) { if (kv.first == job_id) break; ++pos; }
  if (n_param) *n_param = it->second->n_param;
  if (hist_cap) *hist_cap = it->second->hist_cap;
  if (steps_done) *steps_done = b->b.jobs[pos].t;
  return FR_OK;
}

int32_t fr_batch_losses(fr_batch* b, int32_t cap, int32_t* h_ids, float* h_losses, fr_stream stream) {
  if (!b || (cap > 0 && (!h_ids || !h_losses))) return -FR_ERR_INVALID_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int32_t n = 0;
  size_t pos = 0;
  for (auto& kv : b->jobs) {
    if (n >= cap) break;
    h_ids[n] = kv.first;
    if (hipMemcpyAsync(h_losses + n, b->b.jobs[pos].loss, 4, hipMemcpyDeviceToHost, st) != hipSuccess)
      return -FR_ERR_DEVICE;
    ++n;
    ++pos;
  }
  if (hipStreamSynchronize(st) != hipSuccess) return -FR_ERR_DEVICE;
  return n;
}

int fr_batch_read(fr_batch* b, int32_t job_id, float* h_params, float* h_grad, float* h_loss_hist, float* h_image,
                  int32_t* h_t, fr_stream stream) {
  if (!b) return FR_ERR_INVALID_ARG;
  auto it = b->jobs.find(job_id);
  if (it == b->jobs.end()) return FR_ERR_NOT_FOUND;
  JobHost* jh = it->second;
  int pos = 0;
  for (auto& kv : b->jobs) { if (kv.first == job_id) break; ++pos; }
  const fr::JobDev& J = b->b.jobs[pos];
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  bool ok = true;
  if (h_params) ok = ok && hipMemcpyAsync(h_params, J.param, 4 * jh->n_param, hipMemcpyDeviceToHost, st) == hipSuccess;
  if (h_grad) ok = ok && hipMemcpyAsync(h_grad, J.grad, 4 * jh->n_param, hipMemcpyDeviceToHost, st) == hipSuccess;
  if (h_loss_hist)
    ok = ok && hipMemcpyAsync(h_loss_hist, J.loss_hist, 4 * jh->hist_cap, hipMemcpyDeviceToHost, st) == hipSuccess;
  if (h_image)
    ok = ok && hipMemcpyAsync(h_image, J.image, 12 * (size_t)jh->W * jh->H, hipMemcpyDeviceToHost, st) == hipSuccess;
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (h_t) *h_t = J.t;
  return ok ? FR_OK : FR_ERR_DEVICE;
}

}  // extern "C"
