// Host-side view of the device state and the launchers of each kernel file.
#pragma once

#include <vector>

#include "../../include/fr.h"
#include "fr_device.h"

namespace fr {

__host__ __device__ inline int cdiv(int a, int b) { return (a + b - 1) / b; }
__device__ inline int cdiv_d(int a, int b) { return (a + b - 1) / b; }

struct Taps { float c, e, k; };   // smoothing weights: centre, edge, corner

// Adam's bias correction 1 - b^t, computed identically on host and device
// (square-and-multiply in double, one rounding to float at the end).
__host__ __device__ inline float adam_bias(float b, int t) {
  double r = 1.0, x = (double)b;
  for (unsigned e = (unsigned)t; e; e >>= 1) {
    if (e & 1u) r *= x;
    x *= x;
  }
  return (float)(1.0 - r);
}

// Fixed-point gradient accumulation.  Every contribution is rounded once to a
// multiple of 2^-32 and summed in 64-bit two's-complement integers, so a sum
// does not depend on the order in which waves and blocks add to it: gradients
// are identical from run to run and whatever else shares the launch.
// Range: |sum| < 2^31; resolution 2^-32.
typedef unsigned long long fix_t;
constexpr double kFixOne = 4294967296.0;   // 2^32
// A contribution beyond the range saturates at +-2^62 (the conversion is then
// defined; a gradient that large is far outside any render's range).
__device__ __forceinline__ fix_t to_fix(float v) {
  return (fix_t)__float2ll_rn(fminf(fmaxf(v * 4294967296.0f, -4.611686e18f), 4.611686e18f));
}
__device__ __forceinline__ fix_t to_fix_d(double v) {
  return (fix_t)__double2ll_rn(fmin(fmax(v * kFixOne, -4.611686018427388e18), 4.611686018427388e18));
}
__device__ __forceinline__ void fix_add(fix_t* p, float v) {
  if (v != 0.0f) atomicAdd(p, to_fix(v));
}
__device__ __forceinline__ void fix_add_d(fix_t* p, double v) {
  if (v != 0.0) atomicAdd(p, to_fix_d(v));
}
__host__ __device__ __forceinline__ double from_fix(fix_t a) { return (double)(long long)a * (1.0 / kFixOne); }

// The quantum 2^-32 is absolute, so a backward scales its per-sample seeds
// dE/dp / S by a power of two s chosen from their maximum (the bits of
// max |dE/dp| / S, gathered by k_abs_max): s = 2^-floor(log2(max / S)),
// clamped to [2^-60, 2^60], which brings the largest seed into [1, 2) at any
// sample count and any scale of the caller's dE/dp; the conversions to FP32
// divide by s.  Scaling by a power of two is exact.  The sums then hold s
// times the gradient, well inside the range for the renders this library
// takes.  gmax null: s = 1.
__device__ __forceinline__ float grad_scale(const uint32_t* gmax) {
  if (!gmax) return 1.0f;
  const uint32_t b = *gmax;
  if (b == 0u) return 1.0f;
  const int e = (int)((b >> 23) & 0xffu) - 127;   // floor(log2 max); -127 for subnormals
  return ldexpf(1.0f, max(-60, min(-e, 60)));
}

// Fixed-point accumulators of the per-vertex gradients (each nullable).
struct FixGrads {
  fix_t* verts;       // [N*3]
  fix_t* normals;     // [N*3] dE/dn before the normalisation adjoint
  fix_t* diffuse;     // [N*3]
  fix_t* specular;    // [N*3]
  fix_t* roughness;   // [N]
  fix_t* tex_c;       // [M*M*3] reflectance-map texels (maps in use)
  fix_t* tex_s;       // [M*M*3]
  fix_t* tex_r;       // [M*M]
};

// Arguments of the shadow-edge (secondary visibility) kernel.
struct ShadowEdgeArgs {
  const int32_t* nbr;   // [F*3] face across edge k (tris[3f+k], tris[3f+(k+1)%3]) of face f, -1 if none
  int n_samples;
  const float* dEdp;    // [H*W*3]
  const uint32_t* gmax; // bits of max |dE/dp| (grad_scale; nullable)
  fix_t* gverts;        // [N*3] fixed-point (nullable)
  fix_t* glight;        // [L*9] fixed-point p0, e1, e2 (nullable)
  fix_t* gcam;          // [12] fixed-point (nullable)
  int32_t* dbg_rec;     // [n*4]: camera sample, light, jumps, edge-key sum (nullable)
  uint8_t* dbg_flag;    // [n]
};

// Arguments of the edge-sampling kernel.
struct EdgeArgs {
  const int32_t* edges;
  const double* cdf;
  int E, n_samples;
  double th, aspect;
  const float* dEdp;
  const uint32_t* gmax; // bits of max |dE/dp| (grad_scale; nullable)
  fix_t* gverts;        // [N*3] fixed-point
  fix_t* gcam;          // [12] fixed-point
  int32_t* dbg_rec;     // [n*4]: edge, pixel, hit-, hit+
  uint8_t* dbg_flag;    // [n]
  // The lights are cut into n_groups groups of gsize (the last may be
  // shorter); block b takes sample block b % bx of group b / bx, its four
  // waves the group's four light chunks.
  int gsize, n_groups, bx;
};

// Light groups of the boundary term for L lights and n edge samples: at most
// 128 lights a group, and enough groups that the launch holds at least 2048
// blocks (a whole chip of waves) while every wave keeps a light.
void edge_groups(int L, int n_samples, EdgeArgs& e);

// Primary hit of one camera sample: the closest-hit triangle (-1: miss), its
// distance, and the FP64 barycentrics b1, b2 of the crossing (b0 = 1 - b1 -
// b2).  Written once per render call by the primary pass and read by every
// light-chunk work item of the same sample.
struct PrimHit {
  int32_t id;
  float t;
  double b1, b2;
};
static_assert(sizeof(PrimHit) == 24, "primary hit is 24 bytes");

// Device buffers owned by one mesh (topology fixed at creation).
struct MeshDev {
  int N = 0, F = 0, E = 0;
  int32_t* tris = nullptr;          // [F*3]
  // vertex -> incident faces (CSR), for normals and their adjoint
  int32_t* vf_off = nullptr;        // [N+1]
  int32_t* vf_idx = nullptr;        // [3F]
  float* normals = nullptr;         // [N*3]
  float* nlen = nullptr;            // [N] length of the unnormalised normal sum
  // Per-call buffers of the adjoint.  A render call takes them from the
  // caller's workspace; only a batch job's mesh holds its own.
  float* gnorm = nullptr;           // [N*3] projected dE/dn
  // fixed-point backward accumulators [13N + 12]: verts, normals, diffuse,
  // specular (3N each), roughness (N), camera (12)
  fix_t* acc = nullptr;
  // unique edges and their faces, for the boundary term
  int32_t* edges = nullptr;         // [E*2]
  int32_t* edge_faces = nullptr;    // [E*2]
  int32_t* face_nbr = nullptr;      // [F*3] face across each edge of a face (-1: open edge)
  // BVH: binary tree (build + refit) and its 4-wide collapse (traversal)
  BvhNode* nodes = nullptr;         // [max(F-1,1)]
  Bvh4Node* nodes4 = nullptr;       // [n4]
  int32_t* n4_src = nullptr;        // [n4*4]: binary parent * 2 + side holding each child box, -1 unused
  int n4 = 0, n4_cap = 0, depth4 = 0;
  // refit: nodes spanning several leaf tiles, by level (children first)
  int32_t* top_nodes = nullptr;     // [n_top]
  int32_t* top_level_off = nullptr; // [n_top_levels + 1]
  int n_top = 0, n_top_levels = 0, top_cap = 0;
  TriRec* recs = nullptr;           // [F]
  int32_t* order = nullptr;         // [F] sorted slot -> triangle id
  int32_t* node_parent = nullptr;   // [max(F-1,1)]
  int32_t* leaf_parent = nullptr;   // [F]
  uint32_t* flags = nullptr;        // [max(F-1,1)]
  uint32_t* keys[2] = {nullptr, nullptr};
  int32_t* vals[2] = {nullptr, nullptr};
  uint32_t* hist = nullptr;         // [256 * ceil(F/1024)]
  float* partial = nullptr;         // [64*6]
  float* scene_box = nullptr;       // [6]
  int32_t* depth = nullptr;         // [2]: depth, validation error count
  // per-call buffers of the boundary term (as gnorm and acc above)
  double* edge_len = nullptr;       // [E] film length of silhouette edges (0 otherwise)
  double* edge_cdf = nullptr;       // [E] inclusive running sum
  uint8_t* face_front = nullptr;    // [F]
  double* scan_part = nullptr;      // [ceil(E/1024)] tile totals of the edge CDF scan
  int bvh_depth = -1;
  int built = 0;
};

// Per-render constants shared by the forward, backward and edge kernels.
constexpr int kMaxShBands = 11;   // spherical-harmonics lighting: bands 0..10

struct RenderArgs {
  const Bvh4Node* nodes;
  const TriRec* recs;
  const int32_t* tris;
  const float* verts;
  const float* normals;
  const float* diffuse;
  const float* specular;
  const float* roughness;
  const LightRec* lights;
  const float* cam;       // [12]
  const float* uv;        // [F*6] per-corner texture coordinates (M > 0)
  const float* tex_c;     // [M*M*3] reflectance maps (M > 0)
  const float* tex_s;     // [M*M*3]
  const float* tex_r;     // [M*M]
  int M;                  // map size; 0: per-vertex reflectance
  int N, F, L;
  int W, H, S;
  int tile_w, tile_h, tiles_x, tiles_y, n_tiles;   // wave tiles (S <= 64)
  int chunks;             // S / 64 when S > 64, else 1
  int lanes_per_pixel;    // min(S, 64)
  int lc, n_lchunks;      // lights per work item, light chunks per tile
  int shadow_traversal;   // forward: 0 wave packet, 1 per-lane walk
  const uint32_t* gmax;   // adjoint: bits of max |dE/dp| (grad_scale; nullable)
  int light0;             // global index of lights[0] (> 0 in the adjoint's later light groups)
  // spherical-harmonics lighting: coefficients [B*B*3] (B = sh_bands, 0 =
  // none), A_l, and the basis normalisation per (l, m >= 0) at
  // l(l+1)/2 + m (sqrt 2 folded in for m > 0)
  const float* sh;
  int sh_bands;
  float sh_ash[kMaxShBands];
  float sh_norm[kMaxShBands * (kMaxShBands + 1) / 2];
  float* partial;         // [n_lchunks][H*W*3] per-chunk pixel sums (n_lchunks > 1)
  PrimHit* prim;          // [H*W*S] primary hits, sample index (y*W + x)*S + s
  // Shadow masks, word (c, sample) at c*W*H*S + sample: bit b is light
  // c*vis_lc + b.  The forward writes them (vis_out, with vis_lc = lc) when
  // asked; the adjoint then reads them (vis_in) in place of its shadow rays.
  uint32_t* vis_out;
  const uint32_t* vis_in;
  int vis_lc;
  float tan_half, aspect;
  double tan_half_d, aspect_d;   // the same in FP64 (texture coordinates)
  uint32_t k0, k1, step;
  int variant, components;
  int32_t* dbg_hit;
  uint8_t* dbg_pflag;
  uint8_t* dbg_vis;
  uint64_t* dbg_stats;
};

// shadow_edges.hip
void launch_shadow_edges(const RenderArgs& a, const ShadowEdgeArgs& e, hipStream_t st);
// bvh.hip
int bvh_build(MeshDev& m, const float* d_verts, hipStream_t st, bool sah, int* depth_out);
void bvh_refit(MeshDev& m, const float* d_verts, hipStream_t st);
// model.hip
// Blocks of 256 threads for the vertex-normal kernels over N vertices.
int normals_blocks(int N);
void launch_normals(MeshDev& m, const float* d_verts, hipStream_t st);
void launch_normals_backward(MeshDev& m, const float* d_verts, const fix_t* acc_n, float* gn_tmp, fix_t* acc_v,
                             hipStream_t st);
// out += acc / grad_scale(gmax)
void launch_fix_to_float(const fix_t* acc, float* out, int n, hipStream_t st, const uint32_t* gmax = nullptr);
// *gmax = max(*gmax, bits of max |x[i]|) (the caller zeroes *gmax)
void launch_abs_max(const float* x, int n, int spp, uint32_t* gmax, hipStream_t st);
void launch_zero_fix(fix_t* p, size_t n, hipStream_t st);
void launch_blend(const float* mean, const float* basis, const float* coef, int K, int M, float* out, hipStream_t st);
void launch_blend_backward(const float* basis, const float* gout, int K, int M, float* gcoef, hipStream_t st);
void launch_pose(const float* v, int N, const float* pose, float* vw, hipStream_t st);
void launch_pose_backward(const float* v, int N, const float* pose, const float* gw, float* gv, float* gpose,
                          hipStream_t st);
void launch_adam(float* p, const float* g, float* m, float* v, const float* lr, int n, int t, float b1, float b2,
                 float eps, hipStream_t st);
void launch_light_setup(const fr_scene& sc, LightRec* out, hipStream_t st);
void launch_light_stage(const float* faces, const float* P, int J, float* p0, float* e1, float* e2, float* rad,
                        int32_t* shape, hipStream_t st);
void launch_light_stage_backward(const float* faces, const float* P, int J, const float* gg, const float* gr,
                                 float* gP, hipStream_t st);
void launch_bake_map(const int32_t* tris, const float* uv, int F, const float* attr, int C, int M, float* map,
                     hipStream_t st);
void launch_zero(float* p, int n, hipStream_t st);
void launch_axpy(float* dst, const float* src, float a, const float* s, int n, hipStream_t st);   // dst += a s[0] src
// render.hip
// The render kernels of single calls read their arguments from device memory
// (`d_args`, kRenderArgSlots copies from the call's workspace), written by
// launch_put_args on the same stream: read through a pointer, the arguments
// leave the kernels' scalar registers free (passed by value they were held
// in them, and spilled).
constexpr int kRenderArgSlots = 2;   // the call's arguments, and an adjoint light group's
void launch_put_args(const RenderArgs& a, RenderArgs* d_slot, hipStream_t st);
// The primary pass (camera-ray hits into a.prim) with the arguments already
// in d_slot; the render launchers run it first.
void launch_primary(const RenderArgs& a, const RenderArgs* d_slot, hipStream_t st);
void launch_render_forward(const RenderArgs& a, RenderArgs* d_args, float* image, hipStream_t st,
                           hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Default lights per work item: short items balance the forward launch; the
// backward repeats more per-item work (primary trace, chain, scatter), so it
// takes longer items.
constexpr int kLightChunkFwd = 12;
constexpr int kBwdMaxLights = 128;   // four chunks of at most 32 lights: one adjoint launch's light group
constexpr size_t kBwdPartBytes = 4 * 64 * 16 * sizeof(float) + 16;   // backward LDS: sample adjoints of 4 waves, arrivals
// The boundary term has one wave per 64 edge samples and light chunk: short
// chunks give the launch enough waves to fill the chip.
// Partial slots of the backward light/camera gradients (reduced in a fixed order).
constexpr int kSlots = 1024;
// loss.hip
struct MapRegWeights { float w_sym, w_chroma, w_smooth, w_box; };
void launch_landmarks(const float* V, const int32_t* idx, int n, const float* cam, float tan_half, int W, int H,
                      const float* z, float* loss, float* gV, float* gcam, hipStream_t st);
void launch_prior(const float* x, const float* sigma, int n, int kind, float w, float* loss, float* g, hipStream_t st);
void launch_map_regularizers(const float* Cm, const float* Sm, const float* Rm, const float* C0, const float* S0, int M,
                             const MapRegWeights& w, float* loss, float* gC, float* gS, float* gR, double* scratch,
                             hipStream_t st);
// scratch: ceil(W H / 256) FP64 block sums; gtmp: the [H*W*3] sign image (smoothing only)
void launch_loss(const float* img, const float* target, int W, int H, int smooth, float* loss, float* dEdp,
                 double* scratch, float* gtmp, hipStream_t st);
// Device bytes of fr_loss's scratch for a W x H image, and of the map
// regularisers' for M x M maps (both 256-byte aligned pieces).
size_t loss_scratch_bytes(int W, int H, int smooth);
// noalloc.hip: device address of fr_loss_noalloc's static scratch on device
// dev (the current device), resolved once per device; nullptr on failure.
void* noalloc_scratch(int dev);
size_t map_reg_scratch_bytes(int M);
// backward.hip
// Interior adjoint: per-vertex gradients into `fg`, light and camera
// gradients into the slots and then added to g.light_geom, g.light_rad, g.cam.
// With trace_primary false, a.prim already holds this call's camera-ray hits.
void launch_render_backward(const RenderArgs& a, RenderArgs* d_args, const float* dEdp, const FixGrads& fg,
                            fix_t* slots, const fr_grads& g, hipStream_t st, hipEvent_t e0 = nullptr,
                            hipEvent_t e1 = nullptr, bool trace_primary = true);
// edges.hip
void launch_edges(MeshDev& m, const RenderArgs& a, const float* dEdp, int n_samples, fix_t* gverts, fix_t* gcam,
                  int32_t* dbg_rec, uint8_t* dbg_flag, double tan_half, hipStream_t st);

}  // namespace fr
