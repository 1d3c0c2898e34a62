// Sampling, shading frame and Cook-Torrance BRDF shared by the forward,
// backward and edge kernels, so that all of them take the same decisions from
// the same arithmetic.
//
// Counters of the Philox generator: (pixel id y*W + x, sample s, purpose,
// step) with key = 64-bit seed.  Purpose 0: film jitter; 1 + j: point on
// light j.  Each 32-bit output maps to [0,1) through its top 24 bits.
#pragma once

#include "fr_kernels.h"

namespace fr {

// ---------------------------------------------------------------------------
// Wave -> tile mapping
// ---------------------------------------------------------------------------
// Work items are (tile, light chunk): a tile of 64/S pixels x S samples
// shaded with lights [chunk * lc, chunk * lc + lc).  Splitting the light loop
// keeps every wave short (a face tile with all lights costs ~100x a background
// tile), which removes the long tail of the launch.
//
// Blocks are dispatched round-robin over the 8 XCDs (block b on XCD b % 8).
// The image is cut into strips of 4 tile rows; XCD x walks strips x, x+8,
// x+16, ... in order, a block covering 4 consecutive items (the chunks of one
// tile share its primary rays in cache).  Each XCD's L2 then holds the BVH
// around its current strip while every XCD gets work from the whole image.
struct Item { int tile, chunk; };

// nl = light chunks per tile (1 for the primary pass, which has one item per tile).
__device__ __forceinline__ Item wave_item(const RenderArgs& a, int b, int nl) {
  const int per_strip = a.tiles_x * nl;                 // blocks per strip
  const int x = b & 7, k = b >> 3;
  const int si = k / per_strip, bi = k - si * per_strip;
  const int strip = si * 8 + x;
  const int item = strip * 4 * per_strip + bi * 4 + (threadIdx.x >> 6);
  Item it;
  it.tile = item / nl;
  it.chunk = item - it.tile * nl;
  if (it.tile / a.tiles_x >= a.tiles_y) it.tile = -1;
  return it;
}
__device__ __forceinline__ Item wave_item(const RenderArgs& a, int b) { return wave_item(a, b, a.n_lchunks); }

inline int wave_blocks_items(const RenderArgs& a, int nl) {
  const int strips = (a.tiles_y + 3) / 4;
  return 8 * a.tiles_x * nl * ((strips + 7) / 8);
}
inline int wave_blocks_items(const RenderArgs& a) { return wave_blocks_items(a, a.n_lchunks); }

// One tile per block (the backward, whose four waves are the tile's light
// chunks): the same XCD-aware strip order as wave_item.
__device__ __forceinline__ int block_tile(const RenderArgs& a, int b) {
  const int per_strip = a.tiles_x * 4;                 // tiles per strip of 4 tile rows
  const int x = b & 7, k = b >> 3;
  const int si = k / per_strip, bi = k - si * per_strip;
  const int tile = (si * 8 + x) * per_strip + bi;
  return tile / a.tiles_x < a.tiles_y ? tile : -1;
}
inline int tile_blocks(const RenderArgs& a) {
  const int strips = (a.tiles_y + 3) / 4;
  return 8 * a.tiles_x * 4 * ((strips + 7) / 8);
}

struct PixelSample {
  int px, py, pid, s0;
  bool valid;
};

__device__ __forceinline__ PixelSample pixel_sample(const RenderArgs& a, int tile, int lane) {
  PixelSample p;
  const int lpp = a.lanes_per_pixel;
  const int pix = lane / lpp;
  p.s0 = lane - pix * lpp;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  p.px = tx * a.tile_w + pix % a.tile_w;
  p.py = ty * a.tile_h + pix / a.tile_w;
  p.valid = p.px < a.W && p.py < a.H;
  p.pid = p.valid ? p.py * a.W + p.px : 0;
  return p;
}

// Sum over aligned groups of n lanes (n a power of 2, wave-uniform), every
// lane of a group receiving its group's sum, in a fixed order: DPP within a
// row of 16 lanes (quad swaps, half-row and row mirrors), LDS permutes
// beyond.  All 64 lanes must be active.
__device__ __forceinline__ float group_sum(float x, int n) {
  if (n >= 2) x = dpp_add<0xb1, 0xf>(x);    // quad_perm [1,0,3,2]
  if (n >= 4) x = dpp_add<0x4e, 0xf>(x);    // quad_perm [2,3,0,1]
  if (n >= 8) x = dpp_add<0x141, 0xf>(x);   // row_half_mirror
  if (n >= 16) x = dpp_add<0x140, 0xf>(x);  // row_mirror
  for (int off = 16; off < n; off <<= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// ---------------------------------------------------------------------------
// Camera sample
// ---------------------------------------------------------------------------
struct Sample {
  Ray ray;
  V3 dc;          // camera-space direction (unnormalised)
  V3 dw;          // R dc (unnormalised)
  float inv_len;  // 1 / |R dc|
};

__device__ __forceinline__ void camera_ray_film(const RenderArgs& a, float fx, float fy, Sample& sm) {
  const float sx = (2.0f * fx / (float)a.W - 1.0f) * a.tan_half * a.aspect;
  const float sy = (1.0f - 2.0f * fy / (float)a.H) * a.tan_half;
  const float* R = a.cam;
  sm.dc = {sx, sy, -1.0f};
  sm.dw = {R[0] * sx + R[1] * sy - R[2], R[3] * sx + R[4] * sy - R[5], R[6] * sx + R[7] * sy - R[8]};
  sm.inv_len = 1.0f / sqrtf(dot(sm.dw, sm.dw));
  sm.ray.o = {R[9], R[10], R[11]};
  sm.ray.d = sm.dw * sm.inv_len;
  sm.ray.tmin = 0.0f;
  sm.ray.tmax = 3.4e38f;
  ray_setup(sm.ray);
}

__device__ __forceinline__ void camera_sample(const RenderArgs& a, const PixelSample& ps, int s, Sample& sm) {
  const U4 r = philox((uint32_t)ps.pid, (uint32_t)s, PURPOSE_JITTER, a.step, a.k0, a.k1);
  camera_ray_film(a, (float)ps.px + unit24(r.x), (float)ps.py + unit24(r.y), sm);
}

// Exact film point of a camera sample (pixel + jitter, an FP64 sum), for the
// FP64 barycentrics of the shading point.  The jitter is drawn again here,
// after the traversal: the empty asm keeps the compiler from reusing the
// first draw, whose two values would otherwise stay live through it.
__device__ __forceinline__ void film_point(const RenderArgs& a, const PixelSample& ps, int s, double& fx, double& fy) {
  uint32_t pid = (uint32_t)ps.pid;
  asm volatile("" : "+v"(pid));
  const U4 r = philox(pid, (uint32_t)s, PURPOSE_JITTER, a.step, a.k0, a.k1);
  fx = (double)ps.px + (double)unit24(r.x);
  fy = (double)ps.py + (double)unit24(r.y);
}

// ---------------------------------------------------------------------------
// Shading frame at the hit
// ---------------------------------------------------------------------------
struct Frame {
  V3 x, ns, wo, c, s;
  V3 m;            // unnormalised interpolated normal
  float inv_m;     // 1 / |m|
  float r;         // clamped roughness
  bool r_free;     // roughness inside the clamp range (gradient passes)
  float cos_o;
  int vi[3];
  float b[3];
  float t;         // hit distance (the crossing point o + t d, in the adjoint)
};

// Barycentrics of the shading point, in FP64: the crossing of the exact
// camera ray through film point (fx, fy) (FP64 direction from the FP32
// camera) with the plane of triangle vi (FP32 vertices, exact in FP64),
// Moller-Trumbore with the ray origin at the camera centre (the scale of the
// direction cancels).  The FP32 ray of the traversal places the hit only to
// ~ulp(|o|) in world units, i.e. ~1e-5 of a face-scale triangle: a weight b_k
// near 0 then carries a large relative error into the vertex and texel
// gradients.  The cost is one FP64 solve per camera sample.
__device__ __forceinline__ void bary64(const RenderArgs& a, double fx, double fy, const int vi[3], double b[3]) {
  const double sx = (2.0 * fx / (double)a.W - 1.0) * a.tan_half_d * a.aspect_d;
  const double sy = (1.0 - 2.0 * fy / (double)a.H) * a.tan_half_d;
  const float* R = a.cam;
  const double dx = (double)R[0] * sx + (double)R[1] * sy - (double)R[2];
  const double dy = (double)R[3] * sx + (double)R[4] * sy - (double)R[5];
  const double dz = (double)R[6] * sx + (double)R[7] * sy - (double)R[8];
  const float* p0 = a.verts + 3 * vi[0];
  const float* p1 = a.verts + 3 * vi[1];
  const float* p2 = a.verts + 3 * vi[2];
  const double e1x = (double)p1[0] - p0[0], e1y = (double)p1[1] - p0[1], e1z = (double)p1[2] - p0[2];
  const double e2x = (double)p2[0] - p0[0], e2y = (double)p2[1] - p0[1], e2z = (double)p2[2] - p0[2];
  const double svx = (double)R[9] - p0[0], svy = (double)R[10] - p0[1], svz = (double)R[11] - p0[2];
  const double pvx = dy * e2z - dz * e2y, pvy = dz * e2x - dx * e2z, pvz = dx * e2y - dy * e2x;
  const double qvx = svy * e1z - svz * e1y, qvy = svz * e1x - svx * e1z, qvz = svx * e1y - svy * e1x;
  const double idet = 1.0 / (e1x * pvx + e1y * pvy + e1z * pvz);
  b[1] = (svx * pvx + svy * pvy + svz * pvz) * idet;
  b[2] = (dx * qvx + dy * qvy + dz * qvz) * idet;
  b[0] = 1.0 - b[1] - b[2];
}

// Bilinear footprint on an M x M reflectance map (Sec. 3.2) at the shading
// point's texture coordinates (u, v) = sum_k b_k uv_k (FP64 barycentrics):
// texel (i, j) centred at ((i + 1/2)/M, (j + 1/2)/M), border-clamped
// addresses; the taps (i0,j0), (i1,j0), (i0,j1), (i1,j1) weigh (1-fx)(1-fy),
// fx(1-fy), (1-fx)fy, fx fy.  The cell corner is clamped in FP64 before the
// integer conversion so that any input, NaN included, addresses inside the
// map.
struct TexTap {
  int t00, t10, t01, t11;   // texel indices j M + i
  float fx, fy;
};

__device__ __forceinline__ TexTap tex_tap(const RenderArgs& a, int tri, const double b[3]) {
  const float* q = a.uv + 6 * tri;
  const double u = b[0] * q[0] + b[1] * q[2] + b[2] * q[4];
  const double v = b[0] * q[1] + b[1] * q[3] + b[2] * q[5];
  const double x = u * (double)a.M - 0.5, y = v * (double)a.M - 0.5;
  const double x0 = floor(x), y0 = floor(y);
  TexTap t;
  t.fx = (float)(x - x0);
  t.fy = (float)(y - y0);
  const int M = a.M;
  const int ix = (int)fmin(fmax(x0, -1.0), (double)M), iy = (int)fmin(fmax(y0, -1.0), (double)M);
  const int i0 = min(max(ix, 0), M - 1), i1 = min(max(ix + 1, 0), M - 1);
  const int j0 = min(max(iy, 0), M - 1), j1 = min(max(iy + 1, 0), M - 1);
  t.t00 = j0 * M + i0; t.t10 = j0 * M + i1; t.t01 = j1 * M + i0; t.t11 = j1 * M + i1;
  return t;
}

// TEX selects the reflectance maps at compile time (a.M > 0 on the host), so
// the per-vertex kernels keep their register budget.
// Frame at the crossing of the sample's ray with triangle `id` at distance t,
// with FP64 barycentrics bd (as bary64 gives them).
template <bool TEX>
__device__ __forceinline__ bool shading_frame(const RenderArgs& a, const Sample& sm, int id, float t_hit,
                                              const double bd[3], Frame& f) {
  const int* t = a.tris + 3 * id;
  f.vi[0] = t[0]; f.vi[1] = t[1]; f.vi[2] = t[2];
  const V3 v0 = ld3(a.verts, f.vi[0]), v1 = ld3(a.verts, f.vi[1]), v2 = ld3(a.verts, f.vi[2]);
  const float b0 = (float)bd[0], b1 = (float)bd[1], b2 = (float)bd[2];
  f.b[0] = b0; f.b[1] = b1; f.b[2] = b2;
  f.t = t_hit;
  f.x = v0 * b0 + v1 * b1 + v2 * b2;
  const V3 n0 = ld3(a.normals, f.vi[0]), n1 = ld3(a.normals, f.vi[1]), n2 = ld3(a.normals, f.vi[2]);
  f.m = n0 * b0 + n1 * b1 + n2 * b2;
  f.inv_m = 1.0f / sqrtf(dot(f.m, f.m));
  f.ns = f.m * f.inv_m;
  f.wo = {-sm.ray.d.x, -sm.ray.d.y, -sm.ray.d.z};
  float r;
  if (TEX) {
    const TexTap tp = tex_tap(a, id, bd);
    const float w00 = (1.0f - tp.fx) * (1.0f - tp.fy), w10 = tp.fx * (1.0f - tp.fy);
    const float w01 = (1.0f - tp.fx) * tp.fy, w11 = tp.fx * tp.fy;
    f.c = ld3(a.tex_c, tp.t00) * w00 + ld3(a.tex_c, tp.t10) * w10 + ld3(a.tex_c, tp.t01) * w01 +
          ld3(a.tex_c, tp.t11) * w11;
    f.s = ld3(a.tex_s, tp.t00) * w00 + ld3(a.tex_s, tp.t10) * w10 + ld3(a.tex_s, tp.t01) * w01 +
          ld3(a.tex_s, tp.t11) * w11;
    r = a.tex_r[tp.t00] * w00 + a.tex_r[tp.t10] * w10 + a.tex_r[tp.t01] * w01 + a.tex_r[tp.t11] * w11;
  } else {
    f.c = ld3(a.diffuse, f.vi[0]) * b0 + ld3(a.diffuse, f.vi[1]) * b1 + ld3(a.diffuse, f.vi[2]) * b2;
    f.s = ld3(a.specular, f.vi[0]) * b0 + ld3(a.specular, f.vi[1]) * b1 + ld3(a.specular, f.vi[2]) * b2;
    r = a.roughness[f.vi[0]] * b0 + a.roughness[f.vi[1]] * b1 + a.roughness[f.vi[2]] * b2;
  }
  f.r_free = r >= kRoughMin && r <= kRoughMax;
  f.r = fminf(fmaxf(r, kRoughMin), kRoughMax);
  f.cos_o = dot(f.ns, f.wo);
  return f.cos_o > 0.0f;
}

// Frame of a traced hit h of the ray through the exact film point (fx, fy).
template <bool TEX>
__device__ __forceinline__ bool shading_frame(const RenderArgs& a, const Sample& sm, const HitState& h, Frame& f,
                                              double fx, double fy) {
  const int* t = a.tris + 3 * h.id;
  const int vi[3] = {t[0], t[1], t[2]};
  double bd[3];
  bary64(a, fx, fy, vi, bd);
  return shading_frame<TEX>(a, sm, h.id, h.t, bd, f);
}

// The stored primary hit of sample rs (pixel-major) as (id, t, FP64 barycentrics).
__device__ __forceinline__ PrimHit load_prim(const RenderArgs& a, size_t rs, double bd[3]) {
  const PrimHit p = a.prim[rs];
  bd[1] = p.b1;
  bd[2] = p.b2;
  bd[0] = 1.0 - p.b1 - p.b2;
  return p;
}

// ---------------------------------------------------------------------------
// Light sample
// ---------------------------------------------------------------------------
struct LightSample {
  float w1, w2;
  V3 q, l;
  float dist, dist2, cos_s, cos_a, geom;
  bool amb;
};

// Uniform point on the light from two uniforms: parallelogram (u0, u1);
// triangle (sqrt(u0)(1 - u1), sqrt(u0) u1).
__device__ __forceinline__ void light_weights(int shape, float u0, float u1, float& w1, float& w2) {
  if (shape == FR_LIGHT_TRIANGLE) {
    const float su = sqrtf(u0);
    w1 = su * (1.0f - u1);
    w2 = su * u1;
  } else {
    w1 = u0;
    w2 = u1;
  }
}

// Returns true when light j contributes to this shading point before
// visibility: n_s . l > 0 and -n_j . l > 0 (the caller already required
// n_s . o > 0).  geom = (n_s . l) A_j (-n_j . l) / |q - x|^2.  A light at
// infinity: l is its direction, geom = n_s . l, and the shadow segment ends
// at kDirectionalFar (q is left at x: nothing depends on a point).
__device__ __forceinline__ bool light_point(const LightRec& Lj, float u0, float u1, const Frame& f, LightSample& ls) {
  if (Lj.shape == FR_LIGHT_DIRECTIONAL) {
    ls.w1 = 0.0f; ls.w2 = 0.0f;
    ls.l = {Lj.p0[0], Lj.p0[1], Lj.p0[2]};
    ls.q = f.x;
    ls.dist = kDirectionalFar;
    ls.dist2 = 1.0f;
    ls.cos_s = dot(f.ns, ls.l);
    ls.cos_a = 1.0f;
    ls.geom = ls.cos_s;
    ls.amb = fabsf(ls.cos_s) < kFlagCos;
    return ls.cos_s > 0.0f;
  }
  light_weights(Lj.shape, u0, u1, ls.w1, ls.w2);
  ls.q = {Lj.p0[0] + Lj.e1[0] * ls.w1 + Lj.e2[0] * ls.w2, Lj.p0[1] + Lj.e1[1] * ls.w1 + Lj.e2[1] * ls.w2,
          Lj.p0[2] + Lj.e1[2] * ls.w1 + Lj.e2[2] * ls.w2};
  const V3 dq = ls.q - f.x;
  ls.dist2 = dot(dq, dq);
  ls.dist = sqrtf(ls.dist2);
  ls.l = dq * (1.0f / ls.dist);
  ls.cos_s = dot(f.ns, ls.l);
  ls.cos_a = Lj.na[0] * ls.l.x + Lj.na[1] * ls.l.y + Lj.na[2] * ls.l.z;
  ls.geom = ls.cos_s * ls.cos_a / ls.dist2;
  const float alen = sqrtf(Lj.na[0] * Lj.na[0] + Lj.na[1] * Lj.na[1] + Lj.na[2] * Lj.na[2]);
  ls.amb = fabsf(ls.cos_s) < kFlagCos || fabsf(ls.cos_a) < kFlagCos * alen;
  return ls.cos_s > 0.0f && ls.cos_a > 0.0f;
}

// Conservative cull of a whole light for this shading point: false only when
// EVERY point q of the light fails one of light_point's two tests by a
// margin far above the rounding of those tests: n_s . (q - x) < 0 at all
// corners (the light lies below the tangent plane), or the point lies behind
// the light's emitting plane.  A wave whose lanes all return false skips the
// light (no random numbers, no shadow ray): the exact tests would have
// culled every lane anyway, without ambiguity.
__device__ __forceinline__ bool light_may_contribute(const LightRec& Lj, const Frame& f) {
  if (Lj.shape == FR_LIGHT_DIRECTIONAL)
    return !(f.ns.x * Lj.p0[0] + f.ns.y * Lj.p0[1] + f.ns.z * Lj.p0[2] < -1e-4f);
  const V3 d0 = {Lj.p0[0] - f.x.x, Lj.p0[1] - f.x.y, Lj.p0[2] - f.x.z};
  const float a = dot(f.ns, d0);
  const float b = f.ns.x * Lj.e1[0] + f.ns.y * Lj.e1[1] + f.ns.z * Lj.e1[2];
  const float c = f.ns.x * Lj.e2[0] + f.ns.y * Lj.e2[1] + f.ns.z * Lj.e2[2];
  float top = fmaxf(a, fmaxf(a + b, a + c));
  if (Lj.shape != FR_LIGHT_TRIANGLE) top = fmaxf(top, a + b + c);
  // na . (q - x) equals na . (p0 - x) for every q of the (planar) light
  const float side = Lj.na[0] * d0.x + Lj.na[1] * d0.y + Lj.na[2] * d0.z;
  const float alen = fabsf(Lj.na[0]) + fabsf(Lj.na[1]) + fabsf(Lj.na[2]);
  return !(top < -1e-4f) && !(side < -1e-3f * alen);
}

// Shadow decisions of one shading point for lights [j0, j1) (at most 32
// lights): bit j - j0 of the result is set when the point drawn on light j
// (uniforms from draw(j)) passes both cosine tests and no triangle but
// `self` blocks the segment to it.  The shading that follows draws the same
// point again from the same counters (bit-identical), so only these bits
// cross from the traversals to the shading: the two never hold their
// registers at the same time.  note(j, lit, occ, ls, sh) sees every light a
// wave traces (debug dumps); skip(j) every light the wave culls as a whole.
template <bool DUMP, bool LANE = false, class Draw, class Note, class Skip>
__device__ __forceinline__ uint32_t shadow_mask(const RenderArgs& a, int j0, int j1, bool shaded, const Frame& fr,
                                                int self, Draw draw, Note note, Skip skip, TravStats* st) {
  uint32_t mask = 0;
  for (int j = j0; j < j1; ++j) {
    const LightRec Lj = load_const(a.lights, j);
    if (!ballot(shaded && light_may_contribute(Lj, fr))) {   // culled for the whole wave
      skip(j);
      continue;
    }
    const U4 r = Lj.shape == FR_LIGHT_DIRECTIONAL ? U4{0u, 0u, 0u, 0u} : draw(j);
    LightSample ls;
    const bool lit = shaded && light_point(Lj, unit24(r.x), unit24(r.y), fr, ls);
    Ray sr;
    sr.o = fr.x; sr.d = ls.l; sr.tmin = kShadowTmin; sr.tmax = ls.dist;
    ray_setup<!DUMP>(sr);   // production: hardware 1/d (same answers; the dumps keep the division)
    HitState sh;
    sh.tamb = 3.4e38f;
    bool occ = false;
    if (LANE && !DUMP) occ = trace_lane_any(a.nodes, a.recs, a.F, sr, lit, self);
    else trace<true, DUMP>(a.nodes, a.recs, a.F, sr, lit, self, sh, occ, st);
    if (lit && !occ) mask |= 1u << (j - j0);
    if (DUMP) note(j, lit, occ, ls, sh);
  }
  return mask;
}

// ---------------------------------------------------------------------------
// Cook-Torrance BRDF (Appendix A), both readings of D and F.
// ---------------------------------------------------------------------------
// Walter et al.'s rational G1 with a = n.v / (r sqrt(1 - (n.v)^2)).
template <bool DUMP>
__device__ __forceinline__ float smith_g1(float nv, float hv, float r, float& flag) {
  if (!(hv * nv > 0.0f)) return 0.0f;   // h.v / n.v > 0: the same sign
  const float s2 = 1.0f - nv * nv;
  if (s2 <= 0.0f) return 1.0f;
  const float a = nv * rsqrt_hw(s2) * rcp_hw(r);
  if (DUMP && fabsf(a - 1.6f) < kFlagG1 * 1.6f) flag = 1.0f;
  if (a < 1.6f) return (3.535f * a + 2.181f * a * a) * rcp_hw(1.0f + 2.276f * a + 2.577f * a * a);
  return 1.0f;
}

template <bool DUMP>
__device__ __forceinline__ void brdf_eval(int variant, int components, const Frame& f, const LightSample& ls, float out[3],
                                          float& flag) {
  out[0] = out[1] = out[2] = 0.0f;
  if (components & 1) {
    out[0] = f.c.x * (1.0f / kPi);
    out[1] = f.c.y * (1.0f / kPi);
    out[2] = f.c.z * (1.0f / kPi);
  }
  if (components & 2) {
    V3 hv = ls.l + f.wo;
    hv = hv * rsqrt_hw(dot(hv, hv));
    const float nh = dot(f.ns, hv);   // > 0: n.l > 0 and n.o > 0 here
    const float ir = rcp_hw(f.r);
    const float ex = 2.0f * ir - 2.0f;
    const float nd = variant == FR_BRDF_NORMALIZED ? ir * (1.0f / kPi) : (2.0f * ir + 2.0f) * (1.0f / (2.0f * kPi));
    const float D = nd * exp2_hw(ex * log2_hw(nh));
    const float oh = dot(f.wo, hv), lh = dot(ls.l, hv);
    const float G = smith_g1<DUMP>(f.cos_o, oh, f.r, flag) * smith_g1<DUMP>(ls.cos_s, lh, f.r, flag);
    const float om = 1.0f - oh;
    const float fw = variant == FR_BRDF_NORMALIZED ? om * om * om * om * om : om;
    const float spec = D * G * rcp_hw(4.0f * f.cos_o * ls.cos_s);
    out[0] += (f.s.x + (1.0f - f.s.x) * fw) * spec;
    out[1] += (f.s.y + (1.0f - f.s.y) * fw) * spec;
    out[2] += (f.s.z + (1.0f - f.s.z) * fw) * spec;
  }
}

// ---------------------------------------------------------------------------
// Spherical-harmonics lighting (Sec. 6, "Spherical Harmonics (SH) vs. Light
// Stage"): a distant light as real SH coefficients L_lm, no visibility, on
// the diffuse term: (c / pi) E(n_s), E(n) = sum_l A_l sum_m L_lm Y_lm(n).
// ---------------------------------------------------------------------------
// A value with its gradient in (x, y, z).
struct G4 { float v, dx, dy, dz; };
__device__ __forceinline__ G4 operator+(G4 a, G4 b) { return {a.v + b.v, a.dx + b.dx, a.dy + b.dy, a.dz + b.dz}; }
__device__ __forceinline__ G4 operator-(G4 a, G4 b) { return {a.v - b.v, a.dx - b.dx, a.dy - b.dy, a.dz - b.dz}; }
__device__ __forceinline__ G4 operator*(G4 a, float s) { return {a.v * s, a.dx * s, a.dy * s, a.dz * s}; }
__device__ __forceinline__ G4 operator*(G4 a, G4 b) {
  return {a.v * b.v, a.dx * b.v + a.v * b.dx, a.dy * b.v + a.v * b.dy, a.dz * b.v + a.v * b.dz};
}

// Calls f(i, l, Y) for every real SH Y_lm of band l < B at the unit vector
// n (z the polar axis), i = l(l+1) + m, Y with its gradient in n (as a
// polynomial in x, y, z).  Y_l0 = K_l0 Pbar_l0(z); Y_l,+m / Y_l,-m =
// sqrt2 K_lm Pbar_lm(z) times Re / Im (x + i y)^m, with Pbar_lm the
// associated Legendre function (Condon-Shortley phase) over
// (1 - z^2)^(m/2): Pbar_mm = (-1)^m (2m-1)!!, Pbar_(m+1)m = (2m+1) z Pbar_mm,
// then (l - m) Pbar_lm = (2l-1) z Pbar_(l-1)m - (l+m-1) Pbar_(l-2)m.
template <class F>
__device__ __forceinline__ void sh_stream(const RenderArgs& a, V3 n, F f) {
  const G4 X = {n.x, 1.0f, 0.0f, 0.0f}, Y = {n.y, 0.0f, 1.0f, 0.0f}, Z = {n.z, 0.0f, 0.0f, 1.0f};
  G4 cr = {1.0f, 0.0f, 0.0f, 0.0f}, ci = {0.0f, 0.0f, 0.0f, 0.0f};
  float pmm = 1.0f;
  for (int m = 0; m < a.sh_bands; ++m) {
    if (m > 0) {
      const G4 t = X * cr - Y * ci;
      ci = X * ci + Y * cr;
      cr = t;
      pmm *= -(2.0f * (float)m - 1.0f);
    }
    G4 pa = {pmm, 0.0f, 0.0f, 0.0f}, pb = pa;
    for (int l = m; l < a.sh_bands; ++l) {
      G4 p;
      if (l == m) {
        p = pa;
      } else if (l == m + 1) {
        pb = Z * ((2.0f * (float)m + 1.0f) * pmm);
        p = pb;
      } else {
        p = (Z * pb * (2.0f * (float)l - 1.0f) - pa * (float)(l + m - 1)) * (1.0f / (float)(l - m));
        pa = pb;
        pb = p;
      }
      const float k = a.sh_norm[l * (l + 1) / 2 + m];
      if (m == 0) {
        f(l * (l + 1), l, p * k);
      } else {
        f(l * (l + 1) + m, l, p * cr * k);
        f(l * (l + 1) - m, l, p * ci * k);
      }
    }
  }
}

// E(n) per channel (values only).
__device__ __forceinline__ V3 sh_irradiance(const RenderArgs& a, V3 n) {
  V3 e = {0.0f, 0.0f, 0.0f};
  sh_stream(a, n, [&](int i, int l, G4 y) {
    const float w = a.sh_ash[l] * y.v;
    e.x += w * a.sh[3 * i]; e.y += w * a.sh[3 * i + 1]; e.z += w * a.sh[3 * i + 2];
  });
  return e;
}

}  // namespace fr
