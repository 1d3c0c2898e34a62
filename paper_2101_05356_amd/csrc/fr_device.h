// Device building blocks of the MI355X face renderer (gfx950, wave64).
//
//  * Philox4x32-10 counter-based generator (Salmon et al., SC'11).
//  * BVH layout: binary radix tree, one 64-byte node per internal node
//    holding both children's boxes (one scalar 16-dword load per visit), and
//    a leaf-ordered 48-byte triangle record array.
//  * Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013).
//  * Wave-packet traversal: the 64 lanes of a wave trace their own rays
//    through ONE shared, wave-uniform traversal order.  Node and triangle
//    records are fetched with scalar loads into SGPRs and tested against all
//    lanes at once; lanes vote (ballot) on which children to visit.  The
//    traversal stack is wave-uniform, so it lives in a single VGPR with entry
//    k held in lane k (a masked select to push, v_readlane to pop), 64
//    entries deep, using no LDS and no scratch.
//
// The render's rays are coherent by construction: a wave holds the samples of
// a few neighbouring pixels, and all of its lanes trace their shadow rays to
// the same light at the same time.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fr {

constexpr int kWave = 64;
constexpr int kStackDepth = 64;        // entries of the wave-uniform stack
constexpr float kShadowTmin = 1e-4f;   // shadow rays start 1e-4 from the shading point
constexpr float kRoughMin = 1e-3f, kRoughMax = 1.0f;
constexpr float kPi = 3.14159265358979323846f;
constexpr float kBoxPad = 1e-5f;       // absolute box enlargement (conservative traversal)

// Decision-ambiguity bands of the debug dump (FP32, wider than the FP64
// reference's 1e-6 so that every decision FP32 could get wrong is marked).
constexpr float kFlagDist = 4e-6f;     // ray-to-edge distance, plus kFlagDistT * t
constexpr float kFlagDistT = 2e-6f;
constexpr float kFlagT = 1e-5f;        // hit distance ties / range ends
constexpr float kFlagCos = 1e-5f;      // cosines at the cull threshold
constexpr float kFlagG1 = 1e-5f;       // relative distance of G1's a to 1.6

// Visibility codes of the debug dump.
constexpr uint8_t VIS_OCCLUDED = 0, VIS_VISIBLE = 1, VIS_CULLED = 2, VIS_NONE = 3, VIS_FLAG = 0x80;

// Philox purposes (third counter word).
constexpr uint32_t PURPOSE_JITTER = 0u;
constexpr uint32_t PURPOSE_EDGE = 0x80000000u;

struct alignas(16) BvhNode {
  float b0[6];     // child 0 box: min xyz, max xyz
  float b1[6];     // child 1 box
  int32_t c0, c1;  // >= 0: internal node index; < 0: ~leaf slot
  int32_t pad0, pad1;
};
static_assert(sizeof(BvhNode) == 64, "node must be one 64-byte line");

struct alignas(16) TriRec {
  float v[9];      // v0, v1, v2
  int32_t id;      // original triangle id
  int32_t pad0, pad1;
};
static_assert(sizeof(TriRec) == 48, "triangle record is 48 bytes");

// Per-light constants, built once per render: 16 floats.
struct alignas(16) LightRec {
  float p0[3], e1[3], e2[3];
  float na[3];     // -kappa (e1 x e2): A_j (-n_j) with kappa = 1 (parallelogram) or 1/2 (triangle)
  float rad[3];
  int32_t shape;
};
static_assert(sizeof(LightRec) == 64, "light record is 64 bytes");

// ---------------------------------------------------------------------------
// Philox4x32-10
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                     uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// Top 24 bits -> [0,1), exact in FP32.
__device__ __forceinline__ float unit24(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

// ---------------------------------------------------------------------------
// Small vector helpers (no FMA contraction is assumed: the library is built
// with -ffp-contract=off; fused operations are written explicitly).
// ---------------------------------------------------------------------------
struct V3 { float x, y, z; };
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(V3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 ld3(const float* __restrict__ p, int i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// Rays
// ---------------------------------------------------------------------------
// The Woop-Benthin-Wald test maps vertices into a ray frame in which the ray
// is the +z axis: permute axes so that z is the dominant direction component,
// then shear.  Here the permutation and shear are folded into one per-lane
// affine map (rows Mx, My, Mz and offsets -M.o): a sheared coordinate costs
// three FMAs and no per-lane component selects.  Watertightness is kept: a
// vertex shared by two triangles gets bitwise the same sheared coordinates in
// both tests, and an edge function evaluated from the other side is the exact
// negation (products commute, a - b = -(b - a); FMA contraction is off).
struct Ray {
  V3 o, d;
  V3 inv;                // 1/d with zero components replaced by +-1e-30 first
  V3 oinv;               // -o * inv (slab test: t = b * inv + oinv)
  V3 Mx, My, Mz;         // shear rows
  float cx, cy, cz;      // -(M . o)
  float tmin, tmax;
};

__device__ __forceinline__ float comp(V3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }
__device__ __forceinline__ V3 unit_axis(int k, float s) {
  return {k == 0 ? s : 0.0f, k == 1 ? s : 0.0f, k == 2 ? s : 0.0f};
}

__device__ __forceinline__ void ray_setup(Ray& r) {
  const float ax = fabsf(r.d.x), ay = fabsf(r.d.y), az = fabsf(r.d.z);
  const int kz = ax > ay ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  const float dz = comp(r.d, kz);
  if (dz < 0.0f) { const int t = kx; kx = ky; ky = t; }
  const float Sx = comp(r.d, kx) / dz, Sy = comp(r.d, ky) / dz, Sz = 1.0f / dz;
  r.Mx = unit_axis(kx, 1.0f) + unit_axis(kz, -Sx);
  r.My = unit_axis(ky, 1.0f) + unit_axis(kz, -Sy);
  r.Mz = unit_axis(kz, Sz);
  r.cx = -fmaf(r.Mx.x, r.o.x, fmaf(r.Mx.y, r.o.y, r.Mx.z * r.o.z));
  r.cy = -fmaf(r.My.x, r.o.x, fmaf(r.My.y, r.o.y, r.My.z * r.o.z));
  r.cz = -fmaf(r.Mz.x, r.o.x, fmaf(r.Mz.y, r.o.y, r.Mz.z * r.o.z));
  const float tiny = 1e-30f;
  const V3 dd = {fabsf(r.d.x) < tiny ? copysignf(tiny, r.d.x) : r.d.x,
                 fabsf(r.d.y) < tiny ? copysignf(tiny, r.d.y) : r.d.y,
                 fabsf(r.d.z) < tiny ? copysignf(tiny, r.d.z) : r.d.z};
  r.inv = {1.0f / dd.x, 1.0f / dd.y, 1.0f / dd.z};
  r.oinv = {-r.o.x * r.inv.x, -r.o.y * r.inv.y, -r.o.z * r.inv.z};
}

// Slab test of one (wave-uniform) box against this lane's ray; returns the
// entry distance in tnear.  Branch-free.  Boxes are padded by kBoxPad at refit,
// which covers the rounding of the plane distances (conservative traversal).
__device__ __forceinline__ bool slab(const Ray& r, const float* b, float tmax, float& tnear) {
  const float tx0 = fmaf(b[0], r.inv.x, r.oinv.x), tx1 = fmaf(b[3], r.inv.x, r.oinv.x);
  const float ty0 = fmaf(b[1], r.inv.y, r.oinv.y), ty1 = fmaf(b[4], r.inv.y, r.oinv.y);
  const float tz0 = fmaf(b[2], r.inv.z, r.oinv.z), tz1 = fmaf(b[5], r.inv.z, r.oinv.z);
  const float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), r.tmin));
  const float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
  tnear = tn;
  return tn <= tf;
}

__device__ __forceinline__ float shear(const V3& M, float c, float x, float y, float z) {
  return fmaf(x, M.x, fmaf(y, M.y, fmaf(z, M.z, c)));
}

// Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013) of this
// lane's ray against a (wave-uniform) triangle v[9].  Accepts crossings with
// t in (tmin, tmax) by comparing T against tmin*det and tmax*det (no division);
// on acceptance t = T/det.  `amb_t` (dump builds only) is lowered to the
// crossing distance when the ray passes within the ambiguity band of the
// triangle boundary, or crosses it within kFlagT of tmin / tmax (0 for grazing
// rays, whose distance is ill-conditioned).
template <bool DUMP>
__device__ __forceinline__ bool tri_test(const Ray& r, const float* v, float tmax, float& t, float& amb_t) {
  const float Ax = shear(r.Mx, r.cx, v[0], v[1], v[2]), Ay = shear(r.My, r.cy, v[0], v[1], v[2]);
  const float Bx = shear(r.Mx, r.cx, v[3], v[4], v[5]), By = shear(r.My, r.cy, v[3], v[4], v[5]);
  const float Cx = shear(r.Mx, r.cx, v[6], v[7], v[8]), Cy = shear(r.My, r.cy, v[6], v[7], v[8]);
  float U = Cx * By - Cy * Bx;
  float V = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
    V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
    W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
  }
  const float Az = shear(r.Mz, r.cz, v[0], v[1], v[2]);
  const float Bz = shear(r.Mz, r.cz, v[3], v[4], v[5]);
  const float Cz = shear(r.Mz, r.cz, v[6], v[7], v[8]);
  const float det = U + V + W;
  const float T = U * Az + V * Bz + W * Cz;
  if (DUMP) {
    // distance (in the sheared plane) of the ray from each edge line
    const float lU = sqrtf((Bx - Cx) * (Bx - Cx) + (By - Cy) * (By - Cy));
    const float lV = sqrtf((Cx - Ax) * (Cx - Ax) + (Cy - Ay) * (Cy - Ay));
    const float lW = sqrtf((Ax - Bx) * (Ax - Bx) + (Ay - By) * (Ay - By));
    const float sg = det < 0.0f ? -1.0f : 1.0f;
    const float dU = sg * U / fmaxf(lU, 1e-30f), dV = sg * V / fmaxf(lV, 1e-30f), dW = sg * W / fmaxf(lW, 1e-30f);
    const float tc = det != 0.0f ? T / det : 0.0f;
    const float band = kFlagDist + kFlagDistT * fmaxf(fabsf(tc), 1.0f);
    const bool inside_ish = dU > -band && dV > -band && dW > -band;
    const bool at_edge = fminf(fabsf(dU), fminf(fabsf(dV), fabsf(dW))) < band;
    const bool grazing = fabsf(det) <= 1e-6f * (lU * lV + lV * lW + lW * lU);
    const bool in_range = grazing || (tc > r.tmin - kFlagT && tc < tmax + kFlagT);
    if (inside_ish && (at_edge || grazing) && in_range) amb_t = fminf(amb_t, grazing ? 0.0f : tc);
    const bool inside_all = (U >= 0.0f && V >= 0.0f && W >= 0.0f) || (U <= 0.0f && V <= 0.0f && W <= 0.0f);
    if (inside_all && det != 0.0f && (fabsf(tc - r.tmin) < kFlagT || fabsf(tc - tmax) < kFlagT))
      amb_t = fminf(amb_t, tc);
  }
  if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
  if (det == 0.0f) return false;
  const bool in_range = det > 0.0f ? (T > r.tmin * det && T < tmax * det) : (T < r.tmin * det && T > tmax * det);
  if (!in_range) return false;
  t = T / det;
  return true;
}

struct HitState {
  float t;
  int id;
  float tamb;    // dump builds: nearest ambiguous crossing (+inf if none)
};

// Closest-hit decision is ambiguous when an ambiguous crossing was recorded
// at or before the hit (or anywhere, for a miss).
__device__ __forceinline__ bool hit_ambiguous(const HitState& h) {
  return h.tamb < 3.0e38f && (h.id < 0 || h.tamb <= h.t + kFlagT);
}

// Traversal statistics of dump builds.  Lane counts: child boxes this lane's
// ray enters (internal nodes / leaves), i.e. the visits a single-ray
// traversal of the same tree would make.  Wave counts: node and leaf visits
// the packet executes.
struct TravStats {
  uint32_t lane_int, lane_leaf, wave_int, wave_leaf, rays;
};

// Wave-packet traversal.  Every lane of the wave must call it (uniform control
// flow).  ANY = true: shadow/any-hit query over (tmin, tmax), `occluded` is set
// on the first accepted triangle and the lane drops out.  ANY = false:
// closest hit, ties in t resolved to the lowest triangle id.
template <bool ANY, bool DUMP>
__device__ __forceinline__ void trace(const BvhNode* __restrict__ nodes, const TriRec* __restrict__ tris, int n_tris,
                                      const Ray& r, bool active, int exclude, HitState& h, bool& occluded,
                                      TravStats* st = nullptr) {
  uint64_t live = ballot(active);
  if (live == 0) return;
  if (DUMP && st && active) { st->rays += 1; st->lane_int += n_tris > 1 ? 1 : 0; st->lane_leaf += n_tris > 1 ? 0 : 1; }
  const int lane = lane_id();
  int stack = 0;
  int sp = 0;
  int node = n_tris > 1 ? 0 : ~0;
  const float tpad = DUMP ? kFlagT : 0.0f;
  // A tree visits each of its 2F - 1 nodes at most once; the cap only guards
  // against a corrupted structure.
  int budget = 2 * n_tris + 64;
  while (--budget > 0) {
    if (node >= 0) {
      const BvhNode nd = nodes[node];               // one 64-byte scalar load
      const float tcur = (ANY ? r.tmax : h.t) + tpad;
      float tn0, tn1;
      const bool h0 = slab(r, nd.b0, tcur, tn0) & active;
      const bool h1 = slab(r, nd.b1, tcur, tn1) & active;
      const uint64_t m0 = ballot(h0), m1 = ballot(h1);
      if (DUMP && st) {
        st->wave_int += 1;
        st->lane_int += (h0 && nd.c0 >= 0 ? 1 : 0) + (h1 && nd.c1 >= 0 ? 1 : 0);
        st->lane_leaf += (h0 && nd.c0 < 0 ? 1 : 0) + (h1 && nd.c1 < 0 ? 1 : 0);
      }
      if (m0 && m1) {
        const uint64_t both = m0 & m1;
        const int ref = both ? (int)__builtin_ctzll(both) : (int)__builtin_ctzll(m0);
        const bool near0 = readlane_i(tn0 <= tn1 ? 1 : 0, ref) != 0;
        const int nearc = near0 ? nd.c0 : nd.c1, farc = near0 ? nd.c1 : nd.c0;
        if (sp < kStackDepth) {                 // depth <= 64 is checked at build
          stack = (lane == sp) ? farc : stack;  // entry sp lives in lane sp
          ++sp;
        }
        node = nearc;
        continue;
      }
      if (m0) { node = nd.c0; continue; }
      if (m1) { node = nd.c1; continue; }
    } else {
      const TriRec tr = tris[~node];                // 48-byte scalar load
      if (DUMP && st) st->wave_leaf += 1;
      float t = 0.0f;
      const float tmax = ANY ? r.tmax : h.t;
      const bool hit = tri_test<DUMP>(r, tr.v, tmax, t, h.tamb) & active & (tr.id != exclude);
      if (DUMP && !ANY && hit && h.id >= 0 && fabsf(t - h.t) < kFlagT) h.tamb = fminf(h.tamb, t);
      if (ANY) {
        occluded = occluded | hit;
        active = active & !hit;
        live = ballot(active);
        if (live == 0) break;
      } else if (hit && (t < h.t || (t == h.t && tr.id < h.id))) {
        h.t = t;
        h.id = tr.id;
      }
    }
    if (sp == 0) break;
    --sp;
    node = readlane_i(stack, sp);
  }
}

}  // namespace fr
