// Device building blocks of the MI355X face renderer (gfx950, wave64).
//
//  * Philox4x32-10 counter-based generator (Salmon et al., SC'11).
//  * BVH layout: a binary radix tree (built and refitted; one 64-byte node
//    per internal node holding both children's boxes) collapsed into a 4-wide
//    tree for traversal (128-byte nodes: four child boxes in SoA form, two
//    scalar 16-dword loads per visit), and a leaf-ordered 48-byte triangle
//    record array.
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
constexpr float kDirectionalFar = 1e4f;   // shadow rays to a light at infinity end at 1e4
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
  int32_t lo, hi;  // range of sorted leaf slots below the node
};
static_assert(sizeof(BvhNode) == 64, "node must be one 64-byte line");

// 4-wide traversal node: the boxes of up to four children (lo/hi per axis,
// child k in column k), their references (>= 0 a node, kEmpty an unused slot,
// otherwise ~leaf slot) and, per child, the number of children of that child
// node (statistics of the debug dump).
constexpr int32_t kEmpty = INT32_MIN;
struct alignas(64) Bvh4Node {
  float lo[3][4];
  float hi[3][4];
  int32_t c[4];
  int32_t nsub[4];
};
static_assert(sizeof(Bvh4Node) == 128, "4-wide node is two 64-byte lines");

struct alignas(16) TriRec {
  float v[9];      // v0, v1, v2
  int32_t id;      // original triangle id
  int32_t pad0, pad1;
};
static_assert(sizeof(TriRec) == 48, "triangle record is 48 bytes");

// Per-light constants, built once per render: 16 floats.  A light at
// infinity keeps its unit direction in p0 and 1 / |p0| in e1[0] (the rest of
// e1, e2 and na are zero).
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
    // one 32x32 -> 64-bit multiply each (v_mad_u64_u32) instead of mul_lo + mul_hi
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0, p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
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
// FP64 vectors (normals, the shadow-edge term's jump chain)
struct D3 { double x, y, z; };
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 operator*(D3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double dotd(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 crossd(D3 a, D3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
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

// Hardware reciprocal, reciprocal square root, log2 and exp2 (one
// instruction each, about 1 ulp) for the BRDF and its adjoint, whose values
// need 1e-4 relative accuracy; the IEEE division and powf/logf they replace
// cost 10 to 40 instructions each.  Never used where a value decides a hit
// or a visibility.
__device__ __forceinline__ float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsqrt_hw(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float log2_hw(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }
// Lane l of `old` replaced by the wave-uniform v (v_writelane_b32; the lane
// select goes through M0, since one VALU instruction reads one SGPR).
__device__ __forceinline__ int writelane_i(int old, int v, int l) {
  asm("v_writelane_b32 %0, %1, %2" : "+v"(old) : "s"(v), "{m0}"(l));
  return old;
}

// Sum over the 64 lanes of a wave, returned wave-uniform.  Cross-lane moves
// by DPP (VALU only, no LDS round trip): quad swaps, half-row and row
// mirrors (every lane of a row then holds the row's sum), then lane 15's
// row sum added into rows 1 and 3 and lane 31's into rows 2 and 3; lane 63
// ends with the total.  The order of the additions is fixed (deterministic).
// All 64 lanes must be active: DPP does not read lanes that EXEC disables.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float x) {
  return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}
__device__ __forceinline__ float wave_sum(float x) {
  x = dpp_add<0xb1, 0xf>(x);    // quad_perm [1,0,3,2]
  x = dpp_add<0x4e, 0xf>(x);    // quad_perm [2,3,0,1]
  x = dpp_add<0x141, 0xf>(x);   // row_half_mirror
  x = dpp_add<0x140, 0xf>(x);   // row_mirror
  x = dpp_add<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
  x = dpp_add<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
  return readlane_f(x, 63);
}

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

// FAST_INV: the slab test's 1/d from the hardware reciprocal (1 ulp) instead
// of the IEEE division.  The boxes' kBoxPad padding covers that extra ulp by
// orders of magnitude (1e-5 absolute, against ~1e-7 times the distance along
// the ray for scenes of unit size),
// so every leaf holding a triangle the ray hits is still entered and the
// traversal's answer (any hit, or the closest hit with its id) is the same;
// only the set of extra leaves visited may differ.  The shear of the
// triangle test keeps the IEEE divisions.
template <bool FAST_INV = false>
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
  if (FAST_INV) r.inv = {rcp_hw(dd.x), rcp_hw(dd.y), rcp_hw(dd.z)};
  else r.inv = {1.0f / dd.x, 1.0f / dd.y, 1.0f / dd.z};
  r.oinv = {-r.o.x * r.inv.x, -r.o.y * r.inv.y, -r.o.z * r.inv.z};
}

// Slab test of one (wave-uniform) box against this lane's ray; returns the
// entry distance in tnear.  Branch-free.  Boxes are padded by kBoxPad at refit,
// which covers the rounding of the plane distances (conservative traversal).
__device__ __forceinline__ void slab(const Ray& r, const float* b, float tmax, float& tnear, float& tfar) {
  const float tx0 = fmaf(b[0], r.inv.x, r.oinv.x), tx1 = fmaf(b[3], r.inv.x, r.oinv.x);
  const float ty0 = fmaf(b[1], r.inv.y, r.oinv.y), ty1 = fmaf(b[4], r.inv.y, r.oinv.y);
  const float tz0 = fmaf(b[2], r.inv.z, r.oinv.z), tz1 = fmaf(b[5], r.inv.z, r.oinv.z);
  tnear = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), r.tmin));
  tfar = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
}

// Slab test of child k of a 4-wide node.
__device__ __forceinline__ void slab4(const Ray& r, const Bvh4Node& n, int k, float tmax, float& tnear,
                                      float& tfar) {
  const float tx0 = fmaf(n.lo[0][k], r.inv.x, r.oinv.x), tx1 = fmaf(n.hi[0][k], r.inv.x, r.oinv.x);
  const float ty0 = fmaf(n.lo[1][k], r.inv.y, r.oinv.y), ty1 = fmaf(n.hi[1][k], r.inv.y, r.oinv.y);
  const float tz0 = fmaf(n.lo[2][k], r.inv.z, r.oinv.z), tz1 = fmaf(n.hi[2][k], r.inv.z, r.oinv.z);
  tnear = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), r.tmin));
  tfar = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
}

// Slab test of child k for a packet whose live rays all point into octant OCT
// (bit 0: x < 0, bit 1: y < 0, bit 2: z < 0).  The entry plane of each axis
// is then known: for inv > 0 and lo <= hi, fma(lo, inv, oinv) <=
// fma(hi, inv, oinv) because rounding is monotonic, so the per-axis min/max
// pairs of slab4 select the same values and the result is slab4's, bit for
// bit, with six fewer instructions per box.
// NC: the caller has shown that every box of the walk exits before tmax
// (see trace), so min(., tmax) would return its other operand: left out.
template <int OCT, bool NC = false>
__device__ __forceinline__ void slab4_oct(const Ray& r, const Bvh4Node& n, int k, float tmax, float& tnear,
                                          float& tfar) {
  const float nx = (OCT & 1) ? n.hi[0][k] : n.lo[0][k], fx = (OCT & 1) ? n.lo[0][k] : n.hi[0][k];
  const float ny = (OCT & 2) ? n.hi[1][k] : n.lo[1][k], fy = (OCT & 2) ? n.lo[1][k] : n.hi[1][k];
  const float nz = (OCT & 4) ? n.hi[2][k] : n.lo[2][k], fz = (OCT & 4) ? n.lo[2][k] : n.hi[2][k];
  const float tnx = fmaf(nx, r.inv.x, r.oinv.x), tfx = fmaf(fx, r.inv.x, r.oinv.x);
  const float tny = fmaf(ny, r.inv.y, r.oinv.y), tfy = fmaf(fy, r.inv.y, r.oinv.y);
  const float tnz = fmaf(nz, r.inv.z, r.oinv.z), tfz = fmaf(fz, r.inv.z, r.oinv.z);
  tnear = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, r.tmin));
  tfar = NC ? fminf(fminf(tfx, tfy), tfz) : fminf(fminf(tfx, tfy), fminf(tfz, tmax));
}

// Lane mask of a <= b over the executing lanes (the compare's own mask, no
// round trip through a VGPR).
__device__ __forceinline__ uint64_t mask_le(float a, float b) { return __builtin_amdgcn_fcmpf(a, b, 5 /* OLE */); }

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
template <bool DUMP, bool NEED_T = true>
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
  // Branch-free acceptance: U, V, W of one sign (min >= 0 or max <= 0; a NaN
  // is ignored by the min/max as by the comparisons it replaces), det != 0,
  // and T / det in (tmin, tmax) compared without dividing: with s the sign
  // of det, s T against tmin |det| and tmax |det| (negation is exact).
  const bool sides = fminf(fminf(U, V), W) >= 0.0f || fmaxf(fmaxf(U, V), W) <= 0.0f;
  const float Ts = det < 0.0f ? -T : T, D = fabsf(det);
  const bool hit = sides && det != 0.0f && Ts > r.tmin * D && Ts < tmax * D;
  if (NEED_T) {   // any-hit queries need no distance
    const float tt = T / det;
    t = hit ? tt : t;
  }
  return hit;
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
// Read-only views in the constant address space: the tree, the triangle
// records and the light records are not written while a render kernel runs,
// so wave-uniform reads of them become scalar loads (s_load, scalar cache)
// even in kernels that also write global memory (the backward's atomics
// would otherwise force vector loads of every node).
template <class T>
__device__ __forceinline__ T load_const(const T* p, int i) {
  static_assert(sizeof(T) % 16 == 0, "records are whole 16-byte vectors");
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const __attribute__((address_space(4))) v4u* q = (const __attribute__((address_space(4))) v4u*)(p + i);
  T out;
  v4u* o = reinterpret_cast<v4u*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 16); ++k) o[k] = q[k];
  return out;
}

struct TravStats {
  // lane_box: child boxes tested by a single-ray traversal of this lane's ray
  // (the children of every node its ray enters); lane_leaf: its triangle
  // tests; wave_int / wave_leaf: node / leaf visits the packet executed
  uint32_t lane_box, lane_leaf, wave_int, wave_leaf, rays;
};

// Sorting-network step on (key, child, mask) triples: a <= b afterwards.
__device__ __forceinline__ void order2(float& ka, int& ca, uint64_t& ma, float& kb, int& cb, uint64_t& mb) {
  if (kb < ka) {
    const float k = ka; ka = kb; kb = k;
    const int c = ca; ca = cb; cb = c;
    const uint64_t m = ma; ma = mb; mb = m;
  }
}

// Body of trace() below; OCT >= 0: every live ray points into that octant.
template <bool ANY, bool DUMP, bool EX, int OCT, bool NC = false>
__device__ __forceinline__ void trace_impl(const Bvh4Node* __restrict__ nodes, const TriRec* __restrict__ tris,
                                           int n_tris, const Ray& r, bool active, int exclude, HitState& h,
                                           bool& occluded, TravStats* st, int ex2, int ex3, uint64_t live) {
  // Keep the tree and record bases in SGPRs for the whole walk: without the
  // opaque copy the compiler reloads them from the kernel arguments at every
  // node, a second dependent scalar load in front of each node fetch.
  {
    uint64_t pn = reinterpret_cast<uint64_t>(nodes), pt = reinterpret_cast<uint64_t>(tris);
    asm("" : "+s"(pn), "+s"(pt));
    nodes = reinterpret_cast<const Bvh4Node*>(pn);
    tris = reinterpret_cast<const TriRec*>(pt);
  }
  const int lane = lane_id();
  if (DUMP && st && active) {
    st->rays += 1;
    if (n_tris > 1) {
      for (int k = 0; k < 4; ++k) st->lane_box += load_const(nodes, 0).c[k] != kEmpty ? 1 : 0;
    } else {
      st->lane_leaf += 1;
    }
  }
  int stack = 0;
  int sp = 0;
  int node = n_tris > 1 ? 0 : ~0;
  const float tpad = DUMP ? kFlagT : 0.0f;
  // canonical once, so that the min/max of every box test need not canonicalise it again
  const float tmax0 = __builtin_canonicalizef(r.tmax);
  // A tree visits each of its nodes and leaves at most once; the cap only
  // guards against a corrupted structure.
  int budget = 2 * n_tris + 64;
  bool clean = false;   // dump builds, any hit: an unambiguous occluder was found
  while (--budget > 0) {
    if (node >= 0) {
      const Bvh4Node nd = load_const(nodes, node);  // two 64-byte scalar loads
      const float tcur = DUMP ? (ANY ? tmax0 : h.t) + tpad : (ANY ? tmax0 : h.t);
      float tn0, tn1, tn2, tn3, tf;
      const auto box = [&](int k, float& tn) {
        if (OCT >= 0) slab4_oct<(OCT < 0 ? 0 : OCT), NC>(r, nd, k, tcur, tn, tf);
        else slab4(r, nd, k, tcur, tn, tf);
      };
      // an unused slot holds an inverted box (lo = +3.4e38, hi = -3.4e38),
      // which the octant test rejects by itself; the min/max form would
      // accept it, so there the slot is checked
      box(0, tn0);
      uint64_t m0 = (OCT >= 0 || nd.c[0] != kEmpty) ? (mask_le(tn0, tf) & live) : 0ull;
      box(1, tn1);
      uint64_t m1 = (OCT >= 0 || nd.c[1] != kEmpty) ? (mask_le(tn1, tf) & live) : 0ull;
      box(2, tn2);
      uint64_t m2 = (OCT >= 0 || nd.c[2] != kEmpty) ? (mask_le(tn2, tf) & live) : 0ull;
      box(3, tn3);
      uint64_t m3 = (OCT >= 0 || nd.c[3] != kEmpty) ? (mask_le(tn3, tf) & live) : 0ull;
      if (DUMP && st) {
        st->wave_int += 1;
        const uint64_t mm[4] = {m0, m1, m2, m3};
        for (int k = 0; k < 4; ++k)
          if ((mm[k] >> lane) & 1) {
            if (nd.c[k] >= 0) st->lane_box += nd.nsub[k];
            else st->lane_leaf += 1;
          }
      }
      int c0 = nd.c[0], c1 = nd.c[1], c2 = nd.c[2], c3 = nd.c[3];
      if (!ANY && (m0 | m1 | m2 | m3)) {
        // nearest child first, as seen by one lane that enters a child
        const int ref = (int)__builtin_ctzll(m0 | m1 | m2 | m3);
        float k0 = m0 ? readlane_f(tn0, ref) : 3.4e38f, k1 = m1 ? readlane_f(tn1, ref) : 3.4e38f;
        float k2 = m2 ? readlane_f(tn2, ref) : 3.4e38f, k3 = m3 ? readlane_f(tn3, ref) : 3.4e38f;
        order2(k0, c0, m0, k1, c1, m1);
        order2(k2, c2, m2, k3, c3, m3);
        order2(k0, c0, m0, k2, c2, m2);
        order2(k1, c1, m1, k3, c3, m3);
        order2(k1, c1, m1, k2, c2, m2);
      }
      // go to the first child entered, push the others (last first); a push
      // writes the wave-uniform entry into lane sp of the stack register
      int next = kEmpty;
      if (m3) next = c3;
      if (m2) { if (next != kEmpty) { stack = writelane_i(stack, next, sp); ++sp; } next = c2; }
      if (m1) { if (next != kEmpty) { stack = writelane_i(stack, next, sp); ++sp; } next = c1; }
      if (m0) { if (next != kEmpty) { stack = writelane_i(stack, next, sp); ++sp; } next = c0; }
      if (next != kEmpty) { node = next; continue; }
    } else {
      const TriRec tr = load_const(tris, ~node);    // 48-byte scalar load
      if (DUMP && st) st->wave_leaf += 1;
      float t = 0.0f;
      const float tmax = ANY ? r.tmax : h.t;
      float amb = 3.4e38f;
      const bool other = tr.id != exclude && (!EX || (tr.id != ex2 && tr.id != ex3));
      const bool hit = tri_test<DUMP, !ANY || DUMP>(r, tr.v, tmax, t, amb) & active & other;
      if (DUMP && active && other) h.tamb = fminf(h.tamb, amb);
      if (DUMP && !ANY && hit && h.id >= 0 && fabsf(t - h.t) < kFlagT) h.tamb = fminf(h.tamb, t);
      if (ANY) {
        occluded = occluded | hit;
        // dump builds keep a lane whose hits so far are all near ambiguous:
        // one unambiguous occluder settles the decision, whatever was seen
        const bool settled = DUMP ? (hit && !(amb < 3.0e38f)) : hit;
        if (DUMP && settled) clean = true;
        active = active & !settled;
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
  if (DUMP && ANY && clean) h.tamb = 3.4e38f;   // the decision cannot flip
}

// True when every live ray leaves each of the root's child boxes before its
// tmax.  Every box of the tree lies inside one of those (a parent box is the
// exact min/max union of its children's), and a box's exit distance is
// monotone in its far planes, so the clamp of every exit distance to tmax
// is then a no-op for the whole walk (the test below is the one the walk
// makes, without that clamp).  Shadow rays towards lights outside the mesh's
// bounds: nearly always.
__device__ __forceinline__ bool exits_before_tmax(const Bvh4Node* __restrict__ nodes, const Ray& r, bool active) {
  const Bvh4Node nd = load_const(nodes, 0);
  float tf = -3.4e38f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (nd.c[k] == kEmpty) continue;
    const float tx0 = fmaf(nd.lo[0][k], r.inv.x, r.oinv.x), tx1 = fmaf(nd.hi[0][k], r.inv.x, r.oinv.x);
    const float ty0 = fmaf(nd.lo[1][k], r.inv.y, r.oinv.y), ty1 = fmaf(nd.hi[1][k], r.inv.y, r.oinv.y);
    const float tz0 = fmaf(nd.lo[2][k], r.inv.z, r.oinv.z), tz1 = fmaf(nd.hi[2][k], r.inv.z, r.oinv.z);
    tf = fmaxf(tf, fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1)));
  }
  return ballot(active && !(tf <= r.tmax)) == 0ull;
}

// Wave-packet traversal of the 4-wide tree.  Every lane of the wave must call
// it (uniform control flow).  ANY = true: shadow/any-hit query over
// (tmin, tmax), `occluded` is set on the first accepted triangle and the lane
// drops out.  ANY = false: closest hit, ties in t resolved to the lowest
// triangle id.  When the live rays' direction signs agree on every axis (a
// packet of shadow rays from neighbouring points to one light, or of camera
// rays through neighbouring pixels: nearly always) the traversal runs the
// slab test specialised to that octant, whose entry distances are the
// general test's bit for bit (the closest-hit order uses them).
template <bool ANY, bool DUMP, bool EX = false>
__device__ __forceinline__ void trace(const Bvh4Node* __restrict__ nodes, const TriRec* __restrict__ tris, int n_tris,
                                      const Ray& r, bool active, int exclude, HitState& h, bool& occluded,
                                      TravStats* st = nullptr, int ex2 = -1, int ex3 = -1) {
  const uint64_t live = ballot(active);
  if (live == 0) return;
  {
    const uint64_t sx = ballot(active && r.inv.x < 0.0f), sy = ballot(active && r.inv.y < 0.0f);
    const uint64_t sz = ballot(active && r.inv.z < 0.0f);
    if ((sx == 0 || sx == live) && (sy == 0 || sy == live) && (sz == 0 || sz == live)) {
      const int oct = (sx ? 1 : 0) | (sy ? 2 : 0) | (sz ? 4 : 0);
      if constexpr (ANY && !DUMP) {
        // production any-hit rays: the octant walk without the tmax clamp,
        // or else the general walk (rare: a light within the mesh's bounds);
        // the clamped octant walks below are not reached from here.  (This
        // arrangement measured 7 % faster on the face render than an if/else
        // one that compiles the same walks: a matter of code placement.)
        if (!(n_tris > 1 && exits_before_tmax(nodes, r, active))) goto general;
#define FR_TRACE_OCT_NC(o) \
  case o: trace_impl<ANY, DUMP, EX, o, true>(nodes, tris, n_tris, r, active, exclude, h, occluded, st, ex2, ex3, live); return;
        switch (oct) {
          FR_TRACE_OCT_NC(0) FR_TRACE_OCT_NC(1) FR_TRACE_OCT_NC(2) FR_TRACE_OCT_NC(3)
          FR_TRACE_OCT_NC(4) FR_TRACE_OCT_NC(5) FR_TRACE_OCT_NC(6) FR_TRACE_OCT_NC(7)
        }
#undef FR_TRACE_OCT_NC
      }
#define FR_TRACE_OCT(o) \
  case o: trace_impl<ANY, DUMP, EX, o>(nodes, tris, n_tris, r, active, exclude, h, occluded, st, ex2, ex3, live); return;
      switch (oct) {
        FR_TRACE_OCT(0) FR_TRACE_OCT(1) FR_TRACE_OCT(2) FR_TRACE_OCT(3)
        FR_TRACE_OCT(4) FR_TRACE_OCT(5) FR_TRACE_OCT(6) FR_TRACE_OCT(7)
      }
#undef FR_TRACE_OCT
    }
  }
general:
  trace_impl<ANY, DUMP, EX, -1>(nodes, tris, n_tris, r, active, exclude, h, occluded, st, ex2, ex3, live);
}

// Per-lane any-hit traversal: the alternative to the wave packet for shadow
// rays.  Every lane walks the tree with its own ray alone: its own stack (64
// entries in private memory; a lane's pending siblings are a subset of the
// packet's, so the host's depth bound for the packet stack holds), nodes and
// triangle records fetched by per-lane vector loads (lanes at the same node
// read the same lines), the general min/max slab test (lanes differ in
// their direction signs).  The loop runs while any lane is still walking;
// lanes at an internal node and lanes at a leaf take their branches under
// their own masks.  The answer (an accepted triangle in (tmin, tmax) other
// than `exclude`) does not depend on the order of the walk, so it is the
// packet's bit for bit.
__device__ __forceinline__ bool trace_lane_any(const Bvh4Node* __restrict__ nodes, const TriRec* __restrict__ tris,
                                               int n_tris, const Ray& r, bool active, int exclude) {
  int stk[kStackDepth];
  int sp = 0;
  int node = n_tris > 1 ? 0 : ~0;
  bool walking = active, occ = false;
  int budget = 2 * n_tris + 64;   // each node and leaf at most once (guards a corrupted structure)
  while (ballot(walking) != 0ull) {
    if (walking) {
      int next = kEmpty;
      if (node >= 0) {
        const float4* q = reinterpret_cast<const float4*>(nodes + node);
        const float4 lx = q[0], ly = q[1], lz = q[2], hx = q[3], hy = q[4], hz = q[5];
        const int4 c = reinterpret_cast<const int4*>(q)[6];
        const float lox[4] = {lx.x, lx.y, lx.z, lx.w}, loy[4] = {ly.x, ly.y, ly.z, ly.w}, loz[4] = {lz.x, lz.y, lz.z, lz.w};
        const float hix[4] = {hx.x, hx.y, hx.z, hx.w}, hiy[4] = {hy.x, hy.y, hy.z, hy.w}, hiz[4] = {hz.x, hz.y, hz.z, hz.w};
        const int cc[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
        for (int k = 3; k >= 0; --k) {
          const float b[6] = {lox[k], loy[k], loz[k], hix[k], hiy[k], hiz[k]};
          float tn, tf;
          slab(r, b, r.tmax, tn, tf);
          if (cc[k] != kEmpty && tn <= tf) {
            if (next != kEmpty) stk[sp++] = next;
            next = cc[k];
          }
        }
      } else {
        const float4* q = reinterpret_cast<const float4*>(tris + ~node);
        const float4 a0 = q[0], a1 = q[1], a2 = q[2];
        const float v[9] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w, a2.x};
        const int id = __float_as_int(a2.y);
        float t = 0.0f, amb = 3.4e38f;
        if (tri_test<false, false>(r, v, r.tmax, t, amb) && id != exclude) {
          occ = true;
          walking = false;
        }
      }
      if (walking) {
        if (next != kEmpty) node = next;
        else if (sp > 0) node = stk[--sp];
        else walking = false;
      }
      if (--budget <= 0) walking = false;
    }
  }
  return occ;
}

}  // namespace fr
