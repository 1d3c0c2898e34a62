// Primary-visibility boundary term of edge sampling (Sec. 4 "Edge Sampling").
//
// 1. Facing of every face w.r.t. the camera centre T: sign of
//    ((v1 - v0) x (v2 - v0)) . (T - v0), in FP64 and in exactly that order, so
//    the classification is bitwise that of an FP64 evaluation.
// 2. Silhouette edges (faces of opposite facing, or a single face) get their
//    film length in pixels (FP64); every other edge gets 0.  A fixed-order
//    FP64 scan gives the running sum.
// 3. Edge sample k picks the edge whose running-sum interval holds
//    ((k + u0)/n) * total (stratified), a point y = a + u1 (b - a) on its film
//    image, and traces two camera rays through y -/+ 1e-2 m (m the unit film
//    normal), each shaded with one point per light from counters
//    (k, 0, 0x80000001 + j, step).  The estimate
//       (total / n) ((f- - f+) . dE/dp[pixel of y]) (m . dy/dtheta)
//    goes to both edge vertices and to the camera; dy/dtheta is the film
//    velocity of the 3D edge point that projects to y.
#include "fr_shade.h"

namespace fr {

// Film offset of the side rays from the edge, in pixels.  It must exceed the
// FP32 tracer's near-edge band (4e-6 + 2e-6 t world units) on the film: at a
// 256^2 face 1e-3 pixel is ~8e-6 world units and would leave every side ray
// undecidable; 1e-2 pixel is ~8e-5 (and ~2e-5 at 1024^2).
constexpr double kEdgeSide = 1e-2;

__device__ __forceinline__ void face_front_block(const float* __restrict__ v, const int32_t* __restrict__ tris, int F,
                                                    const float* __restrict__ cam, uint8_t* __restrict__ front, int bid) {
  const int f = bid * 256 + threadIdx.x;
  if (f >= F) return;
  const int i0 = tris[3 * f], i1 = tris[3 * f + 1], i2 = tris[3 * f + 2];
  const double v0x = v[3 * i0], v0y = v[3 * i0 + 1], v0z = v[3 * i0 + 2];
  const double ax = (double)v[3 * i1] - v0x, ay = (double)v[3 * i1 + 1] - v0y, az = (double)v[3 * i1 + 2] - v0z;
  const double bx = (double)v[3 * i2] - v0x, by = (double)v[3 * i2 + 1] - v0y, bz = (double)v[3 * i2 + 2] - v0z;
  const double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
  const double wx = (double)cam[9] - v0x, wy = (double)cam[10] - v0y, wz = (double)cam[11] - v0z;
  front[f] = (nx * wx + ny * wy + nz * wz) > 0.0 ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_face_front(const float* __restrict__ v, const int32_t* __restrict__ tris, int F,
                                                    const float* __restrict__ cam, uint8_t* __restrict__ front) {
  face_front_block(v, tris, F, cam, front, blockIdx.x);
}

struct FilmD { double x, y, z; };

__device__ __forceinline__ FilmD project_d(const float* __restrict__ cam, double th, double aspect, int W, int H,
                                           double X, double Y, double Z) {
  const double dx = X - (double)cam[9], dy = Y - (double)cam[10], dz = Z - (double)cam[11];
  // camera frame R^T (X - T)
  const double px = (double)cam[0] * dx + (double)cam[3] * dy + (double)cam[6] * dz;
  const double py = (double)cam[1] * dx + (double)cam[4] * dy + (double)cam[7] * dz;
  const double pz = (double)cam[2] * dx + (double)cam[5] * dy + (double)cam[8] * dz;
  const double z = -pz;
  FilmD f;
  f.x = (px / z / (th * aspect) + 1.0) * (0.5 * W);
  f.y = (1.0 - py / z / th) * (0.5 * H);
  f.z = z;
  return f;
}

__device__ __forceinline__ void edge_len_block(const float* __restrict__ v, const int32_t* __restrict__ edges,
                                                  const int32_t* __restrict__ edge_faces, int E,
                                                  const uint8_t* __restrict__ front, const float* __restrict__ cam,
                                                  double th, double aspect, int W, int H, double* __restrict__ len, int bid) {
  const int e = bid * 256 + threadIdx.x;
  if (e >= E) return;
  const int f0 = edge_faces[2 * e], f1 = edge_faces[2 * e + 1];
  const bool sil = f1 < 0 || front[f0] != front[f1];
  double l = 0.0;
  if (sil) {
    const int a = edges[2 * e], b = edges[2 * e + 1];
    const FilmD pa = project_d(cam, th, aspect, W, H, v[3 * a], v[3 * a + 1], v[3 * a + 2]);
    const FilmD pb = project_d(cam, th, aspect, W, H, v[3 * b], v[3 * b + 1], v[3 * b + 2]);
    if (pa.z > 0.0 && pb.z > 0.0) l = hypot(pb.x - pa.x, pb.y - pa.y);
  }
  len[e] = l;
}

__global__ __launch_bounds__(256) void k_edge_len(const float* __restrict__ v, const int32_t* __restrict__ edges,
                                                  const int32_t* __restrict__ edge_faces, int E,
                                                  const uint8_t* __restrict__ front, const float* __restrict__ cam,
                                                  double th, double aspect, int W, int H, double* __restrict__ len) {
  edge_len_block(v, edges, edge_faces, E, front, cam, th, aspect, W, H, len, blockIdx.x);
}

// Inclusive FP64 scan in fixed order: per-thread serial runs + block scan.
// Inclusive running sum of the edge lengths (the sampling CDF) in two
// passes over tiles of 1024 edges: (1) each tile scans its edges (4 per
// thread, then a wave scan and the wave totals) and stores its total;
// (2) each tile adds the sum of the totals before it.  Fixed summation order.
constexpr int kScanTile = 1024;

__device__ __forceinline__ double wave_scan_incl(double x, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    const double y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

__device__ __forceinline__ void edge_scan_local_block(const double* __restrict__ len, int E, double* __restrict__ cdf,
                                                      double* __restrict__ part, int bid) {
  __shared__ double wsum[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int base = bid * kScanTile + 4 * threadIdx.x;
  double v[4], run = 0.0;
  for (int k = 0; k < 4; ++k) {
    run += base + k < E ? len[base + k] : 0.0;
    v[k] = run;
  }
  const double incl = wave_scan_incl(run, lane);
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  double pre = 0.0;
  for (int w = 0; w < wave; ++w) pre += wsum[w];
  const double excl = pre + (incl - run);
  for (int k = 0; k < 4; ++k)
    if (base + k < E) cdf[base + k] = excl + v[k];
  if (threadIdx.x == 255) part[bid] = pre + incl;
}

__device__ __forceinline__ void edge_scan_add_block(double* __restrict__ cdf, int E, const double* __restrict__ part,
                                                    int bid) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < bid; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double off = red[0];
  if (bid == 0) return;
  const int base = bid * kScanTile + 4 * threadIdx.x;
  for (int k = 0; k < 4; ++k)
    if (base + k < E) cdf[base + k] += off;
}

__global__ __launch_bounds__(256) void k_edge_scan_local(const double* __restrict__ len, int E,
                                                         double* __restrict__ cdf, double* __restrict__ part) {
  edge_scan_local_block(len, E, cdf, part, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_edge_scan_add(double* __restrict__ cdf, int E,
                                                       const double* __restrict__ part) {
  edge_scan_add_block(cdf, E, part, blockIdx.x);
}

// Side ray through film point (fx, fy) (FP64: at a grazing silhouette the
// shading point moves ~1/cos_o times faster than the film point, so an FP32
// film point would misplace it): its closest hit with the FP64
// barycentrics of the crossing (traced once per edge sample and side).
template <bool DUMP>
__device__ __forceinline__ PrimHit side_trace(const RenderArgs& a, double fx, double fy, bool active, bool& amb) {
  Sample sm;
  camera_ray_film(a, (float)fx, (float)fy, sm);
  HitState h;
  h.t = 3.4e38f; h.id = -1; h.tamb = 3.4e38f;
  bool dummy = false;
  trace<false, DUMP>(a.nodes, a.recs, a.F, sm.ray, active, -1, h, dummy);
  if (DUMP && active && hit_ambiguous(h)) amb = true;
  PrimHit ph = {active ? h.id : -1, h.t, 0.0, 0.0};
  if (ph.id >= 0) {
    const int* t = a.tris + 3 * h.id;
    const int vi[3] = {t[0], t[1], t[2]};
    double bd[3];
    bary64(a, fx, fy, vi, bd);
    ph.b1 = bd[1];
    ph.b2 = bd[2];
  }
  return ph;
}

// Shaded radiance (no 1/S) of the side ray through (fx, fy) with hit ph, over
// lights [j0, j1).
template <bool DUMP, bool TEX>
__device__ __forceinline__ V3 side_shade(const RenderArgs& a, double fx, double fy, const PrimHit& ph, int k, int j0,
                                         int j1, bool with_sh, bool& amb) {
  Sample sm;
  camera_ray_film(a, (float)fx, (float)fy, sm);
  const double bd[3] = {1.0 - ph.b1 - ph.b2, ph.b1, ph.b2};
  Frame fr = {};
  const bool shaded = ph.id >= 0 && shading_frame<TEX>(a, sm, ph.id, ph.t, bd, fr);
  if (DUMP && ph.id >= 0 && fabsf(fr.cos_o) < kFlagCos) amb = true;
  V3 L = {0.0f, 0.0f, 0.0f};
  // shadow decisions of every light of the chunk, then the shading of the visible ones
  const auto draw = [&](int j) { return philox((uint32_t)k, 0u, PURPOSE_EDGE + 1u + (uint32_t)(a.light0 + j), a.step, a.k0, a.k1); };
  const auto note = [&](int, bool lit, bool, const LightSample& ls, const HitState& sh) {
    if (shaded && ls.amb) amb = true;
    if (lit && sh.tamb < 3.0e38f) amb = true;
  };
  const auto skip = [](int) {};
  const uint32_t vmask = shadow_mask<DUMP>(a, j0, j1, shaded, fr, ph.id, draw, note, skip, nullptr);
  for (int j = j0; j < j1; ++j) {
    const bool vis = (vmask >> (j - j0)) & 1u;
    if (!ballot(vis)) continue;
    const LightRec Lj = load_const(a.lights, j);
    const U4 r = Lj.shape == FR_LIGHT_DIRECTIONAL ? U4{0u, 0u, 0u, 0u} : draw(j);
    LightSample ls;
    light_point(Lj, unit24(r.x), unit24(r.y), fr, ls);
    if (vis) {
      float f[3], g1f = 0.0f;
      brdf_eval<DUMP>(a.variant, a.components, fr, ls, f, g1f);
      if (DUMP && g1f != 0.0f) amb = true;
      L.x += Lj.rad[0] * f[0] * ls.geom;
      L.y += Lj.rad[1] * f[1] * ls.geom;
      L.z += Lj.rad[2] * f[2] * ls.geom;
    }
  }
  if (with_sh && a.sh_bands > 0 && (a.components & 1)) {
    const V3 e = sh_irradiance(a, shaded ? fr.ns : V3{0.0f, 0.0f, 1.0f});
    if (shaded) L = L + V3{fr.c.x * e.x, fr.c.y * e.y, fr.c.z * e.z} * (1.0f / kPi);
  }
  return L;
}

// One block = 64 consecutive edge samples (lane = sample) and one group of
// lights; its four waves are the group's light chunks.  Waves 0 and 1 trace
// the minus and plus side rays into LDS; every wave shades both sides with
// its lights; the last wave to arrive sums the chunks in order and scatters
// the group's part of the estimate (linear in f- - f+, so the groups' parts
// add up in the integer sums).
template <bool DUMP, bool TEX>
__device__ __forceinline__ void edge_samples_block(const RenderArgs& a, const EdgeArgs& e, int bid) {
  __shared__ PrimHit side_hit[2][64];
  __shared__ float side_L[4][64][6];
  __shared__ int arrived;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lgroup = bid / e.bx, sblock = bid - lgroup * e.bx;
  const int light0 = lgroup * e.gsize;
  const int Lg = max(0, min(e.gsize, a.L - light0));
  const int lc = max(1, cdiv(Lg, 4));
  const int nch = max(1, cdiv(Lg, lc));
  const int j0 = light0 + wv * lc, j1 = min(light0 + Lg, j0 + lc);
  const int k = sblock * 64 + lane;
  if (threadIdx.x == 0) arrived = 0;
  const bool in = k < e.n_samples;
  const double ltot = e.cdf[e.E - 1];
  int eid = 0, pid = -1;
  bool amb = false;
  double fx = 0.0, fy = 0.0, mxd = 0.0, myd = 0.0;
  float mx = 0.0f, my = 0.0f, u1 = 0.0f;
  double pax = 0, pay = 0, paz = 1, pbz = 1;
  if (in && ltot > 0.0) {
    const U4 r = philox((uint32_t)k, 0u, PURPOSE_EDGE, a.step, a.k0, a.k1);
    const double target = ((double)k + (double)unit24(r.x)) / (double)e.n_samples * ltot;
    int lo = 0, hi = e.E - 1;          // first e with cdf[e] > target
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (e.cdf[mid] > target) hi = mid; else lo = mid + 1;
    }
    eid = lo;
    const double c1 = e.cdf[eid], c0 = eid > 0 ? e.cdf[eid - 1] : 0.0;
    if (fabs(target - c0) < 1e-9 * ltot || fabs(target - c1) < 1e-9 * ltot) amb = true;
    const int va = e.edges[2 * eid], vb = e.edges[2 * eid + 1];
    const FilmD pa = project_d(a.cam, e.th, e.aspect, a.W, a.H, a.verts[3 * va], a.verts[3 * va + 1], a.verts[3 * va + 2]);
    const FilmD pb = project_d(a.cam, e.th, e.aspect, a.W, a.H, a.verts[3 * vb], a.verts[3 * vb + 1], a.verts[3 * vb + 2]);
    const double u = (double)unit24(r.y);
    const double yx = pa.x + u * (pb.x - pa.x), yy = pa.y + u * (pb.y - pa.y);
    const double lx = pb.x - pa.x, ly = pb.y - pa.y, ll = hypot(lx, ly);
    mxd = -ly / ll;
    myd = lx / ll;
    mx = (float)mxd;
    my = (float)myd;
    fx = yx;
    fy = yy;
    const int pxi = (int)floor(yx), pyi = (int)floor(yy);
    if (pxi >= 0 && pxi < a.W && pyi >= 0 && pyi < a.H) pid = pyi * a.W + pxi;
    u1 = (float)u;
    pax = pa.x; pay = pa.y; paz = pa.z; pbz = pb.z;
  }
  const bool active = pid >= 0;
  const double fxm = fx - kEdgeSide * mxd, fym = fy - kEdgeSide * myd, fxp = fx + kEdgeSide * mxd,
               fyp = fy + kEdgeSide * myd;
  if (wv < 2) side_hit[wv][lane] = side_trace<DUMP>(a, wv ? fxp : fxm, wv ? fyp : fym, active, amb);
  __syncthreads();
  const PrimHit hm = side_hit[0][lane], hp = side_hit[1][lane];
  const bool with_sh = wv == 0 && lgroup == 0;   // the SH light once per sample
  const V3 Lm = side_shade<DUMP, TEX>(a, fxm, fym, hm, k, j0, j1, with_sh, amb);
  const V3 Lp = side_shade<DUMP, TEX>(a, fxp, fyp, hp, k, j0, j1, with_sh, amb);
  if (DUMP && in) {
    if (wv == 0 && lgroup == 0) {
      e.dbg_rec[4 * k] = eid; e.dbg_rec[4 * k + 1] = pid; e.dbg_rec[4 * k + 2] = hm.id; e.dbg_rec[4 * k + 3] = hp.id;
    }
    if (amb) e.dbg_flag[k] = 1;   // OR over the waves: the caller zeroes the flags
  }
  {
    float* q = side_L[wv][lane];
    q[0] = Lm.x; q[1] = Lm.y; q[2] = Lm.z; q[3] = Lp.x; q[4] = Lp.y; q[5] = Lp.z;
  }
  __threadfence_block();
  int n_arr = 0;
  if (lane == 0) n_arr = atomicAdd(&arrived, 1);
  if (__builtin_amdgcn_readlane(n_arr, 0) != 3) return;   // another wave finishes this group
  __threadfence_block();
  V3 Sm = {0.0f, 0.0f, 0.0f}, Sp = {0.0f, 0.0f, 0.0f};
  for (int c = 0; c < nch; ++c) {
    const float* q = side_L[c][lane];
    Sm = Sm + V3{q[0], q[1], q[2]};
    Sp = Sp + V3{q[3], q[4], q[5]};
  }
  float gcam[12];
  for (int q = 0; q < 12; ++q) gcam[q] = 0.0f;
  if (active) {
    const float dl = (Sm.x - Sp.x) * e.dEdp[3 * pid] + (Sm.y - Sp.y) * e.dEdp[3 * pid + 1] +
                     (Sm.z - Sp.z) * e.dEdp[3 * pid + 2];
    const float wgt = (float)(ltot / (double)e.n_samples) * (dl * grad_scale(e.gmax));
    if (wgt != 0.0f) {
      // film velocity of X(w) = (1 - w) A + w B, w perspective-correct
      const float w = (float)(((double)u1 / pbz) / ((1.0 - (double)u1) / paz + (double)u1 / pbz));
      const int va = e.edges[2 * eid], vb = e.edges[2 * eid + 1];
      const V3 A = ld3(a.verts, va), B = ld3(a.verts, vb);
      const V3 X = A * (1.0f - w) + B * w;
      const float* R = a.cam;
      const V3 dX = {X.x - R[9], X.y - R[10], X.z - R[11]};
      const V3 pc = {R[0] * dX.x + R[3] * dX.y + R[6] * dX.z, R[1] * dX.x + R[4] * dX.y + R[7] * dX.z,
                     R[2] * dX.x + R[5] * dX.y + R[8] * dX.z};
      const float z = -pc.z;
      const float Ax = (float)(0.5 * a.W / (e.th * e.aspect)), Ay = (float)(0.5 * a.H / e.th);
      // m . d(film)/d(pc)
      const V3 gpc = {mx * Ax / z, -my * Ay / z, mx * Ax * pc.x / (z * z) - my * Ay * pc.y / (z * z)};
      const V3 gX = {R[0] * gpc.x + R[1] * gpc.y + R[2] * gpc.z, R[3] * gpc.x + R[4] * gpc.y + R[5] * gpc.z,
                     R[6] * gpc.x + R[7] * gpc.y + R[8] * gpc.z};
      const float sa = wgt * (1.0f - w), sb = wgt * w;
      if (e.gverts) {
        fix_add(e.gverts + 3 * va, gX.x * sa); fix_add(e.gverts + 3 * va + 1, gX.y * sa);
        fix_add(e.gverts + 3 * va + 2, gX.z * sa);
        fix_add(e.gverts + 3 * vb, gX.x * sb); fix_add(e.gverts + 3 * vb + 1, gX.y * sb);
        fix_add(e.gverts + 3 * vb + 2, gX.z * sb);
      }
      // pc_i = sum_k R[k][i] (X - T)_k  ->  dR[k][i] = (X - T)_k gpc_i ; dT = -R gpc
      const float gp[3] = {gpc.x, gpc.y, gpc.z}, dd[3] = {dX.x, dX.y, dX.z};
      for (int kk = 0; kk < 3; ++kk)
        for (int ii = 0; ii < 3; ++ii) gcam[3 * kk + ii] = wgt * dd[kk] * gp[ii];
      gcam[9] = -wgt * gX.x; gcam[10] = -wgt * gX.y; gcam[11] = -wgt * gX.z;
    }
  }
  if (e.gcam) {
    for (int q = 0; q < 12; ++q) {
      const float t = wave_sum(gcam[q]);
      if (lane == 0 && t != 0.0f) fix_add(e.gcam + q, t);
    }
  }
}

template <bool DUMP, bool TEX>
// Eight waves per SIMD (64 VGPRs): alone no faster than six, but it runs
// beside the interior adjoint (128 VGPRs per wave), and the registers it
// leaves free hold adjoint waves (face step 2.43 -> 2.41 ms).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_edge_samples(RenderArgs a, EdgeArgs e) {
  edge_samples_block<DUMP, TEX>(a, e, blockIdx.x);
}

void launch_edges(MeshDev& m, const RenderArgs& a, const float* dEdp, int n_samples, fix_t* gverts, fix_t* gcam,
                  int32_t* dbg_rec, uint8_t* dbg_flag, double tan_half, hipStream_t st) {
  // the edge samples read dE/dp under the same scale as the interior adjoint (a.gmax)
  hipLaunchKernelGGL(k_face_front, dim3((m.F + 255) / 256), dim3(256), 0, st, a.verts, m.tris, m.F, a.cam,
                     m.face_front);
  const double aspect = (double)a.W / (double)a.H;
  hipLaunchKernelGGL(k_edge_len, dim3((m.E + 255) / 256), dim3(256), 0, st, a.verts, m.edges, m.edge_faces, m.E,
                     m.face_front, a.cam, tan_half, aspect, a.W, a.H, m.edge_len);
  const int tiles = cdiv(m.E, kScanTile);
  hipLaunchKernelGGL(k_edge_scan_local, dim3(tiles), dim3(256), 0, st, m.edge_len, m.E, m.edge_cdf, m.scan_part);
  hipLaunchKernelGGL(k_edge_scan_add, dim3(tiles), dim3(256), 0, st, m.edge_cdf, m.E, m.scan_part);
  EdgeArgs e;
  e.edges = m.edges; e.cdf = m.edge_cdf; e.E = m.E; e.n_samples = n_samples;
  e.th = tan_half; e.aspect = aspect; e.dEdp = dEdp; e.gmax = a.gmax; e.gverts = gverts; e.gcam = gcam;
  e.dbg_rec = dbg_rec; e.dbg_flag = dbg_flag;
  edge_groups(a.L, n_samples, e);
  const int blocks = e.bx * e.n_groups;
  if (a.M > 0) {
    if (dbg_rec)
      hipLaunchKernelGGL((k_edge_samples<true, true>), dim3(blocks), dim3(256), 0, st, a, e);
    else
      hipLaunchKernelGGL((k_edge_samples<false, true>), dim3(blocks), dim3(256), 0, st, a, e);
  } else if (dbg_rec) {
    hipLaunchKernelGGL((k_edge_samples<true, false>), dim3(blocks), dim3(256), 0, st, a, e);
  } else {
    hipLaunchKernelGGL((k_edge_samples<false, false>), dim3(blocks), dim3(256), 0, st, a, e);
  }
}

void edge_groups(int L, int n_samples, EdgeArgs& e) {
  e.bx = std::max(1, cdiv(n_samples, 64));
  // light groups only to reach ~1024 blocks (fewer samples): each group repeats the
  // sample's setup and side rays (65,536 samples: 1 group 451 us, 2 groups 472 us)
  int ng = std::max(1, std::max(cdiv(L, kBwdMaxLights), cdiv(1024, e.bx)));
  ng = std::min(ng, std::max(1, cdiv(L, 4)));
  e.gsize = cdiv(L, ng);
  e.n_groups = L > 0 ? cdiv(L, e.gsize) : 1;
}

}  // namespace fr
