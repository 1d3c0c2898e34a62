// Shadow-edge (secondary visibility) boundary term of the adjoint, Sec. 4
// "Edge Sampling" applied to the shadow rays of Sec. 3.3.
//
// Light j seen from a shading point x contributes kappa^-1 int int h V dw1
// dw2 over the light's parameters (y = p0 + w1 e1 + w2 e2; kappa = 1 for a
// parallelogram, 1/2 for a triangle), h the render's per-sample value of the
// light at y.  On a line w2 = v the visibility V is piecewise constant in
// w1; the derivative of the line integral gains h(w1_k) J_k dw1_k/dtheta at
// each jump (J_k = V(w1_k-) - V(w1_k+)).  One thread per line sample: it
// draws a camera sample, a light and v, traces the camera ray, then walks
// the 4-wide tree with the wedge spanned by x and the line (a box is entered
// when it straddles the wedge's plane and overlaps the wedge's bounding
// box).  An edge (a, b) of a visited triangle is a jump when it crosses the
// plane inside the wedge, its faces other than x's own triangle fold to one
// side as seen from x, and a shadow ray from x to the jump's light point,
// excluding those faces, is free.  Each edge is handled once, by its lower
// face.  The jump solves D(w1) = det[a - x, b - x, y(w1) - x] = 0 (linear in
// w1), so dw1/dtheta = -(dD/dtheta) / (dD/dw1), scattered to a, b, the light's
// p0, e1, e2 and, through the camera ray's crossing with x's triangle plane
// (x = o + t d, t = (v0 - o) . n / d . n), to that triangle and the camera.
#include "fr_kernels.h"
#include "fr_shade.h"

namespace fr {

constexpr uint32_t PURPOSE_SHADOW_EDGE = 0xC0000000u;
constexpr float kSePlane = 1e-5f;   // relative distance of a vertex to the wedge plane
constexpr float kSeW = 1e-5f;       // jump position at the ends of the line
constexpr float kSeSide = 1e-5f;    // a face's slice nearly along the ray from x

// Exact probability of floor(r n / 2^32) == i over the 2^32 values of r.
__device__ __forceinline__ double pick_prob(uint64_t i, uint64_t n) {
  const uint64_t hi = (((i + 1) << 32) + n - 1) / n, lo = ((i << 32) + n - 1) / n;
  return (double)(hi - lo) * (1.0 / 4294967296.0);
}

// FP64 vectors of the jumps' derivative chain: a jump's position and its
// dw1/dtheta are ill conditioned when x is far from the occluder edge or the
// edge nearly parallel to the line (1/D1); jumps are rare (under 1 % of the
// line samples at the face workload), so they are solved in FP64.
__device__ __forceinline__ D3 d3(V3 a) { return {(double)a.x, (double)a.y, (double)a.z}; }
__device__ __forceinline__ void fix_add3(fix_t* p, D3 v) { fix_add_d(p, v.x); fix_add_d(p + 1, v.y); fix_add_d(p + 2, v.z); }

template <bool DUMP, bool TEX>
__device__ __forceinline__ void shadow_edge_sample(const RenderArgs& a, const ShadowEdgeArgs& e, int i) {
  const int lane = lane_id();
  const bool valid = i < e.n_samples;
  // group of 64 samples (one wave): an 8 x 8 pixel tile and a light; per
  // sample a camera sample within the tile and a line across the light
  const U4 rg = philox((uint32_t)(i / 64), 0u, PURPOSE_SHADOW_EDGE, a.step, a.k0, a.k1);
  const U4 r = philox((uint32_t)i, 1u, PURPOSE_SHADOW_EDGE, a.step, a.k0, a.k1);
  const int tx = (a.W + 7) / 8, ty = (a.H + 7) / 8;
  const uint64_t n_t = (uint64_t)tx * ty;
  const int tile = (int)(((uint64_t)rg.x * n_t) >> 32);
  const int x0 = 8 * (tile % tx), y0p = 8 * (tile / tx);
  const int tw = min(8, a.W - x0), th = min(8, a.H - y0p);
  const uint64_t n_in = (uint64_t)tw * th * a.S;
  const uint64_t kin = ((uint64_t)r.x * n_in) >> 32;
  const int s = (int)(kin % a.S), q = (int)(kin / a.S);
  const int pid = (y0p + q / tw) * a.W + x0 + q % tw;
  const uint64_t cs = (uint64_t)pid * a.S + s;
  const int j = a.L > 0 ? (int)(((uint64_t)rg.y * (uint64_t)a.L) >> 32) : -1;
  const float v = unit24(r.y);
  PixelSample ps;
  ps.pid = pid; ps.px = pid % a.W; ps.py = pid / a.W; ps.s0 = 0; ps.valid = valid;
  bool amb = false;
  // camera ray and its shading frame, as in the render
  Sample sm;
  camera_sample(a, ps, s, sm);
  HitState h;
  h.t = 3.4e38f; h.id = -1; h.tamb = 3.4e38f;
  bool dummy = false;
  trace<false, DUMP>(a.nodes, a.recs, a.F, sm.ray, valid, -1, h, dummy);
  if (DUMP && valid && hit_ambiguous(h)) amb = true;
  Frame fr;
  double fx = 0.0, fy = 0.0;
  film_point(a, ps, s, fx, fy);
  bool shaded = valid && h.id >= 0 && shading_frame<TEX>(a, sm, h, fr, fx, fy);
  if (DUMP && valid && h.id >= 0 && fabsf(fr.cos_o) < kFlagCos) amb = true;
  LightRec Lj = load_const(a.lights, max(j, 0));
  shaded = shaded && j >= 0 && Lj.shape != FR_LIGHT_DIRECTIONAL;
  // a light wholly below x's tangent plane, or x behind the light's emitting
  // plane (by the render's cull margins), gives h = 0 on every line: no walk
  if (shaded) {
    const V3 d0 = {Lj.p0[0] - fr.x.x, Lj.p0[1] - fr.x.y, Lj.p0[2] - fr.x.z};
    const float ca = dot(fr.ns, d0);
    const float cb = fr.ns.x * Lj.e1[0] + fr.ns.y * Lj.e1[1] + fr.ns.z * Lj.e1[2];
    const float cc = fr.ns.x * Lj.e2[0] + fr.ns.y * Lj.e2[1] + fr.ns.z * Lj.e2[2];
    float top = fmaxf(ca, fmaxf(ca + cb, ca + cc));
    if (Lj.shape != FR_LIGHT_TRIANGLE) top = fmaxf(top, ca + cb + cc);
    const float side = Lj.na[0] * d0.x + Lj.na[1] * d0.y + Lj.na[2] * d0.z;
    const float alen = fabsf(Lj.na[0]) + fabsf(Lj.na[1]) + fabsf(Lj.na[2]);
    if (DUMP && (fabsf(top + 1e-4f) < 1e-5f || fabsf(side + 1e-3f * alen) < 1e-5f * (1.0f + alen))) amb = true;
    shaded = !(top < -1e-4f) && !(side < -1e-3f * alen);
  }
  // the wedge: x and the line y0 -> y1 = y0 + ell e1 on the light
  const V3 p0 = {Lj.p0[0], Lj.p0[1], Lj.p0[2]}, e1 = {Lj.e1[0], Lj.e1[1], Lj.e1[2]},
           e2 = {Lj.e2[0], Lj.e2[1], Lj.e2[2]};
  const float ell = Lj.shape == FR_LIGHT_TRIANGLE ? 1.0f - v : 1.0f;
  // x = fr.x + xlo: the FP32 shading point plus its residual against the
  // FP64 barycentric point, so that differences p - x with nearby points keep
  // the FP64 point's accuracy (a near occluder's jump moves ~|light| /
  // |occluder| times as fast as x)
  const V3 x = fr.x;
  V3 xlo = {0.0f, 0.0f, 0.0f};
  double bd[3] = {1.0, 0.0, 0.0};
  D3 Xd = {0.0, 0.0, 0.0};   // the FP64 barycentric point
  if (shaded) {
    const int* tv = a.tris + 3 * h.id;
    const int vi[3] = {tv[0], tv[1], tv[2]};
    bary64(a, fx, fy, vi, bd);
    double X[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 3; ++k)
      for (int c = 0; c < 3; ++c) X[c] += bd[k] * (double)a.verts[3 * vi[k] + c];
    xlo = {(float)(X[0] - (double)x.x), (float)(X[1] - (double)x.y), (float)(X[2] - (double)x.z)};
    Xd = {X[0], X[1], X[2]};
  }
  const auto rel = [&](V3 p) { return (p - x) - xlo; };
  const V3 y0 = p0 + e2 * v, y1 = y0 + e1 * ell;
  // (y0 - x) x (y1 - x) = (y0 - x) x (y1 - y0): the second form keeps the wedge's
  // normal free of the cancellation of two nearly parallel long vectors
  const V3 Nw = cross(rel(y0), e1 * ell);
  const float nN = sqrtf(dot(Nw, Nw));
  shaded = shaded && nN > 0.0f;
  const float pad = 1e-4f;
  const V3 blo = {fminf(x.x, fminf(y0.x, y1.x)) - pad, fminf(x.y, fminf(y0.y, y1.y)) - pad,
                  fminf(x.z, fminf(y0.z, y1.z)) - pad};
  const V3 bhi = {fmaxf(x.x, fmaxf(y0.x, y1.x)) + pad, fmaxf(x.y, fmaxf(y0.y, y1.y)) + pad,
                  fmaxf(x.z, fmaxf(y0.z, y1.z)) + pad};
  // outward in-plane normals of the wedge triangle's sides x -> y0 -> y1 -> x
  const V3 sn0 = cross(rel(y0), Nw), sn1 = cross(y1 - y0, Nw), sn2 = cross(rel(y1) * -1.0f, Nw);
  const float kinv = Lj.shape == FR_LIGHT_TRIANGLE ? 2.0f : 1.0f;
  const double wgt = valid && a.L > 0
                         ? 1.0 / ((double)e.n_samples * pick_prob((uint64_t)tile, n_t) * pick_prob(kin, n_in) *
                                  pick_prob((uint64_t)max(j, 0), (uint64_t)a.L))
                         : 0.0;
  const float* g = e.dEdp + 3 * (size_t)pid;
  const float gs = grad_scale(e.gmax);   // exact power of two; the conversions divide by it
  const V3 gpix = valid ? V3{g[0] * gs, g[1] * gs, g[2] * gs} : V3{0.0f, 0.0f, 0.0f};
  int n_ok = 0;
  long long key = 0;
  D3 gx_tot = {0.0, 0.0, 0.0};
  D3 gy_tot = {0.0, 0.0, 0.0}, ge1_tot = {0.0, 0.0, 0.0}, ge2_tot = {0.0, 0.0, 0.0};
  const auto near_plane = [&](float sv, V3 E) { return fabsf(sv) < kSePlane * nN * (1.0f + sqrtf(dot(rel(E), rel(E)))); };

  // ---- wave-cooperative walk of the tree with every lane's wedge
  uint64_t live = ballot(shaded);
  int stack = 0, sp = 0;
  int node = a.F > 1 ? 0 : ~0;
  int budget = 2 * a.F + 64;
  while (live != 0 && --budget > 0) {
    if (node >= 0) {
      const Bvh4Node nd = load_const(a.nodes, node);
      uint64_t mk[4];
      for (int k = 0; k < 4; ++k) {
        const V3 lo = {nd.lo[0][k], nd.lo[1][k], nd.lo[2][k]}, hi = {nd.hi[0][k], nd.hi[1][k], nd.hi[2][k]};
        const V3 c = (lo + hi) * 0.5f, ex = (hi - lo) * 0.5f;
        const float dc = dot(Nw, rel(c));
        const float rad = fabsf(Nw.x) * ex.x + fabsf(Nw.y) * ex.y + fabsf(Nw.z) * ex.z;
        const bool straddle = fabsf(dc) <= rad * 1.0001f + 2.0f * kSePlane * nN * (1.0f + sqrtf(dot(rel(c), rel(c))) + rad / fmaxf(nN, 1e-30f));
        const bool overlap = !(hi.x < blo.x || lo.x > bhi.x || hi.y < blo.y || lo.y > bhi.y || hi.z < blo.z ||
                               lo.z > bhi.z);
        // a side's normal separates the box from the triangle when the whole
        // box lies beyond that side (with a relative margin)
        const auto beyond = [&](V3 m, V3 p) {
          const float r = fabsf(m.x) * ex.x + fabsf(m.y) * ex.y + fabsf(m.z) * ex.z;
          return dot(m, c - p) - r > 1e-4f * (r + sqrtf(dot(m, m)) * (1.0f + sqrtf(dot(c - p, c - p))));
        };
        const bool inside = !beyond(sn0, x) && !beyond(sn1, y0) && !beyond(sn2, y1);
        mk[k] = nd.c[k] != kEmpty ? (ballot(shaded && straddle && overlap && inside) & live) : 0ull;
      }
      int next = kEmpty;
      for (int k = 3; k >= 0; --k) {
        if (!mk[k]) continue;
        if (next != kEmpty) { stack = (lane == sp) ? next : stack; ++sp; }
        next = nd.c[k];
      }
      if (next != kEmpty) { node = next; continue; }
    } else {
      const TriRec tr = load_const(a.recs, ~node);
      const int f = tr.id;
      for (int k = 0; k < 3; ++k) {
        int ia = a.tris[3 * f + k], ib = a.tris[3 * f + (k + 1) % 3];
        const int ic = a.tris[3 * f + (k + 2) % 3];
        const int nb = e.nbr[3 * f + k];
        V3 A = {tr.v[3 * k], tr.v[3 * k + 1], tr.v[3 * k + 2]};
        V3 B = {tr.v[3 * ((k + 1) % 3)], tr.v[3 * ((k + 1) % 3) + 1], tr.v[3 * ((k + 1) % 3) + 2]};
        const V3 C = {tr.v[3 * ((k + 2) % 3)], tr.v[3 * ((k + 2) % 3) + 1], tr.v[3 * ((k + 2) % 3) + 2]};
        if (ia > ib) { const int t = ia; ia = ib; ib = t; const V3 tv = A; A = B; B = tv; }
        const bool lead = nb < 0 || f < nb;
        const float sa = dot(Nw, rel(A)), sb = dot(Nw, rel(B));
        if (DUMP && shaded && lead && (near_plane(sa, A) || near_plane(sb, B))) {
          // an end on the plane matters when it lies inside the wedge's span
          const V3 E = near_plane(sa, A) ? A : B, u0 = rel(y0), u1 = rel(y1), w = rel(E);
          const float g00 = dot(u0, u0), g01 = dot(u0, u1), g11 = dot(u1, u1), r0 = dot(u0, w), r1 = dot(u1, w);
          const float det = g00 * g11 - g01 * g01;
          const float al = (g11 * r0 - g01 * r1) / det, be = (g00 * r1 - g01 * r0) / det, tot = al + be;
          if (tot > -0.01f && be > -0.02f * fabsf(tot) && be < 1.02f * fabsf(tot) && tot < 1.02f) amb = true;
        }
        bool cand = shaded && lead && ((sa > 0.0f && sb < 0.0f) || (sa < 0.0f && sb > 0.0f));
        V3 P = {0.0f, 0.0f, 0.0f}, nab = {0.0f, 0.0f, 0.0f}, yk = {0.0f, 0.0f, 0.0f};
        float w1 = 0.0f, D1 = 1.0f, dist = 1.0f;
        int J = 0;
        if (cand) {
          P = A + (B - A) * (sa / (sa - sb));
          // (A - x) x (B - x) = (A - x) x (B - A): an edge far from x makes the two
          // x-relative vectors nearly parallel, and 1 / D1 would amplify their
          // product's cancellation
          nab = cross(rel(A), B - A);
          D1 = dot(nab, e1);
          w1 = D1 != 0.0f ? -dot(nab, rel(y0)) / D1 : -1.0f;
          yk = p0 + e1 * w1 + e2 * v;
          const V3 dy = rel(yk);
          dist = sqrtf(dot(dy, dy));
          const float tau = dot(rel(P), dy) / (dist * dist);
          const float dP = tau * dist;
          const bool in_w = w1 > 0.0f && w1 < ell, in_t = tau > 0.0f && dP > kShadowTmin && tau < 1.0f;
          if (DUMP && tau > 0.0f &&
              (fabsf(w1) < kSeW || fabsf(w1 - ell) < kSeW || fabsf(dP - kShadowTmin) < kFlagT || fabsf(dist - dP) < kFlagT))
            amb = true;
          cand = in_w && in_t;
          if (cand && DUMP && (near_plane(sa, A) || near_plane(sb, B))) amb = true;
          // an edge nearly parallel to the line: ill-conditioned position
          if (cand && DUMP && fabsf(D1) < 2e-3f * sqrtf(dot(nab, nab)) * sqrtf(dot(e1, e1))) amb = true;
        }
        if (cand) {
          // faces of the edge other than x's own triangle, and their sides
          int n = 0, right = 0;
          for (int q = 0; q < 2; ++q) {
            const int fq = q == 0 ? f : nb;
            if (fq < 0 || fq == h.id) continue;
            V3 Cq = C;
            if (q == 1) {
              const int* t = a.tris + 3 * fq;
              const int cv = (t[0] != ia && t[0] != ib) ? t[0] : ((t[1] != ia && t[1] != ib) ? t[1] : t[2]);
              Cq = ld3(a.verts, cv);
            } else {
              (void)ic;
            }
            const float scq = dot(Nw, rel(Cq));
            if (DUMP && near_plane(scq, Cq)) amb = true;
            const bool with_a = (scq > 0.0f) == (sa > 0.0f);
            const V3 Q = with_a ? B + (Cq - B) * (sb / (sb - scq)) : A + (Cq - A) * (sa / (sa - scq));
            const float o = dot(cross(rel(P), rel(Q)), Nw);
            if (DUMP && fabsf(o) < kSeSide * sqrtf(dot(rel(P), rel(P))) * sqrtf(dot(Q - P, Q - P)) * nN) amb = true;
            ++n;
            right += o > 0.0f ? 1 : 0;
          }
          J = (n == 0 || (right != 0 && right != n)) ? 0 : (right == n ? 1 : -1);
          cand = J != 0;
        }
        // the shadow ray to the jump's light point, the edge's faces and x's triangle excluded
        Ray sr;
        sr.o = x;
        sr.d = rel(yk) * (1.0f / dist);
        sr.tmin = kShadowTmin;
        sr.tmax = dist;
        ray_setup(sr);
        HitState shd;
        shd.tamb = 3.4e38f;
        bool occ = false;
        trace<true, DUMP, true>(a.nodes, a.recs, a.F, sr, cand, h.id, shd, occ, nullptr, f, nb);
        if (DUMP && cand && shd.tamb < 3.0e38f) amb = true;
        cand = cand && !occ;
        if (cand) {
          ++n_ok;
          key = (key + (long long)ia * a.N + ib) % 2147483648LL;
          // h at the jump: the render's light value there (cosine culls included)
          LightSample ls;
          ls.w1 = w1; ls.w2 = v; ls.q = yk;
          const V3 dq = rel(yk);
          ls.dist2 = dot(dq, dq);
          ls.dist = sqrtf(ls.dist2);
          ls.l = dq * (1.0f / ls.dist);
          ls.cos_s = dot(fr.ns, ls.l);
          ls.cos_a = Lj.na[0] * ls.l.x + Lj.na[1] * ls.l.y + Lj.na[2] * ls.l.z;
          ls.geom = ls.cos_s * ls.cos_a / ls.dist2;
          const float alen = sqrtf(Lj.na[0] * Lj.na[0] + Lj.na[1] * Lj.na[1] + Lj.na[2] * Lj.na[2]);
          if (DUMP && (fabsf(ls.cos_s) < kFlagCos || fabsf(ls.cos_a) < kFlagCos * alen)) amb = true;
          if (ls.cos_s > 0.0f && ls.cos_a > 0.0f) {
            float fv[3], gflag = 0.0f;
            brdf_eval<DUMP>(a.variant, a.components, fr, ls, fv, gflag);
            if (DUMP && gflag != 0.0f) amb = true;
            const float hv = gpix.x * fv[0] * Lj.rad[0] + gpix.y * fv[1] * Lj.rad[1] + gpix.z * fv[2] * Lj.rad[2];
            const double coef = wgt * (double)kinv / (double)a.S * (double)J * (double)hv * (double)ls.geom;
            if (coef != 0.0) {
              // the jump again in FP64: D(w1) = det[A - x, B - x, y(w1) - x] = (A - x) x (B - A) . (y(w1) - x)
              const D3 Ad = d3(A), Bd = d3(B), e1d = d3(e1), e2d = d3(e2);
              const D3 nabd = crossd(Ad - Xd, Bd - Ad);
              const double D1d = dotd(nabd, e1d);
              const D3 y0d = d3(p0) + e2d * (double)v;
              const double w1d = -dotd(nabd, y0d - Xd) / D1d;
              const D3 Yd = y0d + e1d * w1d;
              const double c = -coef / D1d;
              // dw1/dtheta = -(dD/dtheta) / (dD/dw1); dD/dx = -(dD/da + dD/db + dD/dy) by
              // translation invariance, and Bx x Yx + Yx x Ax + Ax x Bx = (B - A) x (Y - A)
              const D3 ga = crossd(Bd - Xd, Yd - Xd) * c, gb = crossd(Yd - Xd, Ad - Xd) * c, gy = nabd * c;
              gx_tot = gx_tot - crossd(Bd - Ad, Yd - Ad) * c;
              gy_tot = gy_tot + gy;
              ge1_tot = ge1_tot + gy * w1d;
              ge2_tot = ge2_tot + gy * (double)v;
              if (e.gverts) {
                fix_add3(e.gverts + 3 * ia, ga);
                fix_add3(e.gverts + 3 * ib, gb);
              }
            }
          }
        }
      }
    }
    if (sp == 0) break;
    --sp;
    node = readlane_i(stack, sp);
  }

  // ---- light geometry, and x's path to its triangle and the camera (FP64:
  // x = o + t d, t = (v0 - o) . n / (d . n), d = R dc / |R dc|, o = T)
  const bool has = gy_tot.x != 0.0 || gy_tot.y != 0.0 || gy_tot.z != 0.0 || gx_tot.x != 0.0 || gx_tot.y != 0.0 ||
                   gx_tot.z != 0.0;
  if (has) {
    if (e.glight) {
      fix_t* gl = e.glight + 9 * (size_t)j;
      fix_add3(gl, gy_tot);
      fix_add3(gl + 3, ge1_tot);
      fix_add3(gl + 6, ge2_tot);
    }
    const int* tv = a.tris + 3 * h.id;
    const D3 v0 = d3(ld3(a.verts, tv[0])), v1 = d3(ld3(a.verts, tv[1])), v2 = d3(ld3(a.verts, tv[2]));
    const float* R = a.cam;
    const D3 dc = {(2.0 * fx / (double)a.W - 1.0) * a.tan_half_d * a.aspect_d, (1.0 - 2.0 * fy / (double)a.H) * a.tan_half_d,
                   -1.0};
    const D3 dw = {R[0] * dc.x + R[1] * dc.y + R[2] * dc.z, R[3] * dc.x + R[4] * dc.y + R[5] * dc.z,
                   R[6] * dc.x + R[7] * dc.y + R[8] * dc.z};
    const double inv_len = 1.0 / sqrt(dotd(dw, dw));
    const D3 d = dw * inv_len, o = {(double)R[9], (double)R[10], (double)R[11]};
    const D3 ea = v1 - v0, eb = v2 - v0;
    const D3 n = crossd(ea, eb);
    const double idn = 1.0 / dotd(d, n);
    const double t = dotd(v0 - o, n) * idn;
    const double g_t = dotd(gx_tot, d);
    const D3 go = gx_tot - n * (g_t * idn);
    const D3 gd = gx_tot * t - n * (g_t * t * idn);
    // v0 - x = -(b1 ea + b2 eb) from the FP64 barycentrics of the shading point
    const D3 gn = (ea * bd[1] + eb * bd[2]) * (-g_t * idn);
    const D3 gea = crossd(eb, gn), geb = crossd(gn, ea);
    const D3 gv0 = n * (g_t * idn) - gea - geb;
    if (e.gverts) {
      fix_add3(e.gverts + 3 * tv[0], gv0);
      fix_add3(e.gverts + 3 * tv[1], gea);
      fix_add3(e.gverts + 3 * tv[2], geb);
    }
    if (e.gcam) {
      // d = dw / |dw|, dw = R dc
      const D3 gdw = (gd - d * dotd(gd, d)) * inv_len;
      const double gdv[3] = {gdw.x, gdw.y, gdw.z}, dcv[3] = {dc.x, dc.y, dc.z};
      for (int r = 0; r < 3; ++r)
        for (int q2 = 0; q2 < 3; ++q2) fix_add_d(e.gcam + 3 * r + q2, gdv[r] * dcv[q2]);
      fix_add3(e.gcam + 9, go);
    }
  }
  if (DUMP && valid) {
    e.dbg_rec[4 * (size_t)i] = (int32_t)cs;
    e.dbg_rec[4 * (size_t)i + 1] = j;
    e.dbg_rec[4 * (size_t)i + 2] = n_ok;
    e.dbg_rec[4 * (size_t)i + 3] = (int32_t)key;
    e.dbg_flag[i] = amb ? 1 : 0;
  }
}

template <bool DUMP, bool TEX>
__global__ __launch_bounds__(256) void k_shadow_edges(RenderArgs a, ShadowEdgeArgs e) {
  shadow_edge_sample<DUMP, TEX>(a, e, (int)(blockIdx.x * 256 + threadIdx.x));
}

void launch_shadow_edges(const RenderArgs& a, const ShadowEdgeArgs& e, hipStream_t st) {
  if (e.n_samples <= 0) return;
  const int blocks = (e.n_samples + 255) / 256;
  const bool dump = e.dbg_rec != nullptr, tex = a.M > 0;
  if (dump && tex) hipLaunchKernelGGL((k_shadow_edges<true, true>), dim3(blocks), dim3(256), 0, st, a, e);
  else if (dump) hipLaunchKernelGGL((k_shadow_edges<true, false>), dim3(blocks), dim3(256), 0, st, a, e);
  else if (tex) hipLaunchKernelGGL((k_shadow_edges<false, true>), dim3(blocks), dim3(256), 0, st, a, e);
  else hipLaunchKernelGGL((k_shadow_edges<false, false>), dim3(blocks), dim3(256), 0, st, a, e);
}

}  // namespace fr
