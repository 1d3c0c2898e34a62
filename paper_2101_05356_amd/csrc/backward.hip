// Fused backward of the render (the "back-propagation based gradients" of
// Sec. 4): for every pixel sample the primary hit and every shadow decision are
// recomputed from the same Philox counters (no stored ray paths), held fixed,
// and the hand-written reverse mode runs through the Cook-Torrance BRDF
// (Appendix A), the light sampling, the shading frame and the ray/triangle
// intersection, into
//   - per-vertex positions, normals, diffuse, specular, roughness: per-wave
//     match-reduce over lanes that hit the same triangle, then one set of
//     fixed-point atomics per distinct triangle;
//   - with reflectance maps, per-texel diffuse, specular, roughness: the same
//     match-reduce over lanes sharing a bilinear footprint;
//   - per-light geometry and radiance, and the camera: wave reduction,
//     fixed-point LDS accumulation per block, then fixed-point atomics into
//     one of kSlots partial slots, summed by a final kernel.
// All cross-wave sums are exact 64-bit integer sums (see fix_t), so the
// gradients do not depend on scheduling.
#include "fr_shade.h"

namespace fr {



__device__ __forceinline__ V3 project_out(V3 g, V3 u, float inv_len) {
  // adjoint of u = w / |w|: (g - u (u . g)) / |w|
  const float d = dot(u, g);
  return (g - u * d) * inv_len;
}

__device__ __forceinline__ void g1_fwd_bwd(float nv, float hv, float r, float& G1, float& dG1_dnv, float& dG1_dr) {
  dG1_dnv = 0.0f;
  dG1_dr = 0.0f;
  if (!(hv * nv > 0.0f)) { G1 = 0.0f; return; }   // h.v / n.v > 0: the same sign
  const float s2 = 1.0f - nv * nv;
  if (s2 <= 0.0f) { G1 = 1.0f; return; }
  const float irs = rsqrt_hw(s2), ir = rcp_hw(r);
  const float a = nv * irs * ir;
  if (!(a < 1.6f)) { G1 = 1.0f; return; }
  const float P = 3.535f * a + 2.181f * a * a, Q = 1.0f + 2.276f * a + 2.577f * a * a;
  const float iQ = rcp_hw(Q);
  G1 = P * iQ;
  const float dP = 3.535f + 4.362f * a, dQ = 2.276f + 5.154f * a;
  const float dG = (dP * Q - P * dQ) * iQ * iQ;
  dG1_dnv = dG * ir * irs * irs * irs;   // da/dnv = (1 - nv^2)^(-3/2) / r
  dG1_dr = -dG * a * ir;                 // da/dr = -a / r
}

// The shadow decisions of lights [j0, j1) (global indices) for sample rs,
// read from the masks the forward kept (its chunks of vis_lc lights need not
// align with these):
// the same bits shadow_mask returns, since a lane's bit depends on its own
// shading point, light draw and ray only.  Zero where the adjoint does not
// shade the sample.
__device__ __forceinline__ uint32_t kept_mask(const RenderArgs& a, int j0, int j1, size_t rs, bool shaded) {
  if (!shaded || j1 <= j0) return 0u;
  const size_t ns = (size_t)a.W * a.H * a.S;
  uint32_t m = 0u;
  for (int c = j0 / a.vis_lc; c * a.vis_lc < j1; ++c) {
    const uint32_t w = a.vis_in[(size_t)c * ns + rs];
    const int sh = c * a.vis_lc - j0;          // in (-vis_lc, j1 - j0): |sh| <= 31
    m |= sh >= 0 ? (w << sh) : (w >> -sh);
  }
  return j1 - j0 >= 32 ? m : (m & ((1u << (j1 - j0)) - 1u));
}

// KEPT: the shadow decisions come from the forward's masks (a.vis_in), and
// the kernel holds no traversal code at all.
template <bool TEX, bool KEPT>
__device__ __forceinline__ void render_bwd_block(const RenderArgs& a, const float* __restrict__ dEdp,
                                                 const FixGrads& g, fix_t* __restrict__ slots, int bid) {
  // LDS: [L*12 + 12] fixed-point sums (per light p0 e1 e2 rad, then camera),
  // then the per-lane sample adjoints of the block's four waves [4][64][16]
  extern __shared__ fix_t lds[];
  const int nl = a.L * 12 + 12 + 3 * a.sh_bands * a.sh_bands;
  float* part = reinterpret_cast<float*>(lds + nl);
  int* arrived = reinterpret_cast<int*>(part + 4 * 64 * 16);
  for (int i = threadIdx.x; i < nl; i += 256) lds[i] = 0;
  if (threadIdx.x == 0) *arrived = 0;
  __syncthreads();
  // one block = one tile; wave wv takes the tile's light chunk wv (at most
  // four chunks: the host sets lc >= L/4), so the sample-level work below
  // runs once per sample instead of once per chunk
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tile = block_tile(a, bid);
  const int j0 = wv * a.lc, j1 = min(a.L, j0 + a.lc);
  if (tile >= 0) {
    const PixelSample ps = pixel_sample(a, tile, lane);
    float gbar[3] = {0.0f, 0.0f, 0.0f};
    if (ps.valid) {
      const float inv = grad_scale(a.gmax) / (float)a.S;   // s a power of two: exactly s times 1 / S
      gbar[0] = dEdp[3 * ps.pid] * inv; gbar[1] = dEdp[3 * ps.pid + 1] * inv; gbar[2] = dEdp[3 * ps.pid + 2] * inv;
    }
    const bool want = ps.valid && (gbar[0] != 0.0f || gbar[1] != 0.0f || gbar[2] != 0.0f);
    for (int chunk = 0; chunk < a.chunks; ++chunk) {
      const int s = ps.s0 + chunk * 64;
      const size_t rs = (size_t)ps.pid * a.S + s;
      double bd0[3] = {1.0, 0.0, 0.0};
      PrimHit ph = {-1, 0.0f, 0.0, 0.0};
      if (want) ph = load_prim(a, rs, bd0);
      // the camera ray (for the view direction) only where a sample has a shading point
      Sample sm;
      if (ballot(want && ph.id >= 0)) camera_sample(a, ps, s, sm);
      Frame fr = {};
      const bool shaded = want && ph.id >= 0 && shading_frame<TEX>(a, sm, ph.id, ph.t, bd0, fr);
      // sample-level adjoint accumulators
      V3 gx = {0, 0, 0}, gns = {0, 0, 0}, gwo = {0, 0, 0}, gc = {0, 0, 0}, gs = {0, 0, 0};
      float gr = 0.0f;
      // shadow decisions of every light of the chunk, then the adjoint of the visible ones
      const auto draw = [&](int j) { return philox((uint32_t)ps.pid, (uint32_t)s, 1u + (uint32_t)(a.light0 + j), a.step, a.k0, a.k1); };
      const auto none = [](int, bool, bool, const LightSample&, const HitState&) {};
      const auto skip = [](int) {};
      uint32_t vmask;
      if (KEPT) vmask = kept_mask(a, a.light0 + j0, a.light0 + j1, rs, shaded);
      else vmask = shadow_mask<false>(a, j0, j1, shaded, fr, ph.id, draw, none, skip, nullptr);
      for (int j = j0; j < j1; ++j) {
        const bool vis = (vmask >> (j - j0)) & 1u;
        if (!ballot(vis)) continue;
        const LightRec Lj = load_const(a.lights, j);
        const U4 r = Lj.shape == FR_LIGHT_DIRECTIONAL ? U4{0u, 0u, 0u, 0u} : draw(j);
        LightSample ls;
        light_point(Lj, unit24(r.x), unit24(r.y), fr, ls);
        float gl12[12];
        for (int k = 0; k < 12; ++k) gl12[k] = 0.0f;
        if (vis) {
          const V3 rad = {Lj.rad[0], Lj.rad[1], Lj.rad[2]};
          const V3 na = {Lj.na[0], Lj.na[1], Lj.na[2]};
          // ---- forward values of the BRDF
          V3 f = {0, 0, 0};
          if (a.components & 1) f = fr.c * (1.0f / kPi);
          V3 hraw = ls.l + fr.wo;
          const float ih = rsqrt_hw(dot(hraw, hraw));
          const V3 hv = hraw * ih;
          float nh = 0, ex = 0, nd = 0, D = 0, oh = 0, G1o = 0, G1l = 0, dG1o = 0, dG1l = 0, dG1o_r = 0, dG1l_r = 0;
          float lg2nh = 0, ir = 0, iden = 0;
          float om = 0, fw = 0, spec = 0;
          V3 Fv = {0, 0, 0};
          const bool do_spec = (a.components & 2) != 0;
          if (do_spec) {
            nh = dot(fr.ns, hv);   // > 0: n.l > 0 and n.o > 0 here
            ir = rcp_hw(fr.r);
            ex = 2.0f * ir - 2.0f;
            nd = a.variant == FR_BRDF_NORMALIZED ? ir * (1.0f / kPi) : (2.0f * ir + 2.0f) * (1.0f / (2.0f * kPi));
            lg2nh = log2_hw(nh);
            D = nd * exp2_hw(ex * lg2nh);
            oh = dot(fr.wo, hv);
            const float lh = dot(ls.l, hv);
            g1_fwd_bwd(fr.cos_o, oh, fr.r, G1o, dG1o, dG1o_r);
            g1_fwd_bwd(ls.cos_s, lh, fr.r, G1l, dG1l, dG1l_r);
            om = 1.0f - oh;
            fw = a.variant == FR_BRDF_NORMALIZED ? om * om * om * om * om : om;
            iden = rcp_hw(4.0f * fr.cos_o * ls.cos_s);
            spec = D * G1o * G1l * iden;
            Fv = {fr.s.x + (1.0f - fr.s.x) * fw, fr.s.y + (1.0f - fr.s.y) * fw, fr.s.z + (1.0f - fr.s.z) * fw};
            f = f + V3{Fv.x * spec, Fv.y * spec, Fv.z * spec};
          }
          // ---- C = rad * f * geom
          gl12[9] = gbar[0] * f.x * ls.geom;
          gl12[10] = gbar[1] * f.y * ls.geom;
          gl12[11] = gbar[2] * f.z * ls.geom;
          const V3 gf = {gbar[0] * rad.x * ls.geom, gbar[1] * rad.y * ls.geom, gbar[2] * rad.z * ls.geom};
          const float ggeom = gbar[0] * rad.x * f.x + gbar[1] * rad.y * f.y + gbar[2] * rad.z * f.z;
          if (a.components & 1) gc = gc + gf * (1.0f / kPi);
          float gcos_o = 0.0f, gcos_s = 0.0f;
          V3 gl = {0, 0, 0};
          if (do_spec) {
            const float gspec = dot(gf, Fv);
            const V3 gF = gf * spec;
            gs = gs + V3{gF.x * (1.0f - fw), gF.y * (1.0f - fw), gF.z * (1.0f - fw)};
            const float gfw = gF.x * (1.0f - fr.s.x) + gF.y * (1.0f - fr.s.y) + gF.z * (1.0f - fr.s.z);
            const float gom = a.variant == FR_BRDF_NORMALIZED ? gfw * 5.0f * om * om * om * om : gfw;
            float goh = -gom;
            const float gD = gspec * G1o * G1l * iden;
            const float gG1o = gspec * D * G1l * iden, gG1l = gspec * D * G1o * iden;
            gcos_o -= gspec * spec * rcp_hw(fr.cos_o);
            gcos_s -= gspec * spec * rcp_hw(ls.cos_s);
            gcos_o += gG1o * dG1o;
            gcos_s += gG1l * dG1l;
            gr += gG1o * dG1o_r + gG1l * dG1l_r;
            // D = nd * nh^ex
            const float gnh = gD * D * ex * rcp_hw(nh);
            const float dlnnd = a.variant == FR_BRDF_NORMALIZED ? -ir : -ir * rcp_hw(1.0f + fr.r);
            // d ln D / dr = dln nd/dr - 2 ln(nh) / r^2 (ln = log2 ln 2)
            gr += gD * D * (dlnnd - 2.0f * 0.69314718f * lg2nh * ir * ir);
            // nh = ns . h, oh = wo . h, h = normalize(l + wo)
            const V3 gh = fr.ns * gnh + fr.wo * goh;
            gns = gns + hv * gnh;
            gwo = gwo + hv * goh;
            const V3 ghraw = project_out(gh, hv, ih);
            gl = gl + ghraw;
            gwo = gwo + ghraw;
          }
          // geom = cos_s cos_a / dist2
          const float id2 = rcp_hw(ls.dist2);
          gcos_s += ggeom * ls.cos_a * id2;
          const float gcos_a = ggeom * ls.cos_s * id2;
          const float gdist2 = -ggeom * ls.geom * id2;
          // cos_o = ns . wo ; cos_s = ns . l ; cos_a = na . l
          gns = gns + fr.wo * gcos_o + ls.l * gcos_s;
          gwo = gwo + fr.ns * gcos_o;
          if (Lj.shape == FR_LIGHT_DIRECTIONAL) {
            // light at infinity: geom = cos_s, l = p0 / |p0| (no point, no
            // dependence on x); the direction's gradient goes to p0
            gl = gl + fr.ns * gcos_s;
            const V3 gp = project_out(gl, ls.l, Lj.e1[0]);
            gl12[0] = gp.x; gl12[1] = gp.y; gl12[2] = gp.z;
          } else {
            gl = gl + fr.ns * gcos_s + na * gcos_a;
            const V3 gna = ls.l * gcos_a;
            // na = -kappa (e1 x e2)
            const float kap = Lj.shape == FR_LIGHT_TRIANGLE ? 0.5f : 1.0f;
            const V3 e1 = {Lj.e1[0], Lj.e1[1], Lj.e1[2]}, e2 = {Lj.e2[0], Lj.e2[1], Lj.e2[2]};
            const V3 ge1n = cross(e2, gna) * (-kap), ge2n = cross(gna, e1) * (-kap);
            // l = dq / |dq|, dist2 = dq . dq
            V3 gdq = project_out(gl, ls.l, rcp_hw(ls.dist));
            gdq = gdq + (ls.q - fr.x) * (2.0f * gdist2);
            gx = gx - gdq;
            // q = p0 + w1 e1 + w2 e2
            gl12[0] = gdq.x; gl12[1] = gdq.y; gl12[2] = gdq.z;
            gl12[3] = gdq.x * ls.w1 + ge1n.x; gl12[4] = gdq.y * ls.w1 + ge1n.y; gl12[5] = gdq.z * ls.w1 + ge1n.z;
            gl12[6] = gdq.x * ls.w2 + ge2n.x; gl12[7] = gdq.y * ls.w2 + ge2n.y; gl12[8] = gdq.z * ls.w2 + ge2n.z;
          }
        }
        for (int k = 0; k < 12; ++k) {
          const float t = wave_sum(gl12[k]);
          if (lane == 0 && t != 0.0f) atomicAdd(&lds[12 * j + k], to_fix(t));
        }
      }
      // The SH light (first light chunk of the first light group only):
      // dE/dc = gbar E / pi, dE/dn_s = sum_ch (gbar c / pi)_ch grad E_ch, and
      // the coefficients' gradient (gbar c / pi) A_l Y_lm into the LDS sums.
      if (a.sh_bands > 0 && wv == 0 && (a.components & 1)) {
        const V3 n = shaded ? fr.ns : V3{0.0f, 0.0f, 1.0f};
        const float w0 = shaded ? gbar[0] * fr.c.x * (1.0f / kPi) : 0.0f;
        const float w1 = shaded ? gbar[1] * fr.c.y * (1.0f / kPi) : 0.0f;
        const float w2 = shaded ? gbar[2] * fr.c.z * (1.0f / kPi) : 0.0f;
        V3 e = {0.0f, 0.0f, 0.0f}, gn = {0.0f, 0.0f, 0.0f};
        fix_t* lsh = lds + 12 * a.L + 12;
        sh_stream(a, n, [&](int i, int l, G4 y) {
          const float A = a.sh_ash[l];
          const float c0 = a.sh[3 * i], c1 = a.sh[3 * i + 1], c2 = a.sh[3 * i + 2];
          e.x += A * y.v * c0; e.y += A * y.v * c1; e.z += A * y.v * c2;
          const float q = A * (w0 * c0 + w1 * c1 + w2 * c2);
          gn = gn + V3{y.dx, y.dy, y.dz} * q;
          const float t0 = wave_sum(w0 * A * y.v), t1 = wave_sum(w1 * A * y.v), t2 = wave_sum(w2 * A * y.v);
          if (lane == 0) {
            if (t0 != 0.0f) atomicAdd(&lsh[3 * i], to_fix(t0));
            if (t1 != 0.0f) atomicAdd(&lsh[3 * i + 1], to_fix(t1));
            if (t2 != 0.0f) atomicAdd(&lsh[3 * i + 2], to_fix(t2));
          }
        });
        if (shaded) {
          gc = gc + V3{gbar[0] * e.x, gbar[1] * e.y, gbar[2] * e.z} * (1.0f / kPi);
          gns = gns + gn;
        }
      }
      // The chunks' sample adjoints meet in LDS; one wave sums them in chunk
      // order and runs the sample-level chain and scatters once per sample:
      // with one sample round per tile, the last wave to arrive (no block
      // barrier: the others leave at once); otherwise wave 0 after a barrier.
      {
        float* p = part + (size_t)(wv * 64 + lane) * 16;
        p[0] = gx.x; p[1] = gx.y; p[2] = gx.z; p[3] = gns.x; p[4] = gns.y; p[5] = gns.z;
        p[6] = gwo.x; p[7] = gwo.y; p[8] = gwo.z; p[9] = gc.x; p[10] = gc.y; p[11] = gc.z;
        p[12] = gs.x; p[13] = gs.y; p[14] = gs.z; p[15] = gr;
      }
      bool run;
      if (a.chunks == 1) {
        __threadfence_block();   // this wave's partials and LDS sums before its arrival
        int n = 0;
        if (lane == 0) n = atomicAdd(arrived, 1);
        run = __builtin_amdgcn_readlane(n, 0) == 3;
        __threadfence_block();
      } else {
        __syncthreads();
        run = wv == 0;
      }
      if (run) {
        gx = gns = gwo = gc = gs = V3{0.0f, 0.0f, 0.0f};
        gr = 0.0f;
        for (int k = 0; k < a.n_lchunks; ++k) {
          const float* p = part + (size_t)(k * 64 + lane) * 16;
          gx = gx + V3{p[0], p[1], p[2]}; gns = gns + V3{p[3], p[4], p[5]}; gwo = gwo + V3{p[6], p[7], p[8]};
          gc = gc + V3{p[9], p[10], p[11]}; gs = gs + V3{p[12], p[13], p[14]}; gr += p[15];
        }
        // ---- sample-level adjoint: shading frame, intersection, camera
        V3 gv[3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, gn[3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        float gb[3] = {0.0f, 0.0f, 0.0f};
        // lanes whose chunk of lights left no gradient skip the chain and the scatter
        const bool has_g = shaded && (gx.x != 0.0f || gx.y != 0.0f || gx.z != 0.0f || gns.x != 0.0f ||
                                      gns.y != 0.0f || gns.z != 0.0f || gwo.x != 0.0f || gwo.y != 0.0f ||
                                      gwo.z != 0.0f || gc.x != 0.0f || gc.y != 0.0f || gc.z != 0.0f ||
                                      gs.x != 0.0f || gs.y != 0.0f || gs.z != 0.0f || gr != 0.0f);
        TexTap tp = {0, 0, 0, 0, 0.0f, 0.0f};
        // camera gradient of this chunk (reduced at its end, so that no
        // accumulator stays live through the traversals)
        float gcam[12];
        for (int k = 0; k < 12; ++k) gcam[k] = 0.0f;
        float bb[3] = {0.0f, 0.0f, 0.0f};
        if (has_g) {
          // the primary hit and the triangle's corners again, rather than kept
          // live through the light loop (the empty asm keeps the compiler from
          // reusing the earlier loads)
          size_t rs2 = rs;
          asm volatile("" : "+v"(rs2));
          double bd[3];
          const PrimHit ph2 = load_prim(a, rs2, bd);
          const int id = ph2.id;
          int vi[3];
          for (int k = 0; k < 3; ++k) vi[k] = a.tris[3 * id + k];
          for (int k = 0; k < 3; ++k) bb[k] = (float)bd[k];
          const float grr = fr.r_free ? gr : 0.0f;
          const V3 gm = project_out(gns, fr.ns, fr.inv_m);
          V3 vv[3];
          for (int k = 0; k < 3; ++k) {
            vv[k] = ld3(a.verts, vi[k]);
            const V3 nk = ld3(a.normals, vi[k]);
            if (TEX) {
              gb[k] = dot(nk, gm) + dot(vv[k], gx);
            } else {
              const V3 ck = ld3(a.diffuse, vi[k]), sk = ld3(a.specular, vi[k]);
              const float rk = a.roughness[vi[k]];
              gb[k] = dot(nk, gm) + dot(vv[k], gx) + dot(ck, gc) + dot(sk, gs) + rk * grr;
            }
            gn[k] = gm * bb[k];
            gv[k] = gx * bb[k];
          }
          if (TEX) {
            // reflectance = bilinear read at (u, v) = sum_k b_k uv_k: its slope
            // in (u, v) (d fx / du = M inside a cell) goes to the b_k
            tp = tex_tap(a, id, bd);
            const auto proj = [&](int t) {
              return dot(ld3(a.tex_c, t), gc) + dot(ld3(a.tex_s, t), gs) + a.tex_r[t] * grr;
            };
            const float P00 = proj(tp.t00), P10 = proj(tp.t10), P01 = proj(tp.t01), P11 = proj(tp.t11);
            const float Mf = (float)a.M;
            const float gu = Mf * ((1.0f - tp.fy) * (P10 - P00) + tp.fy * (P11 - P01));
            const float gvv = Mf * ((1.0f - tp.fx) * (P01 - P00) + tp.fx * (P11 - P10));
            const float* q = a.uv + 6 * id;
            for (int k = 0; k < 3; ++k) gb[k] += gu * q[2 * k] + gvv * q[2 * k + 1];
          }
          // b0 = 1 - b1 - b2; Moller-Trumbore adjoint of (b1, b2), solved from
          // the crossing point o' = o + t d itself (t = hit distance, held
          // fixed: g_o += g_o', g_d += t g_o'), placed by the FP64 barycentrics:
          // sv = o' - v0 = b1 e1 + b2 e2, qv = sv x e1.  An FP32 o' would carry
          // ~ulp(|o|) of error into sv, inconsistent with those barycentrics.
          const float g1 = gb[1] - gb[0], g2 = gb[2] - gb[0];
          const V3 d = sm.ray.d;
          const V3 e1 = vv[1] - vv[0], e2 = vv[2] - vv[0];
          const V3 pv = cross(d, e2);
          const float idet = 1.0f / dot(e1, pv);
          const float b1 = bb[1], b2 = bb[2];
          const V3 sv = e1 * b1 + e2 * b2;
          const V3 qv = cross(sv, e1);
          const float gA1 = g1 * idet, gA2 = g2 * idet, gdet = -(g1 * b1 + g2 * b2) * idet;
          V3 gsv = pv * gA1, gp = sv * gA1;
          V3 gd = qv * gA2 - gwo;
          const V3 gq = d * gA2;
          V3 ge1 = pv * gdet;
          gp = gp + e1 * gdet;
          gsv = gsv + cross(e1, gq);
          ge1 = ge1 + cross(gq, sv);
          gd = gd + cross(e2, gp);
          const V3 ge2 = cross(gp, d);
          gv[0] = gv[0] - gsv - ge1 - ge2;
          gv[1] = gv[1] + ge1;
          gv[2] = gv[2] + ge2;
          gd = gd + gsv * ph2.t;
          // d = dw / |dw|, dw = R dc, o = T
          const V3 gdw = project_out(gd, d, sm.inv_len);
          gcam[0] += gdw.x * sm.dc.x; gcam[1] += gdw.x * sm.dc.y; gcam[2] += gdw.x * sm.dc.z;
          gcam[3] += gdw.y * sm.dc.x; gcam[4] += gdw.y * sm.dc.y; gcam[5] += gdw.y * sm.dc.z;
          gcam[6] += gdw.z * sm.dc.x; gcam[7] += gdw.z * sm.dc.y; gcam[8] += gdw.z * sm.dc.z;
          gcam[9] += gsv.x; gcam[10] += gsv.y; gcam[11] += gsv.z;
          gr = grr;
        }
        // camera: wave reduction of this chunk into LDS
        if (ballot(has_g)) {
          for (int k = 0; k < 12; ++k) {
            const float t = wave_sum(gcam[k]);
            if (lane == 0 && t != 0.0f) atomicAdd(&lds[12 * a.L + k], to_fix(t));
          }
        }
        // ---- per-vertex scatter: one atomic set per distinct triangle in the wave
        uint64_t todo = ballot(has_g);
        while (todo) {
          const int leader = (int)__builtin_ctzll(todo);
          const int key = readlane_i(ph.id, leader);
          const bool mine = has_g && ph.id == key;
          todo &= ~ballot(mine);
          const int* tv = a.tris + 3 * key;
          for (int k = 0; k < 3; ++k) {
            const int vi = tv[k];
            const float bk = bb[k];
            if (TEX) {
              // reflectance gradients go to the texels below
              float vals[6] = {gv[k].x, gv[k].y, gv[k].z, gn[k].x, gn[k].y, gn[k].z};
              for (int q = 0; q < 6; ++q) vals[q] = wave_sum(mine ? vals[q] : 0.0f);
              if (lane == leader) {
                if (g.verts) { fix_add(g.verts + 3 * vi, vals[0]); fix_add(g.verts + 3 * vi + 1, vals[1]); fix_add(g.verts + 3 * vi + 2, vals[2]); }
                if (g.normals) { fix_add(g.normals + 3 * vi, vals[3]); fix_add(g.normals + 3 * vi + 1, vals[4]); fix_add(g.normals + 3 * vi + 2, vals[5]); }
              }
            } else {
              float vals[13] = {gv[k].x, gv[k].y, gv[k].z, gn[k].x, gn[k].y, gn[k].z, gc.x * bk, gc.y * bk, gc.z * bk,
                                gs.x * bk, gs.y * bk, gs.z * bk, gr * bk};
              for (int q = 0; q < 13; ++q) vals[q] = wave_sum(mine ? vals[q] : 0.0f);
              if (lane == leader) {
                if (g.verts) { fix_add(g.verts + 3 * vi, vals[0]); fix_add(g.verts + 3 * vi + 1, vals[1]); fix_add(g.verts + 3 * vi + 2, vals[2]); }
                if (g.normals) { fix_add(g.normals + 3 * vi, vals[3]); fix_add(g.normals + 3 * vi + 1, vals[4]); fix_add(g.normals + 3 * vi + 2, vals[5]); }
                if (g.diffuse) { fix_add(g.diffuse + 3 * vi, vals[6]); fix_add(g.diffuse + 3 * vi + 1, vals[7]); fix_add(g.diffuse + 3 * vi + 2, vals[8]); }
                if (g.specular) { fix_add(g.specular + 3 * vi, vals[9]); fix_add(g.specular + 3 * vi + 1, vals[10]); fix_add(g.specular + 3 * vi + 2, vals[11]); }
                if (g.roughness) fix_add(g.roughness + vi, vals[12]);
              }
            }
          }
        }
        // ---- per-texel scatter (maps in use): lanes with the same bilinear
        // footprint (its first and last texel fix the other two) reduce together
        if (TEX) {
          uint64_t tdo = ballot(has_g);
          while (tdo) {
            const int leader = (int)__builtin_ctzll(tdo);
            const int k00 = readlane_i(tp.t00, leader), k11 = readlane_i(tp.t11, leader);
            const bool mine = has_g && tp.t00 == k00 && tp.t11 == k11;
            tdo &= ~ballot(mine);
            const int k10 = readlane_i(tp.t10, leader), k01 = readlane_i(tp.t01, leader);
            const float fx = tp.fx, fy = tp.fy;
            for (int q = 0; q < 4; ++q) {
              const float w = q == 0 ? (1.0f - fx) * (1.0f - fy)
                              : q == 1 ? fx * (1.0f - fy)
                              : q == 2 ? (1.0f - fx) * fy : fx * fy;
              const int t = q == 0 ? k00 : q == 1 ? k10 : q == 2 ? k01 : k11;
              float rv[7] = {gc.x * w, gc.y * w, gc.z * w, gs.x * w, gs.y * w, gs.z * w, gr * w};
              for (int c = 0; c < 7; ++c) rv[c] = wave_sum(mine ? rv[c] : 0.0f);
              if (lane == leader) {
                if (g.tex_c) { fix_add(g.tex_c + 3 * t, rv[0]); fix_add(g.tex_c + 3 * t + 1, rv[1]); fix_add(g.tex_c + 3 * t + 2, rv[2]); }
                if (g.tex_s) { fix_add(g.tex_s + 3 * t, rv[3]); fix_add(g.tex_s + 3 * t + 1, rv[4]); fix_add(g.tex_s + 3 * t + 2, rv[5]); }
                if (g.tex_r) fix_add(g.tex_r + t, rv[6]);
              }
            }
          }
        }
      }
      if (a.chunks > 1) __syncthreads();
      if (a.chunks == 1 && run) {
        // every other wave has arrived: their LDS sums are complete
        fix_t* slot = slots + (size_t)(bid % kSlots) * nl;
        for (int i = lane; i < nl; i += 64)
          if (lds[i] != 0) atomicAdd(slot + i, lds[i]);
      }
    }
  }
  if (a.chunks > 1) {
    __syncthreads();
    fix_t* slot = slots + (size_t)(bid % kSlots) * nl;
    for (int i = threadIdx.x; i < nl; i += 256)
      if (lds[i] != 0) atomicAdd(slot + i, lds[i]);
  }
}

// Occupancy: the traced kernel's shadow traversals and the adjoint shading
// fit five waves per SIMD without spilling; the kept-mask kernel runs at the
// occupancy that measured fastest.
template <bool TEX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_render_bwd(const RenderArgs* __restrict__ pa, const float* __restrict__ dEdp, FixGrads g,
                                                    fix_t* __restrict__ slots) {
  render_bwd_block<TEX, false>(*pa, dEdp, g, slots, blockIdx.x);
}

template <bool TEX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_render_bwd_kept(const RenderArgs* __restrict__ pa, const float* __restrict__ dEdp, FixGrads g,
                                                    fix_t* __restrict__ slots) {
  render_bwd_block<TEX, true>(*pa, dEdp, g, slots, blockIdx.x);
}

// Sum the slots (exact integer sums) into the caller's light and camera gradients.
// Values 12L .. 12L + 11 are the camera's, the rest (3 B^2) the SH
// coefficients'.
__device__ __forceinline__ void slots_reduce_block(const fix_t* __restrict__ slots, int nl, int L,
                                                   float* __restrict__ glight, float* __restrict__ grad,
                                                   float* __restrict__ gcam, float* __restrict__ gsh, int bid,
                                                   const uint32_t* gmax = nullptr) {
  const int i = bid;   // one block per value
  __shared__ fix_t red[256];
  fix_t acc = 0;
  for (int s = threadIdx.x; s < kSlots; s += 256) acc += slots[(size_t)s * nl + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const float v = (float)(from_fix(red[0]) / (double)grad_scale(gmax));
  if (i < 12 * L) {
    const int j = i / 12, k = i % 12;
    if (k < 9) { if (glight) glight[9 * j + k] += v; }
    else if (grad) grad[3 * j + (k - 9)] += v;
  } else if (i < 12 * L + 12) {
    if (gcam) gcam[i - 12 * L] += v;
  } else if (gsh) {
    gsh[i - 12 * L - 12] += v;
  }
}

__global__ __launch_bounds__(256) void k_slots_reduce(const fix_t* __restrict__ slots, int nl, int L,
                                                      float* __restrict__ glight, float* __restrict__ grad,
                                                      float* __restrict__ gcam, float* __restrict__ gsh,
                                                      const uint32_t* gmax) {
  slots_reduce_block(slots, nl, L, glight, grad, gcam, gsh, blockIdx.x, gmax);
}

// `slots` holds kSlots * (12 min(L, 128) + 12) accumulators (the caller sizes
// and owns it).  Lights go in groups of at most 128, one launch each: the
// sample-level chain is linear in the per-sample adjoint it starts from, so
// the groups' chains and scatters add up to the chain of the full sum (the
// vertex, texel and slot sums are exact integer sums).
void launch_render_backward(const RenderArgs& a, RenderArgs* d_args, const float* dEdp, const FixGrads& fg,
                            fix_t* slots, const fr_grads& g, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                            bool trace_primary) {
  const int blocks = tile_blocks(a);
  // slot 0: the call's arguments (camera pass); slot 1: the light group's
  const auto group_args = [&](int g0) {
    RenderArgs ag = a;
    ag.L = std::min(kBwdMaxLights, a.L - g0);
    ag.light0 = a.light0 + g0;
    ag.lights = a.lights + g0;
    ag.lc = std::max(a.lc, std::max(1, cdiv(ag.L, 4)));
    ag.n_lchunks = std::max(1, cdiv(ag.L, ag.lc));
    if (g0 > 0) ag.sh_bands = 0;   // the SH light goes with the first group
    return ag;
  };
  if (trace_primary) launch_put_args(a, d_args, st);
  launch_put_args(group_args(0), d_args + 1, st);
  if (e0) (void)hipEventRecord(e0, st);
  if (trace_primary) launch_primary(a, d_args, st);
  for (int g0 = 0; g0 == 0 || g0 < a.L; g0 += kBwdMaxLights) {
    const RenderArgs ag = group_args(g0);
    if (g0 > 0) launch_put_args(ag, d_args + 1, st);   // the previous group's kernel has finished
    const int nl = ag.L * 12 + 12 + 3 * ag.sh_bands * ag.sh_bands;
    launch_zero_fix(slots, (size_t)kSlots * nl, st);
    const size_t lds = nl * sizeof(fix_t) + kBwdPartBytes;
    const RenderArgs* pg = d_args + 1;
    if (ag.vis_in) {
      if (ag.M > 0)
        hipLaunchKernelGGL(k_render_bwd_kept<true>, dim3(blocks), dim3(256), lds, st, pg, dEdp, fg, slots);
      else
        hipLaunchKernelGGL(k_render_bwd_kept<false>, dim3(blocks), dim3(256), lds, st, pg, dEdp, fg, slots);
    } else {
      if (ag.M > 0)
        hipLaunchKernelGGL(k_render_bwd<true>, dim3(blocks), dim3(256), lds, st, pg, dEdp, fg, slots);
      else
        hipLaunchKernelGGL(k_render_bwd<false>, dim3(blocks), dim3(256), lds, st, pg, dEdp, fg, slots);
    }
    if (e1 && g0 + kBwdMaxLights >= a.L) (void)hipEventRecord(e1, st);
    hipLaunchKernelGGL(k_slots_reduce, dim3(nl), dim3(256), 0, st, slots, nl, ag.L,
                       g.light_geom ? g.light_geom + (size_t)9 * g0 : nullptr,
                       g.light_rad ? g.light_rad + (size_t)3 * g0 : nullptr, g.cam, ag.sh_bands > 0 ? g.sh : nullptr,
                       a.gmax);
  }
}

}  // namespace fr
