// Forward render: primary rays, shadow rays to every area light, Cook-Torrance
// shading, per-pixel Monte-Carlo mean (Sec. 3.3, Sec. 4, Appendix A).
//
// Work decomposition: one wave = one tile of 64/S pixels x S samples (S <= 64),
// lane = (pixel, sample).  All lanes of a wave trace their shadow ray towards
// the same light j at the same time, which keeps the wave-packet traversal
// coherent.  The per-pixel mean is a fixed-order butterfly over the S lanes of
// the pixel (deterministic).  Waves are mapped to tiles XCD-aware (wave_tile).
#include "fr_shade.h"

namespace fr {

template <bool DUMP>
__global__ __launch_bounds__(256) void k_render_fwd(RenderArgs a, float* __restrict__ image) {
  const int lane = threadIdx.x & 63;
  const int tile = wave_tile(a);
  if (tile < 0) return;
  PixelSample ps = pixel_sample(a, tile, lane);
  float acc[3] = {0.0f, 0.0f, 0.0f};
  TravStats st = {0, 0, 0, 0, 0};
  TravStats st2 = {0, 0, 0, 0, 0};
  for (int chunk = 0; chunk < a.chunks; ++chunk) {
    const int s = ps.s0 + chunk * 64;
    Sample sm;
    camera_sample(a, ps, s, sm);
    HitState h;
    h.t = 3.4e38f; h.id = -1; h.tamb = 3.4e38f;
    bool dummy = false;
    trace<false, DUMP>(a.nodes, a.recs, a.F, sm.ray, ps.valid, -1, h, dummy, &st);
    const size_t rs = (size_t)ps.pid * a.S + s;
    Frame fr;
    const bool shaded = ps.valid && h.id >= 0 && shading_frame(a, sm, h, fr);
    if (DUMP && ps.valid) {
      a.dbg_hit[rs] = h.id;
      const bool pf = hit_ambiguous(h) || (h.id >= 0 && fabsf(fr.cos_o) < kFlagCos);
      a.dbg_pflag[rs] = pf ? 1 : 0;
    }
    for (int j = 0; j < a.L; ++j) {
      const LightRec& Lj = a.lights[j];
      LightSample ls;
      const bool lit = shaded && light_sample(a, ps.pid, s, j, Lj, fr, ls);
      Ray sr;
      sr.o = fr.x; sr.d = ls.l; sr.tmin = kShadowTmin; sr.tmax = ls.dist;
      ray_setup(sr);
      HitState sh;
      sh.tamb = 3.4e38f;
      bool occ = false;
      trace<true, DUMP>(a.nodes, a.recs, a.F, sr, lit, h.id, sh, occ, &st2);
      float g1flag = 0.0f;
      if (lit && !occ) {
        float f[3];
        brdf_eval<DUMP>(a.variant, a.components, fr, ls, f, g1flag);
        const float w = ls.geom;
        acc[0] += Lj.rad[0] * f[0] * w;
        acc[1] += Lj.rad[1] * f[1] * w;
        acc[2] += Lj.rad[2] * f[2] * w;
      }
      if (DUMP && ps.valid) {
        uint8_t code = !shaded ? VIS_NONE : (!lit ? VIS_CULLED : (occ ? VIS_OCCLUDED : VIS_VISIBLE));
        const bool amb = (shaded && ls.amb) || sh.tamb < 3.0e38f || g1flag != 0.0f;
        a.dbg_vis[rs * a.L + j] = code | (amb ? VIS_FLAG : 0);
      }
    }
  }
  if (DUMP && a.dbg_stats) {
    // lane counts summed over the wave; wave counts taken once per wave
    const uint32_t v[10] = {st.lane_int, st.lane_leaf, st.rays, st2.lane_int, st2.lane_leaf, st2.rays,
                            st.wave_int, st.wave_leaf, st2.wave_int, st2.wave_leaf};
    for (int k = 0; k < 10; ++k) {
      uint32_t x = v[k];
      if (k < 6)
        for (int off = 32; off >= 1; off >>= 1) x += (uint32_t)__shfl_xor((int)x, off, 64);
      if (lane == 0) atomicAdd(reinterpret_cast<unsigned long long*>(a.dbg_stats) + k, (unsigned long long)x);
    }
  }
  // per-pixel mean over the S samples
  for (int k = 0; k < 3; ++k) acc[k] = group_sum(acc[k], a.lanes_per_pixel);
  if (ps.valid && ps.s0 == 0) {
    const float inv = 1.0f / (float)a.S;
    image[3 * ps.pid] = acc[0] * inv;
    image[3 * ps.pid + 1] = acc[1] * inv;
    image[3 * ps.pid + 2] = acc[2] * inv;
  }
}

void launch_render_forward(const RenderArgs& a, float* image, hipStream_t st) {
  const int blocks = wave_blocks_strips(a);
  if (a.dbg_hit)
    hipLaunchKernelGGL(k_render_fwd<true>, dim3(blocks), dim3(256), 0, st, a, image);
  else
    hipLaunchKernelGGL(k_render_fwd<false>, dim3(blocks), dim3(256), 0, st, a, image);
}

}  // namespace fr
