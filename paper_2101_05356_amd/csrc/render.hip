// Forward render: primary rays, shadow rays to every area light, Cook-Torrance
// shading, per-pixel Monte-Carlo mean (Sec. 3.3, Sec. 4, Appendix A).
//
// Work decomposition: one wave = one tile of 64/S pixels x S samples (S <= 64),
// lane = (pixel, sample).  All lanes of a wave trace their shadow ray towards
// the same light j at the same time, which keeps the wave-packet traversal
// coherent.  The per-pixel mean is a fixed-order butterfly over the S lanes of
// the pixel (deterministic).  Waves are mapped to tiles XCD-aware (wave_tile).
//
// Primary pass: the camera ray of every sample is traced once per render call
// (k_primary) and its hit stored; the (tile, light chunk) work items of the
// forward and backward read it instead of tracing the camera ray again.
#include "fr_shade.h"

namespace fr {

// Normal-direction cosine n_s . o of a stored hit (the forward dump's flag).
__device__ __forceinline__ float prim_cos_o(const RenderArgs& a, const Sample& sm, int id, const double bd[3]) {
  const int* t = a.tris + 3 * id;
  const float b0 = (float)bd[0], b1 = (float)bd[1], b2 = (float)bd[2];
  const V3 m = ld3(a.normals, t[0]) * b0 + ld3(a.normals, t[1]) * b1 + ld3(a.normals, t[2]) * b2;
  const V3 ns = m * (1.0f / sqrtf(dot(m, m)));
  return -dot(ns, sm.ray.d);
}

// One wave per tile: trace every sample's camera ray, store its hit (and,
// in dump builds, the decision, its ambiguity flag and the camera-ray
// statistics).
template <bool DUMP>
__device__ __forceinline__ void primary_block(const RenderArgs& a, int bid) {
  const int lane = threadIdx.x & 63;
  const Item it = wave_item(a, bid, 1);
  if (it.tile < 0) return;
  const PixelSample ps = pixel_sample(a, it.tile, lane);
  TravStats st = {0, 0, 0, 0, 0};
  for (int chunk = 0; chunk < a.chunks; ++chunk) {
    const int s = ps.s0 + chunk * 64;
    Sample sm;
    camera_sample(a, ps, s, sm);
    HitState h;
    h.t = 3.4e38f; h.id = -1; h.tamb = 3.4e38f;
    bool dummy = false;
    trace<false, DUMP>(a.nodes, a.recs, a.F, sm.ray, ps.valid, -1, h, dummy, &st);
    PrimHit ph = {h.id, h.t, 0.0, 0.0};
    double bd[3] = {1.0, 0.0, 0.0};
    if (ps.valid && h.id >= 0) {
      double fxd, fyd;
      film_point(a, ps, s, fxd, fyd);
      const int* t = a.tris + 3 * h.id;
      const int vi[3] = {t[0], t[1], t[2]};
      bary64(a, fxd, fyd, vi, bd);
      ph.b1 = bd[1];
      ph.b2 = bd[2];
    }
    const size_t rs = (size_t)ps.pid * a.S + s;
    if (ps.valid) a.prim[rs] = ph;
    if (DUMP && ps.valid) {
      a.dbg_hit[rs] = h.id;
      const bool pf = hit_ambiguous(h) || (h.id >= 0 && fabsf(prim_cos_o(a, sm, h.id, bd)) < kFlagCos);
      a.dbg_pflag[rs] = pf ? 1 : 0;
    }
  }
  if (DUMP && a.dbg_stats) {
    const uint32_t v[5] = {st.lane_box, st.lane_leaf, st.rays, st.wave_int, st.wave_leaf};
    const int slot[5] = {0, 1, 2, 6, 7};
    for (int k = 0; k < 5; ++k) {
      uint32_t x = v[k];
      if (k < 3)
        for (int off = 32; off >= 1; off >>= 1) x += (uint32_t)__shfl_xor((int)x, off, 64);
      if (lane == 0) atomicAdd(reinterpret_cast<unsigned long long*>(a.dbg_stats) + slot[k], (unsigned long long)x);
    }
  }
}

// eight waves per SIMD (64 VGPRs): 133 us against 139 us at six on the face render
template <bool DUMP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_primary(const RenderArgs* __restrict__ pa) {
  primary_block<DUMP>(*pa, blockIdx.x);
}

// One call's arguments into its device slot (word by word).
__global__ __launch_bounds__(256) void k_put_args(RenderArgs a, RenderArgs* __restrict__ dst) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&a);
  uint32_t* out = reinterpret_cast<uint32_t*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(RenderArgs) / 4); i += 256) out[i] = src[i];
}
static_assert(sizeof(RenderArgs) % 4 == 0, "RenderArgs copied as 32-bit words");

void launch_put_args(const RenderArgs& a, RenderArgs* d_slot, hipStream_t st) {
  hipLaunchKernelGGL(k_put_args, dim3(1), dim3(256), 0, st, a, d_slot);
}

void launch_primary(const RenderArgs& a, const RenderArgs* d_slot, hipStream_t st) {
  const int blocks = wave_blocks_items(a, 1);
  if (a.dbg_hit)
    hipLaunchKernelGGL(k_primary<true>, dim3(blocks), dim3(256), 0, st, d_slot);
  else
    hipLaunchKernelGGL(k_primary<false>, dim3(blocks), dim3(256), 0, st, d_slot);
}

template <bool DUMP, bool TEX, bool LANE = false>
__device__ __forceinline__ void render_fwd_block(const RenderArgs& a, float* __restrict__ image, int bid) {
  const int lane = threadIdx.x & 63;
  const Item it = wave_item(a, bid);
  if (it.tile < 0) return;
  const int tile = it.tile;
  const int j0 = it.chunk * a.lc, j1 = min(a.L, j0 + a.lc);
  PixelSample ps = pixel_sample(a, tile, lane);
  float acc[3] = {0.0f, 0.0f, 0.0f};
  TravStats st2 = {0, 0, 0, 0, 0};
  uint32_t n_shaded = 0;   // dump statistics: camera samples with a shading point (counted by light chunk 0)
  for (int chunk = 0; chunk < a.chunks; ++chunk) {
    const int s = ps.s0 + chunk * 64;
    const size_t rs = (size_t)ps.pid * a.S + s;
    double bd[3] = {1.0, 0.0, 0.0};
    PrimHit ph = {-1, 0.0f, 0.0, 0.0};
    if (ps.valid) ph = load_prim(a, rs, bd);
    // the camera ray (for the view direction) only where a sample has a shading point
    Sample sm;
    if (ballot(ps.valid && ph.id >= 0)) camera_sample(a, ps, s, sm);
    Frame fr;
    const bool shaded = ps.valid && ph.id >= 0 && shading_frame<TEX>(a, sm, ph.id, ph.t, bd, fr);
    if (DUMP && shaded && it.chunk == 0) ++n_shaded;
    // shadow decisions of every light of the chunk, then the shading of the visible ones
    const auto draw = [&](int j) { return philox((uint32_t)ps.pid, (uint32_t)s, 1u + (uint32_t)(a.light0 + j), a.step, a.k0, a.k1); };
    const auto note = [&](int j, bool lit, bool occ, const LightSample& ls, const HitState& sh) {
      if (ps.valid) {
        const uint8_t code = !shaded ? VIS_NONE : (!lit ? VIS_CULLED : (occ ? VIS_OCCLUDED : VIS_VISIBLE));
        const bool amb = (shaded && ls.amb) || sh.tamb < 3.0e38f;
        a.dbg_vis[rs * a.L + j] = code | (amb ? VIS_FLAG : 0);
      }
    };
    const auto skip = [&](int j) {
      if (DUMP && ps.valid) a.dbg_vis[rs * a.L + j] = shaded ? VIS_CULLED : VIS_NONE;
    };
    // (a wave without shading points skips the lights; the dumps record every one)
    const uint32_t vmask = DUMP || ballot(shaded) ? shadow_mask<DUMP, LANE>(a, j0, j1, shaded, fr, ph.id, draw, note, skip, &st2) : 0u;
    if (a.vis_out && ps.valid) a.vis_out[(size_t)it.chunk * ((size_t)a.W * a.H * a.S) + rs] = vmask;
    for (int j = j0; j < j1; ++j) {
      const bool vis = (vmask >> (j - j0)) & 1u;
      if (!ballot(vis)) continue;
      const LightRec Lj = load_const(a.lights, j);
      const U4 r = Lj.shape == FR_LIGHT_DIRECTIONAL ? U4{0u, 0u, 0u, 0u} : draw(j);
      LightSample ls;
      light_point(Lj, unit24(r.x), unit24(r.y), fr, ls);
      if (vis) {
        float f[3], g1flag = 0.0f;
        brdf_eval<DUMP>(a.variant, a.components, fr, ls, f, g1flag);
        const float w = ls.geom;
        acc[0] += Lj.rad[0] * f[0] * w;
        acc[1] += Lj.rad[1] * f[1] * w;
        acc[2] += Lj.rad[2] * f[2] * w;
        if (DUMP && g1flag != 0.0f) a.dbg_vis[rs * a.L + j] |= VIS_FLAG;
      }
    }
    // the SH light, once per sample (by the tile's first light chunk)
    if (a.sh_bands > 0 && it.chunk == 0 && (a.components & 1)) {
      const V3 e = sh_irradiance(a, shaded ? fr.ns : V3{0.0f, 0.0f, 1.0f});
      if (shaded) {
        acc[0] += fr.c.x * e.x * (1.0f / kPi);
        acc[1] += fr.c.y * e.y * (1.0f / kPi);
        acc[2] += fr.c.z * e.z * (1.0f / kPi);
      }
    }
  }
  if (DUMP && a.dbg_stats) {
    // shadow-ray counts (the primary pass adds the camera rays'): lane counts
    // summed over the wave, wave counts taken once per wave
    const uint32_t v[6] = {st2.lane_box, st2.lane_leaf, st2.rays, st2.wave_int, st2.wave_leaf, n_shaded};
    const int slot[6] = {3, 4, 5, 8, 9, 10};
    for (int k = 0; k < 6; ++k) {
      uint32_t x = v[k];
      if (k < 3 || k == 5)
        for (int off = 32; off >= 1; off >>= 1) x += (uint32_t)__shfl_xor((int)x, off, 64);
      if (lane == 0) atomicAdd(reinterpret_cast<unsigned long long*>(a.dbg_stats) + slot[k], (unsigned long long)x);
    }
  }
  // per-pixel mean over the S samples
  for (int k = 0; k < 3; ++k) acc[k] = group_sum(acc[k], a.lanes_per_pixel);
  if (ps.valid && ps.s0 == 0) {
    const float inv = 1.0f / (float)a.S;
    float* out = a.n_lchunks > 1 ? a.partial + (size_t)it.chunk * 3 * a.W * a.H : image;
    out[3 * ps.pid] = acc[0] * inv;
    out[3 * ps.pid + 1] = acc[1] * inv;
    out[3 * ps.pid + 2] = acc[2] * inv;
  }
}

template <bool DUMP, bool TEX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_render_fwd(const RenderArgs* __restrict__ pa, float* __restrict__ image) {
  render_fwd_block<DUMP, TEX>(*pa, image, blockIdx.x);
}

// The forward with the per-lane shadow-ray traversal (fr_render_opts.
// shadow_traversal = 1; production builds only): same results, measured
// against the wave packet.
template <bool TEX>
__global__ __launch_bounds__(256) void k_render_fwd_lane(const RenderArgs* __restrict__ pa, float* __restrict__ image) {
  render_fwd_block<false, TEX, true>(*pa, image, blockIdx.x);
}

// image = sum over light chunks of the partial images, in chunk order.
__device__ __forceinline__ void sum_chunks_block(const float* __restrict__ partial, int n, int nch,
                                                 float* __restrict__ image, int bid) {
  const int i = bid * 256 + threadIdx.x;
  if (i >= n) return;
  float acc = partial[i];
  for (int c = 1; c < nch; ++c) acc += partial[(size_t)c * n + i];
  image[i] = acc;
}

__global__ __launch_bounds__(256) void k_sum_chunks(const float* __restrict__ partial, int n, int nch,
                                                    float* __restrict__ image) {
  sum_chunks_block(partial, n, nch, image, blockIdx.x);
}

void launch_render_forward(const RenderArgs& a, RenderArgs* d_args, float* image, hipStream_t st, hipEvent_t e0,
                           hipEvent_t e1) {
  const int blocks = wave_blocks_items(a);
  launch_put_args(a, d_args, st);
  if (e0) (void)hipEventRecord(e0, st);
  launch_primary(a, d_args, st);
  if (a.shadow_traversal == 1 && !a.dbg_hit) {
    if (a.M > 0) hipLaunchKernelGGL((k_render_fwd_lane<true>), dim3(blocks), dim3(256), 0, st, d_args, image);
    else hipLaunchKernelGGL((k_render_fwd_lane<false>), dim3(blocks), dim3(256), 0, st, d_args, image);
  } else if (a.M > 0) {
    if (a.dbg_hit)
      hipLaunchKernelGGL((k_render_fwd<true, true>), dim3(blocks), dim3(256), 0, st, d_args, image);
    else
      hipLaunchKernelGGL((k_render_fwd<false, true>), dim3(blocks), dim3(256), 0, st, d_args, image);
  } else if (a.dbg_hit) {
    hipLaunchKernelGGL((k_render_fwd<true, false>), dim3(blocks), dim3(256), 0, st, d_args, image);
  } else {
    hipLaunchKernelGGL((k_render_fwd<false, false>), dim3(blocks), dim3(256), 0, st, d_args, image);
  }
  if (e1) (void)hipEventRecord(e1, st);
  if (a.n_lchunks > 1) {
    const int n = 3 * a.W * a.H;
    hipLaunchKernelGGL(k_sum_chunks, dim3((n + 255) / 256), dim3(256), 0, st, a.partial, n, a.n_lchunks, image);
  }
}

}  // namespace fr
