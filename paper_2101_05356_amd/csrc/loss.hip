// Photometric loss (Sec. 4 Eq. energy) with the 3x3 Gaussian smoothing of
// Sec. 4 "Variance Reduction": p~ = K * p (sigma 1, taps normalised to sum 1,
// clamp-to-edge), E = sum |p~ - p^R|, dE/dp = K^T * sign(p~ - p^R) with
// sign(0) = 0.  The loss sum is FP64 in a fixed tree order (deterministic).
#include "fr_kernels.h"

namespace fr {


__device__ __forceinline__ void loss_block(const float* __restrict__ img, const float* __restrict__ tgt, int W, int H,
                                              int smooth, Taps w, float* __restrict__ gsign,
                                              double* __restrict__ partial, int bid) {
  __shared__ double red[256];
  const int pid = bid * 256 + threadIdx.x;
  double acc = 0.0;
  if (pid < W * H) {
    const int x = pid % W, y = pid / W;
    const int xm = max(x - 1, 0), xp = min(x + 1, W - 1), ym = max(y - 1, 0), yp = min(y + 1, H - 1);
    for (int c = 0; c < 3; ++c) {
      float p;
      if (smooth) {
        const float cen = img[3 * (y * W + x) + c];
        const float edg = img[3 * (ym * W + x) + c] + img[3 * (yp * W + x) + c] + img[3 * (y * W + xm) + c] +
                          img[3 * (y * W + xp) + c];
        const float cor = img[3 * (ym * W + xm) + c] + img[3 * (ym * W + xp) + c] + img[3 * (yp * W + xm) + c] +
                          img[3 * (yp * W + xp) + c];
        p = w.c * cen + w.e * edg + w.k * cor;
      } else {
        p = img[3 * pid + c];
      }
      const float d = p - tgt[3 * pid + c];
      acc += (double)fabsf(d);
      if (gsign) gsign[3 * pid + c] = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[bid] = red[0];
}

__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ img, const float* __restrict__ tgt, int W, int H,
                                              int smooth, Taps w, float* __restrict__ gsign,
                                              double* __restrict__ partial) {
  loss_block(img, tgt, W, H, smooth, w, gsign, partial, blockIdx.x);
}

__device__ __forceinline__ void loss_final_block(const double* __restrict__ partial, int n, float* __restrict__ loss, int bid) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)red[0];
}

__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ partial, int n, float* __restrict__ loss) {
  loss_final_block(partial, n, loss, blockIdx.x);
}

// Sources i of a clamp-to-edge tap: clamp(i + o) == q, o in {-1, 0, 1}.
__device__ __forceinline__ int tap_sources(int q, int o, int n, int src[2]) {
  int k = 0;
  if (o == 0) { src[k++] = q; return k; }
  const int i = q - o;
  if (i >= 0 && i < n) src[k++] = i;
  if (o < 0 && q == 0) src[k++] = 0;          // clamp(0 - 1) == 0
  if (o > 0 && q == n - 1) src[k++] = n - 1;  // clamp(n - 1 + 1) == n - 1
  return k;
}

__device__ __forceinline__ void smooth_adjoint_block(const float* __restrict__ g, int W, int H, Taps w,
                                                        float* __restrict__ out, int bid) {
  const int pid = bid * 256 + threadIdx.x;
  if (pid >= W * H) return;
  const int qx = pid % W, qy = pid / W;
  float acc[3] = {0.0f, 0.0f, 0.0f};
  for (int oy = -1; oy <= 1; ++oy) {
    int sy[2];
    const int ny = tap_sources(qy, oy, H, sy);
    for (int ox = -1; ox <= 1; ++ox) {
      int sx[2];
      const int nx = tap_sources(qx, ox, W, sx);
      const float wt = (oy == 0 && ox == 0) ? w.c : ((oy == 0 || ox == 0) ? w.e : w.k);
      for (int a = 0; a < ny; ++a)
        for (int b = 0; b < nx; ++b) {
          const int s = sy[a] * W + sx[b];
          acc[0] += wt * g[3 * s];
          acc[1] += wt * g[3 * s + 1];
          acc[2] += wt * g[3 * s + 2];
        }
    }
  }
  out[3 * pid] = acc[0];
  out[3 * pid + 1] = acc[1];
  out[3 * pid + 2] = acc[2];
}

__global__ __launch_bounds__(256) void k_smooth_adjoint(const float* __restrict__ g, int W, int H, Taps w,
                                                        float* __restrict__ out) {
  smooth_adjoint_block(g, W, H, w, out, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Stage II regularisers of the personalised maps (Sec. 4 "Stage II",
// Eq. loss3): w_sym (E_s(C) + E_s(S)) + w_chroma (E_c(C, C0) + E_c(S, S0))
// + w_smooth (E_m(C) + E_m(S) + E_m(R)) + w_box (E_b(S) + E_b(R)).  Texel
// (i, j) at j M + i; the flip maps i to M - 1 - i; chromaticity
// x / (x_r + x_g + x_b + 1e-6); E_m sums each texel's squared differences to
// its in-map 4-neighbours; E_b(x) = min(x, 0)^2 + max(x - 1, 0)^2.  One
// thread per texel gathers its own gradient (no atomics) and its terms of
// the sum (FP64, fixed-order block and final sums).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float sgnf(float x) { return x > 0.0f ? 1.0f : (x < 0.0f ? -1.0f : 0.0f); }

// Symmetry, smoothness and (optionally) chromaticity terms of channel-
// interleaved map X (nc channels) at texel t; adds to g[0..nc) and returns
// the texel's part of the weighted sum.
__device__ __forceinline__ double map_terms(const float* __restrict__ X, const float* __restrict__ Y, int nc, int M,
                                            int i, int j, const MapRegWeights& w, bool sym, float* g) {
  const int t = j * M + i;
  double e = 0.0;
  const int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
  for (int c = 0; c < nc; ++c) {
    const float x = X[nc * t + c];
    if (sym) {
      const float d = x - X[nc * (j * M + (M - 1 - i)) + c];
      e += (double)w.w_sym * fabs((double)d);
      g[c] += w.w_sym * 2.0f * sgnf(d);
    }
    for (int k = 0; k < 4; ++k) {
      const int ii = nb[k][0], jj = nb[k][1];
      if (ii < 0 || ii >= M || jj < 0 || jj >= M) continue;
      const float d = x - X[nc * (jj * M + ii) + c];
      e += (double)w.w_smooth * (double)d * (double)d;
      g[c] += w.w_smooth * 4.0f * d;
    }
  }
  if (Y) {   // chromaticity against the reference
    const float T = X[3 * t] + X[3 * t + 1] + X[3 * t + 2] + 1e-6f;
    const float U = Y[3 * t] + Y[3 * t + 1] + Y[3 * t + 2] + 1e-6f;
    float s[3], sx = 0.0f;
    for (int c = 0; c < 3; ++c) {
      const float d = X[3 * t + c] / T - Y[3 * t + c] / U;
      e += (double)w.w_chroma * fabs((double)d);
      s[c] = sgnf(d);
      sx += s[c] * X[3 * t + c];
    }
    for (int c = 0; c < 3; ++c) g[c] += w.w_chroma * (s[c] / T - sx / (T * T));
  }
  return e;
}

__device__ __forceinline__ double box_term(float x, float wb, float& g) {
  const float lo = fminf(x, 0.0f), hi = fmaxf(x - 1.0f, 0.0f);
  g += wb * (2.0f * lo + 2.0f * hi);
  return (double)wb * ((double)lo * lo + (double)hi * hi);
}

__global__ __launch_bounds__(256) void k_map_reg(const float* __restrict__ Cm, const float* __restrict__ Sm,
                                                 const float* __restrict__ Rm, const float* __restrict__ C0,
                                                 const float* __restrict__ S0, int M, MapRegWeights w,
                                                 float* __restrict__ gC, float* __restrict__ gS,
                                                 float* __restrict__ gR, double* __restrict__ partial) {
  __shared__ double red[256];
  const int t = blockIdx.x * 256 + threadIdx.x;
  double e = 0.0;
  if (t < M * M) {
    const int i = t % M, j = t / M;
    float g3[3] = {0.0f, 0.0f, 0.0f};
    e += map_terms(Cm, C0, 3, M, i, j, w, true, g3);
    if (gC) for (int c = 0; c < 3; ++c) gC[3 * t + c] += g3[c];
    g3[0] = g3[1] = g3[2] = 0.0f;
    e += map_terms(Sm, S0, 3, M, i, j, w, true, g3);
    for (int c = 0; c < 3; ++c) e += box_term(Sm[3 * t + c], w.w_box, g3[c]);
    if (gS) for (int c = 0; c < 3; ++c) gS[3 * t + c] += g3[c];
    float g1[1] = {0.0f};
    e += map_terms(Rm, nullptr, 1, M, i, j, w, false, g1);
    e += box_term(Rm[t], w.w_box, g1[0]);
    if (gR) gR[t] += g1[0];
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

void launch_map_regularizers(const float* Cm, const float* Sm, const float* Rm, const float* C0, const float* S0, int M,
                             const MapRegWeights& w, float* loss, float* gC, float* gS, float* gR, double* scratch,
                             hipStream_t st) {
  const int blocks = cdiv(M * M, 256);
  hipLaunchKernelGGL(k_map_reg, dim3(blocks), dim3(256), 0, st, Cm, Sm, Rm, C0, S0, M, w, gC, gS, gR, scratch);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, scratch, blocks, loss);
}

// ---------------------------------------------------------------------------
// Stage I priors (Sec. 4 "Stage I", Eq. loss1): statistical w sum (x/sigma)^2,
// soft box w sum (min(x,0)^2 + max(x-1,0)^2), and the light prior
// w sum_j ||I_j - mean_c(I_j)||^2 over RGB triples.  One workgroup: thread t
// takes values (lights, for the light prior) t, t + 256, ... in order, then a
// fixed-order FP64 tree sum (the priors act on parameter vectors of a few
// hundred values; no scratch memory).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_prior(const float* __restrict__ x, const float* __restrict__ sigma, int n,
                                               int kind, float w, float* __restrict__ g, float* __restrict__ loss) {
  __shared__ double red[256];
  double e = 0.0;
  const int m = kind == FR_PRIOR_LIGHT_CHROMA ? n / 3 : n;
  for (int i = threadIdx.x; i < m; i += 256) {
    if (kind == FR_PRIOR_LIGHT_CHROMA) {
      const float mu = (x[3 * i] + x[3 * i + 1] + x[3 * i + 2]) * (1.0f / 3.0f);
      for (int c = 0; c < 3; ++c) {
        const float d = x[3 * i + c] - mu;
        e += (double)w * (double)d * (double)d;
        if (g) g[3 * i + c] += w * 2.0f * d;
      }
    } else if (kind == FR_PRIOR_STATISTICAL) {
      const float q = x[i] / sigma[i];
      e += (double)w * (double)q * (double)q;
      if (g) g[i] += w * 2.0f * q / sigma[i];
    } else {
      const float lo = fminf(x[i], 0.0f), hi = fmaxf(x[i] - 1.0f, 0.0f);
      e += (double)w * ((double)lo * lo + (double)hi * hi);
      if (g) g[i] += w * (2.0f * lo + 2.0f * hi);
    }
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)red[0];
}

void launch_prior(const float* x, const float* sigma, int n, int kind, float w, float* loss, float* g, hipStream_t st) {
  hipLaunchKernelGGL(k_prior, dim3(1), dim3(256), 0, st, x, sigma, n, kind, w, g, loss);
}

// ---------------------------------------------------------------------------
// Landmark loss (Sec. 4 Eq. landmark): sum_l || Pi(v_l) - z_l ||^2 with the
// render's pinhole (Sec. 3.1): p = R^T (X - T), z = -p_z,
// f = ((p_x / z) / (tan_half aspect) + 1) W / 2, (1 - (p_y / z) / tan_half) H / 2.
// One block; each thread takes landmarks l, l + 256, ...; the vertex
// gradients go to their vertices (distinct indices: plain adds), the
// camera's and the loss through fixed-order block sums.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_landmarks(const float* __restrict__ V, const int32_t* __restrict__ idx, int n,
                                                   const float* __restrict__ cam, float th, int W, int H,
                                                   const float* __restrict__ zt, float* __restrict__ loss,
                                                   float* __restrict__ gV, float* __restrict__ gcam) {
  __shared__ double red[256];
  __shared__ float redc[12][256];
  double e = 0.0;
  float gc[12];
  for (int k = 0; k < 12; ++k) gc[k] = 0.0f;
  const float asp = (float)W / (float)H;
  for (int l = threadIdx.x; l < n; l += 256) {
    const int i = idx[l];
    const V3 X = ld3(V, i), T = {cam[9], cam[10], cam[11]};
    const V3 q = X - T;
    const V3 p = {cam[0] * q.x + cam[3] * q.y + cam[6] * q.z, cam[1] * q.x + cam[4] * q.y + cam[7] * q.z,
                  cam[2] * q.x + cam[5] * q.y + cam[8] * q.z};
    const float z = -p.z;
    const float ax = 0.5f * (float)W / (th * asp), ay = 0.5f * (float)H / th;
    const float fx = (p.x / z) * ax + 0.5f * (float)W, fy = 0.5f * (float)H - (p.y / z) * ay;
    const float rx = fx - zt[2 * l], ry = fy - zt[2 * l + 1];
    e += (double)rx * rx + (double)ry * ry;
    // dE/dp through both film coordinates
    const V3 gp = {2.0f * rx * ax / z, -2.0f * ry * ay / z, 2.0f * rx * ax * p.x / (z * z) - 2.0f * ry * ay * p.y / (z * z)};
    const V3 gX = {cam[0] * gp.x + cam[1] * gp.y + cam[2] * gp.z, cam[3] * gp.x + cam[4] * gp.y + cam[5] * gp.z,
                   cam[6] * gp.x + cam[7] * gp.y + cam[8] * gp.z};
    if (gV) { gV[3 * i] += gX.x; gV[3 * i + 1] += gX.y; gV[3 * i + 2] += gX.z; }
    const float qq[3] = {q.x, q.y, q.z}, pp[3] = {gp.x, gp.y, gp.z};
    for (int k = 0; k < 3; ++k)
      for (int c = 0; c < 3; ++c) gc[3 * k + c] += qq[k] * pp[c];
    gc[9] -= gX.x; gc[10] -= gX.y; gc[11] -= gX.z;
  }
  red[threadIdx.x] = e;
  for (int k = 0; k < 12; ++k) redc[k][threadIdx.x] = gc[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[threadIdx.x] += red[threadIdx.x + s];
      for (int k = 0; k < 12; ++k) redc[k][threadIdx.x] += redc[k][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    loss[0] = (float)red[0];
    if (gcam) for (int k = 0; k < 12; ++k) gcam[k] += redc[k][0];
  }
}

void launch_landmarks(const float* V, const int32_t* idx, int n, const float* cam, float tan_half, int W, int H,
                      const float* z, float* loss, float* gV, float* gcam, hipStream_t st) {
  hipLaunchKernelGGL(k_landmarks, dim3(1), dim3(256), 0, st, V, idx, n, cam, tan_half, W, H, z, loss, gV, gcam);
}

static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

size_t loss_scratch_bytes(int W, int H, int smooth) {
  const size_t px = (size_t)W * H;
  return al256((px + 255) / 256 * sizeof(double)) + (smooth ? al256(3 * px * sizeof(float)) : 0);
}

size_t map_reg_scratch_bytes(int M) { return al256(((size_t)M * M + 255) / 256 * sizeof(double)); }

void launch_loss(const float* img, const float* target, int W, int H, int smooth, float* loss, float* dEdp,
                 double* scratch, float* gtmp, hipStream_t st) {
  const double e = 0.60653065971263342;   // exp(-1/2)
  const double z = (1.0 + 2.0 * e) * (1.0 + 2.0 * e);
  const Taps w{(float)(1.0 / z), (float)(e / z), (float)(e * e / z)};
  const int blocks = (W * H + 255) / 256;
  float* gs = dEdp ? (smooth ? gtmp : dEdp) : nullptr;
  hipLaunchKernelGGL(k_loss, dim3(blocks), dim3(256), 0, st, img, target, W, H, smooth, w, gs, scratch);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, scratch, blocks, loss);
  if (smooth && dEdp) hipLaunchKernelGGL(k_smooth_adjoint, dim3(blocks), dim3(256), 0, st, gtmp, W, H, w, dEdp);
}

}  // namespace fr
