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
      gsign[3 * pid + c] = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
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

void launch_loss(const float* img, const float* target, int W, int H, int smooth, float* loss, float* dEdp,
                 double* scratch, float* gtmp, hipStream_t st) {
  const double e = 0.60653065971263342;   // exp(-1/2)
  const double z = (1.0 + 2.0 * e) * (1.0 + 2.0 * e);
  const Taps w{(float)(1.0 / z), (float)(e / z), (float)(e * e / z)};
  const int blocks = (W * H + 255) / 256;
  float* gs = (smooth && dEdp) ? gtmp : (dEdp ? dEdp : gtmp);
  hipLaunchKernelGGL(k_loss, dim3(blocks), dim3(256), 0, st, img, target, W, H, smooth, w, gs, scratch);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, scratch, blocks, loss);
  if (smooth && dEdp) hipLaunchKernelGGL(k_smooth_adjoint, dim3(blocks), dim3(256), 0, st, gtmp, W, H, w, dEdp);
}

}  // namespace fr
