// Measurement probe: the achievable rate of non-packed FP32 FMAs, the unit
// of the ALU roofline the render kernels are measured against (their work
// is counted in lane-operations, one FMA or compare or min/max each).
#include "fr_kernels.h"

namespace fr {

// Eight independent FMA chains per lane, `iters` steps each: 8 iters lane-FMAs
// per thread, with no memory traffic but the final store.
__global__ __launch_bounds__(256) void k_fma_chains(int iters, float a, float b, float* __restrict__ out) {
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = (float)(threadIdx.x + k);
#pragma unroll 8
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace fr

extern "C" int fr_probe_valu(int32_t blocks, int32_t iters, float* d_out, fr_stream stream) {
  if (blocks <= 0 || iters <= 0 || !d_out) return FR_ERR_INVALID_ARG;
  // a = 1 - 2^-20, b = 2^-20: the chains stay finite and non-denormal
  hipLaunchKernelGGL(fr::k_fma_chains, dim3(blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), iters,
                     0.99999905f, 9.5367432e-7f, d_out);
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}
