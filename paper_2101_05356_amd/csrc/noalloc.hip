// fr_loss_noalloc: the photometric loss of fr_loss with its scratch in a
// fixed static device array of the library instead of a caller workspace,
// for callers that cannot allocate device memory.  The array (per device,
// resolved once with hipGetSymbolAddress) holds the per-block FP64 sums and
// the sign image of up to kNoAllocPixels pixels; every call on a device
// shares it, so calls that overlap on one device race.  The kernels write
// every scratch word they read, so nothing needs clearing between calls.
#include <mutex>

#include "fr_kernels.h"

namespace fr {

constexpr int kNoAllocPixels = 1 << 20;   // 1024 x 1024
constexpr size_t kNoAllocBytes = ((size_t)kNoAllocPixels / 256 * sizeof(double) + 255) / 256 * 256 +
                                 ((size_t)3 * kNoAllocPixels * sizeof(float) + 255) / 256 * 256;
constexpr int kNoAllocDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocDevices] = {};
}  // namespace

// Device address of `scratch` on device dev (the current device), resolved on
// the first request for that device; nullptr if the runtime refuses.
void* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kNoAllocDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace fr

extern "C" int fr_loss_noalloc(const float* d_image, const float* d_target, int32_t W, int32_t H, int32_t smooth,
                               float* d_loss, float* d_dEdp, fr_stream stream) {
  if (!d_image || !d_target || !d_loss || W <= 0 || H <= 0) return FR_ERR_INVALID_ARG;
  if ((long long)W * H > fr::kNoAllocPixels) return FR_ERR_LIMIT;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return FR_ERR_DEVICE;
  char* base = static_cast<char*>(fr::noalloc_scratch(dev));
  if (!base) return FR_ERR_DEVICE;
  const size_t part_bytes = (((size_t)W * H + 255) / 256 * sizeof(double) + 255) / 256 * 256;
  double* part = reinterpret_cast<double*>(base);
  float* gtmp = smooth ? reinterpret_cast<float*>(base + part_bytes) : nullptr;
  fr::launch_loss(d_image, d_target, W, H, smooth, d_loss, d_dEdp, part, gtmp, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? FR_OK : FR_ERR_DEVICE;
}
