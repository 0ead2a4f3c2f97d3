// Surrogate-network gradient for callers that cannot allocate device memory:
// the kernels of hca_mlp_gradient, with their scratch (packed bfloat16
// operands, the GELU table, per-workgroup gradient partials and the loss
// slot) in one file-scope device array instead of a trainer's allocations.
#include <mutex>

#include "hca.h"
#include "mlp_dev.h"

namespace hca {
namespace {

// Scratch layout, 256-byte aligned regions.
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kOffPack = 0;
constexpr size_t kOffTab = kOffPack + align256(sizeof(bf16x8) * kPackAll);
constexpr size_t kOffPart = kOffTab + align256(sizeof(float2) * (kGeluN + 1));
constexpr size_t kPartBytes =
    align256(sizeof(float) * (size_t)(HCA_MLP_NOALLOC_MAX_BATCH / 64) * kPartialStride);
constexpr size_t kScratchBytes = kOffPart + kPartBytes;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current (it is current: the caller's).
hipError_t scratch_ptr(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return hipSuccess;
}

}  // namespace
}  // namespace hca

using namespace hca;

extern "C" hca_status hca_mlp_gradient_noalloc(const float* theta, const float* Xs,
                                               const float* Ys, int64_t n_rows,
                                               const int32_t* idx, int batch, float* grad,
                                               float* loss, void* stream) {
  if (!theta || !Xs || !Ys || !idx || !grad || n_rows < 1 || n_rows > 0x7fffffffLL)
    return HCA_E_INVALID;
  if (batch < 64 || batch % 64 || batch > HCA_MLP_NOALLOC_MAX_BATCH) {
    fprintf(stderr, "hca_mlp_gradient_noalloc: batch %d is not a positive multiple of 64 "
                    "at most %d\n", batch, HCA_MLP_NOALLOC_MAX_BATCH);
    return HCA_E_RANGE;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HCA_E_DEVICE;
  unsigned char* base = nullptr;
  if (scratch_ptr(dev, &base) != hipSuccess) return HCA_E_DEVICE;
  bf16x8* packed = reinterpret_cast<bf16x8*>(base + kOffPack);
  float2* tab = reinterpret_cast<float2*>(base + kOffTab);
  float* partial = reinterpret_cast<float*>(base + kOffPart);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // every scratch region the later kernels read is written first in this call
  launch_mlp_gelu_table(s, tab);
  launch_mlp_pack(s, theta, packed);
  launch_mlp_grad(s, packed, theta, tab, Xs, Ys, idx, batch, n_rows, partial);
  // update = 0: the parameters and moments are neither read nor written
  launch_mlp_adam(s, const_cast<float*>(theta), nullptr, nullptr, partial, batch / 64, 1, 0.f, 0.9f,
                  0.999f, 1e-8f, 0, grad, loss, batch);
  return hipGetLastError() == hipSuccess ? HCA_OK : HCA_E_DEVICE;
}
