// Shapes, parameter layout and device descriptor of the ODE surrogate network
// (6 -> 64 -> 64 -> 64 -> 3, GELU), shared by its kernels and the runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hca.h"
#include "hca_internal.h"

namespace hca {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMlpIn = HCA_MLP_NIN, kMlpHid = HCA_MLP_NHID, kMlpOut = HCA_MLP_NOUT;
// Flat FP32 parameter vector: W1 (64x6, row = output unit), b1, W2 (64x64),
// b2, W3, b3, W4 (3x64), b4.
constexpr int kOW1 = 0;
constexpr int kOb1 = kOW1 + kMlpHid * kMlpIn;
constexpr int kOW2 = kOb1 + kMlpHid;
constexpr int kOb2 = kOW2 + kMlpHid * kMlpHid;
constexpr int kOW3 = kOb2 + kMlpHid;
constexpr int kOb3 = kOW3 + kMlpHid * kMlpHid;
constexpr int kOW4 = kOb3 + kMlpHid;
constexpr int kOb4 = kOW4 + kMlpOut * kMlpHid;
constexpr int kMlpNparam = kOb4 + kMlpOut;
static_assert(kMlpNparam == HCA_MLP_NPARAM, "parameter count");
// A workgroup's gradient partial: the parameters, then its summed squared error.
constexpr int kPartialStride = kMlpNparam + 1;

// Training-set statistics (FP32, device): x_s = (x - in_mean) * in_scale,
// y = y_s * out_scale + out_mean, and the range of every input column.
constexpr int kStInMean = 0, kStInScale = 6, kStOutMean = 12, kStOutScale = 15, kStInLo = 18,
              kStInHi = 24, kStN = 30;

// Packed MFMA A operands, in bf16x8 units (64 lanes per 32x32x16 block):
// forward W1 [2 row tiles], W2 and W3 [2 x 4 k-blocks], W4 [4 k-blocks];
// backward W4^T [2], W3^T and W2^T [2 x 4].
constexpr int kPackL1 = 0;
constexpr int kPackL2 = kPackL1 + 2 * 64;
constexpr int kPackL3 = kPackL2 + 8 * 64;
constexpr int kPackL4 = kPackL3 + 8 * 64;
constexpr int kPackFwd = kPackL4 + 4 * 64;
constexpr int kPackL4T = kPackFwd;
constexpr int kPackL3T = kPackL4T + 2 * 64;
constexpr int kPackL2T = kPackL3T + 8 * 64;
constexpr int kPackAll = kPackL2T + 8 * 64;

// Normal CDF Phi on [-6, 6] at 64 points per unit (768 intervals): entry i
// holds (Phi(z_i), Phi(z_{i+1}) - Phi(z_i)), z_i = -6 + i/64, the last slope
// 0.  Forward passes evaluate GELU(z) = z Phi(z) by linear interpolation in
// it (error <= 8e-6 in Phi, a few hundredths of a bfloat16 rounding step of
// the activation); outside [-6, 6] Phi is held at its end values.
constexpr int kGeluN = 768;
constexpr float kGeluScale = 64.f, kGeluOrigin = 384.f;

// Everything a kernel needs to evaluate the network on raw model values.
struct MlpDev {
  const bf16x8* packed;       // kPackAll
  const float* theta;         // kMlpNparam (biases are read from here)
  const float2* gelu_tab;     // kGeluN + 1
  float in_mean[kMlpIn], in_scale[kMlpIn];     // x_s = (x - mean) * scale
  float out_mean[kMlpOut], out_scale[kMlpOut]; // y = y_s * scale + mean
  float in_lo[kMlpIn], in_hi[kMlpIn];          // training box
  int box;                    // 1: fall back outside the training box
  double margin;              // fall back when |phi_new - 1| < margin
};

// Launchers (k_mlp.hip).
void launch_mlp_pack(hipStream_t s, const float* theta, bf16x8* packed);
void launch_mlp_gelu_table(hipStream_t s, float2* tab);
// The network's update for every occupied voxel; the voxels that fall back
// are listed in `fb` (per flat work item, as CaList lists cells) and then
// advanced by the plain integrator (launch_ode_list).  fin (device memory, or
// null): a deferred solve end, made per run of voxels before the run's fields
// are read.
template <typename T>
void launch_mlp_apply(hipStream_t s, const Work& w, const DevParams& p, const MlpDev& net,
                      const uint8_t* L, const T* K, const T* G1, const T* G2, double* P,
                      double* Vc, double* phi, unsigned long long* part, Counters* cnt, CaList fb,
                      const CgFinish<T>* fin);
// Training pairs of one coupled step: before the plain ODE phase,
// save_state keeps (P, Vc, phi); after it, harvest writes one row per
// occupied voxel, in voxel order, at row item_off[item] + rank in the item.
void launch_mlp_count(hipStream_t s, const Work& w, const uint8_t* L, int* item_cnt);
void launch_mlp_scan(hipStream_t s, int n, const int* cnt, long long* off);
void launch_mlp_save_state(hipStream_t s, const Work& w, const double* P, const double* Vc,
                           const double* phi, double* before);
template <typename T>
void launch_mlp_harvest(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L,
                        const T* K, const T* G1, const T* G2, const double* P, const double* Vc,
                        const double* before, const long long* item_off, float* X, float* Y);
// Training set statistics: per column mean, scale and range of X (6) and Y (3).
void launch_mlp_moments(hipStream_t s, const float* X, const float* Y, long long n, double* part,
                        int nblk, float* stats);
int mlp_moments_blocks(long long n);
void launch_mlp_standardize(hipStream_t s, const float* X, const float* Y, long long n,
                            const float* stats, float* Xs, float* Ys);
void launch_mlp_init(hipStream_t s, uint64_t seed, float* theta);
void launch_mlp_sample(hipStream_t s, uint64_t seed, long long t, long long n, int batch, int* idx);
void launch_mlp_grad(hipStream_t s, const bf16x8* pk, const float* th, const float2* tab,
                     const float* Xs, const float* Ys, const int* idx, int batch, long long nrows,
                     float* partial);
void launch_mlp_adam(hipStream_t s, float* th, float* m1, float* m2, const float* partial, int nwg,
                     int t, float lr, float b1, float b2, float eps, int update,
                     float* grad_out, float* loss_out, int batch);
void launch_mlp_eval(hipStream_t s, const bf16x8* pk, const float* th, const float2* tab,
                     const float* stats, const float* X, long long n, int raw, float* Y);

}  // namespace hca
