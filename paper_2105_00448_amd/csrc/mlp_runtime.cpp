// Host side of surrogate training: the hca_mlp_trainer object (standardised
// training set, statistics, parameters, Adam moments) and its C ABI.  All
// arithmetic runs in the k_mlp.hip kernels; this file only sequences them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "hca.h"
#include "mlp_dev.h"

using namespace hca;

struct hca_mlp_trainer {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  long long n = 0;
  uint64_t seed = 0;
  float *Xs = nullptr, *Ys = nullptr;   // standardised rows
  float* stats = nullptr;               // kStN
  float *theta = nullptr, *m1 = nullptr, *m2 = nullptr;
  bf16x8* packed = nullptr;
  float2* gelu_tab = nullptr;           // kGeluN + 1
  float* partial = nullptr;             // kMaxBatch / 64 workgroups
  int* idx = nullptr;                   // kMaxBatch
  float* losses = nullptr;              // device, grows with n_steps
  int losses_cap = 0;
  float* loss1 = nullptr;               // device scalar
  long long t = 0;                      // Adam steps taken
  float h_stats[kStN] = {0};
  std::string err;
};

namespace {

constexpr int kMaxBatch = 65536;

hca_status tfail(hca_mlp_trainer* t, hca_status st, const std::string& msg) {
  if (t) t->err = msg;
  return st;
}

#define TCHK(t, expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return tfail(t, e_ == hipErrorOutOfMemory ? HCA_E_NOMEM : HCA_E_DEVICE,           \
                   std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

template <typename T>
hipError_t talloc(T** p, size_t count) {
  return hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
}

void tfree(hca_mlp_trainer* t) {
  void* bufs[] = {t->Xs, t->Ys, t->stats, t->theta, t->m1, t->m2, (void*)t->packed, t->gelu_tab,
                  t->partial, t->idx, t->losses, t->loss1};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  if (t->own_stream && t->stream) (void)hipStreamDestroy(t->stream);
}

hca_status reset_adam(hca_mlp_trainer* t) {
  TCHK(t, hipMemsetAsync(t->m1, 0, sizeof(float) * kMlpNparam, t->stream));
  TCHK(t, hipMemsetAsync(t->m2, 0, sizeof(float) * kMlpNparam, t->stream));
  t->t = 0;
  return HCA_OK;
}

}  // namespace

extern "C" {

hca_status hca_mlp_trainer_create(hca_mlp_trainer** out, const float* X, const float* Y,
                                  int64_t n_rows, uint64_t seed, void* stream) {
  if (!out || !X || !Y || n_rows < 1 || n_rows > 0x7fffffffLL) return HCA_E_INVALID;
  *out = nullptr;
  hca_mlp_trainer* t = new (std::nothrow) hca_mlp_trainer();
  if (!t) return HCA_E_NOMEM;
  auto bail = [&](hca_status st) {
    if (!t->err.empty()) fprintf(stderr, "hca_mlp_trainer_create: %s\n", t->err.c_str());
    tfree(t);
    delete t;
    return st;
  };
  t->n = n_rows;
  t->seed = seed;
  if (stream) {
    t->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&t->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(HCA_E_DEVICE);
    t->own_stream = true;
  }
  const size_t n = (size_t)n_rows;
  const int nblk = mlp_moments_blocks(n_rows);
  double* part = nullptr;
  if (talloc(&t->Xs, n * kMlpIn) != hipSuccess || talloc(&t->Ys, n * kMlpOut) != hipSuccess)
    return bail(HCA_E_NOMEM);
  if (talloc(&t->stats, kStN) != hipSuccess || talloc(&t->theta, kMlpNparam) != hipSuccess ||
      talloc(&t->m1, kMlpNparam) != hipSuccess || talloc(&t->m2, kMlpNparam) != hipSuccess ||
      talloc(&t->packed, kPackAll) != hipSuccess || talloc(&t->gelu_tab, kGeluN + 1) != hipSuccess ||
      talloc(&t->partial, (size_t)(kMaxBatch / 64) * kPartialStride) != hipSuccess ||
      talloc(&t->idx, kMaxBatch) != hipSuccess || talloc(&t->loss1, 1) != hipSuccess ||
      talloc(&part, (size_t)nblk * (kMlpIn + kMlpOut) * 4) != hipSuccess) {
    if (part) (void)hipFree(part);
    return bail(HCA_E_NOMEM);
  }
  launch_mlp_moments(t->stream, X, Y, n_rows, part, nblk, t->stats);
  launch_mlp_standardize(t->stream, X, Y, n_rows, t->stats, t->Xs, t->Ys);
  launch_mlp_init(t->stream, seed, t->theta);
  launch_mlp_gelu_table(t->stream, t->gelu_tab);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(t->h_stats, t->stats, sizeof t->h_stats, hipMemcpyDeviceToHost, t->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
  (void)hipFree(part);
  if (e != hipSuccess) {
    t->err = hipGetErrorString(e);
    return bail(HCA_E_DEVICE);
  }
  for (float v : t->h_stats)
    if (!std::isfinite(v)) {
      t->err = "training set has non-finite values";
      return bail(HCA_E_NONFINITE);
    }
  if (reset_adam(t) != HCA_OK) return bail(HCA_E_DEVICE);
  *out = t;
  return HCA_OK;
}

hca_status hca_mlp_trainer_set_params(hca_mlp_trainer* t, const float* theta, int is_device) {
  if (!t || !theta) return HCA_E_INVALID;
  TCHK(t, hipMemcpyAsync(t->theta, theta, sizeof(float) * kMlpNparam,
                         is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, t->stream));
  hca_status st = reset_adam(t);
  if (st != HCA_OK) return st;
  TCHK(t, hipStreamSynchronize(t->stream));
  return HCA_OK;
}

hca_status hca_mlp_trainer_params(hca_mlp_trainer* t, float* theta, int is_device) {
  if (!t || !theta) return HCA_E_INVALID;
  TCHK(t, hipMemcpyAsync(theta, t->theta, sizeof(float) * kMlpNparam,
                         is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, t->stream));
  TCHK(t, hipStreamSynchronize(t->stream));
  return HCA_OK;
}

hca_status hca_mlp_trainer_data(hca_mlp_trainer* t, float* Xs, float* Ys) {
  if (!t || !Xs || !Ys) return HCA_E_INVALID;
  TCHK(t, hipMemcpyAsync(Xs, t->Xs, sizeof(float) * kMlpIn * t->n, hipMemcpyDeviceToDevice, t->stream));
  TCHK(t, hipMemcpyAsync(Ys, t->Ys, sizeof(float) * kMlpOut * t->n, hipMemcpyDeviceToDevice, t->stream));
  TCHK(t, hipStreamSynchronize(t->stream));
  return HCA_OK;
}

hca_status hca_mlp_trainer_export(hca_mlp_trainer* t, hca_mlp* out) {
  if (!t || !out) return HCA_E_INVALID;
  out->theta = t->theta;
  out->theta_is_device = 1;
  for (int f = 0; f < kMlpIn; ++f) {
    out->in_mean[f] = t->h_stats[kStInMean + f];
    out->in_scale[f] = t->h_stats[kStInScale + f];
    out->in_lo[f] = t->h_stats[kStInLo + f];
    out->in_hi[f] = t->h_stats[kStInHi + f];
  }
  for (int o = 0; o < kMlpOut; ++o) {
    out->out_mean[o] = t->h_stats[kStOutMean + o];
    out->out_scale[o] = t->h_stats[kStOutScale + o];
  }
  out->box_check = 0;
  return HCA_OK;
}

hca_status hca_mlp_gradient(hca_mlp_trainer* t, const int32_t* idx, int batch, float* grad,
                            float* loss) {
  if (!t || !idx || !grad) return HCA_E_INVALID;
  if (batch < 64 || batch > kMaxBatch || batch % 64) return tfail(t, HCA_E_RANGE, "batch size");
  launch_mlp_pack(t->stream, t->theta, t->packed);
  launch_mlp_grad(t->stream, t->packed, t->theta, t->gelu_tab, t->Xs, t->Ys, idx, batch, t->n, t->partial);
  launch_mlp_adam(t->stream, t->theta, t->m1, t->m2, t->partial, batch / 64, 1, 0.f, 0.9f, 0.999f,
                  1e-8f, 0, grad, t->loss1, batch);
  TCHK(t, hipGetLastError());
  float l = 0.f;
  TCHK(t, hipMemcpyAsync(&l, t->loss1, sizeof l, hipMemcpyDeviceToHost, t->stream));
  TCHK(t, hipStreamSynchronize(t->stream));
  if (loss) *loss = l;
  return HCA_OK;
}

hca_status hca_mlp_train(hca_mlp_trainer* t, int n_steps, int batch, float lr, float* losses) {
  if (!t || n_steps < 0 || !std::isfinite(lr) || lr <= 0.f) return HCA_E_INVALID;
  if (batch < 64 || batch > kMaxBatch || batch % 64) return tfail(t, HCA_E_RANGE, "batch size");
  if (n_steps == 0) return HCA_OK;
  if (t->losses_cap < n_steps) {
    if (t->losses) (void)hipFree(t->losses);
    t->losses = nullptr;
    t->losses_cap = 0;
    TCHK(t, talloc(&t->losses, (size_t)n_steps));
    t->losses_cap = n_steps;
  }
  for (int k = 0; k < n_steps; ++k) {
    const long long step = t->t + 1;
    launch_mlp_sample(t->stream, t->seed, step, t->n, batch, t->idx);
    launch_mlp_pack(t->stream, t->theta, t->packed);
    launch_mlp_grad(t->stream, t->packed, t->theta, t->gelu_tab, t->Xs, t->Ys, t->idx, batch, t->n, t->partial);
    launch_mlp_adam(t->stream, t->theta, t->m1, t->m2, t->partial, batch / 64, (int)step, lr, 0.9f,
                    0.999f, 1e-8f, 1, nullptr, t->losses + k, batch);
    t->t = step;
  }
  TCHK(t, hipGetLastError());
  if (losses)
    TCHK(t, hipMemcpyAsync(losses, t->losses, sizeof(float) * n_steps, hipMemcpyDeviceToHost,
                           t->stream));
  TCHK(t, hipStreamSynchronize(t->stream));
  return HCA_OK;
}

hca_status hca_mlp_apply_gradient(hca_mlp_trainer* t, const float* grad, int is_device, float lr) {
  if (!t || !grad || !std::isfinite(lr) || lr <= 0.f) return HCA_E_INVALID;
  // the gradient takes the place of a single workgroup partial (its loss
  // slot is not read: no loss is reported)
  TCHK(t, hipMemcpyAsync(t->partial, grad, sizeof(float) * kMlpNparam,
                         is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, t->stream));
  const long long step = t->t + 1;
  launch_mlp_adam(t->stream, t->theta, t->m1, t->m2, t->partial, 1, (int)step, lr, 0.9f, 0.999f,
                  1e-8f, 1, nullptr, nullptr, 1);
  TCHK(t, hipGetLastError());
  TCHK(t, hipStreamSynchronize(t->stream));
  t->t = step;
  return HCA_OK;
}

hca_status hca_mlp_eval(hca_mlp_trainer* t, const float* X, int64_t n, int raw, float* Y) {
  if (!t || !X || !Y || n < 0) return HCA_E_INVALID;
  if (n == 0) return HCA_OK;
  launch_mlp_pack(t->stream, t->theta, t->packed);
  launch_mlp_eval(t->stream, t->packed, t->theta, t->gelu_tab, t->stats, X, n, raw ? 1 : 0, Y);
  TCHK(t, hipGetLastError());
  TCHK(t, hipStreamSynchronize(t->stream));
  return HCA_OK;
}

const char* hca_mlp_trainer_last_error(const hca_mlp_trainer* t) { return t ? t->err.c_str() : ""; }

void hca_mlp_trainer_destroy(hca_mlp_trainer* t) {
  if (!t) return;
  (void)hipStreamSynchronize(t->stream);
  tfree(t);
  delete t;
}

}  // extern "C"
