// The C ABI of include/hca.h for contexts: each call goes to the runtime
// instance of the context's storage precision (hca::rt64 for 64, hca::rt32
// for 32), chosen at init from hca_params.precision.
#include "rt_api.h"

#define HCA_DISPATCH(c, call) ((c)->precision == 32 ? hca::rt32::call : hca::rt64::call)

extern "C" {

hca_status hca_init(hca_ctx** out, const hca_params* p, const hca_replicate* reps, int n_reps,
                    void* stream) {
  if (!out || !p) return HCA_E_INVALID;
  if (p->precision == 32) return hca::rt32::api_init(out, p, reps, n_reps, stream);
  if (p->precision == 64) return hca::rt64::api_init(out, p, reps, n_reps, stream);
  *out = nullptr;
  return HCA_E_INVALID;
}

hca_status hca_init_from_state(hca_ctx** out, const hca_params* p, const hca_replicate* reps,
                               const void* const* states, const size_t* state_bytes, int n_reps,
                               void* stream) {
  if (!out || !p) return HCA_E_INVALID;
  if (p->precision == 32)
    return hca::rt32::api_init_from_state(out, p, reps, states, state_bytes, n_reps, stream);
  if (p->precision == 64)
    return hca::rt64::api_init_from_state(out, p, reps, states, state_bytes, n_reps, stream);
  *out = nullptr;
  return HCA_E_INVALID;
}

hca_status hca_run_phases(hca_ctx* c, unsigned mask) {
  return c ? HCA_DISPATCH(c, api_run_phases(c, mask)) : HCA_E_INVALID;
}

hca_status hca_step(hca_ctx* c, int n_steps) {
  return c ? HCA_DISPATCH(c, api_step(c, n_steps)) : HCA_E_INVALID;
}

hca_status hca_fields(hca_ctx* c, int rep, hca_field f, void* dst, size_t dst_bytes,
                      int dst_is_device) {
  return c ? HCA_DISPATCH(c, api_fields(c, rep, f, dst, dst_bytes, dst_is_device)) : HCA_E_INVALID;
}

hca_status hca_set_field(hca_ctx* c, int rep, hca_field f, const void* src, size_t src_bytes,
                         int src_is_device) {
  return c ? HCA_DISPATCH(c, api_set_field(c, rep, f, src, src_bytes, src_is_device)) : HCA_E_INVALID;
}

hca_status hca_set_step(hca_ctx* c, int64_t step) {
  return c ? HCA_DISPATCH(c, api_set_step(c, step)) : HCA_E_INVALID;
}

hca_status hca_state_bytes(hca_ctx* c, int rep, size_t* bytes) {
  return c ? HCA_DISPATCH(c, api_state_bytes(c, rep, bytes)) : HCA_E_INVALID;
}

hca_status hca_export_state(hca_ctx* c, int rep, void* dst, size_t dst_bytes, int dst_is_device) {
  return c ? HCA_DISPATCH(c, api_export_state(c, rep, dst, dst_bytes, dst_is_device)) : HCA_E_INVALID;
}

hca_status hca_import_state(hca_ctx* c, int rep, const void* src, size_t src_bytes,
                            int src_is_device) {
  return c ? HCA_DISPATCH(c, api_import_state(c, rep, src, src_bytes, src_is_device)) : HCA_E_INVALID;
}

hca_status hca_stats(hca_ctx* c, int rep, hca_stats_t* out) {
  return c ? HCA_DISPATCH(c, api_stats(c, rep, out)) : HCA_E_INVALID;
}

hca_status hca_kernel_time(hca_ctx* c, int kernel, double* ms, int64_t* launches,
                           double* bytes_per_launch) {
  return c ? HCA_DISPATCH(c, api_kernel_time(c, kernel, ms, launches, bytes_per_launch))
           : HCA_E_INVALID;
}

hca_status hca_set_profile(hca_ctx* c, int profile) {
  return c ? HCA_DISPATCH(c, api_set_profile(c, profile)) : HCA_E_INVALID;
}

hca_status hca_reset_kernel_time(hca_ctx* c) {
  return c ? HCA_DISPATCH(c, api_reset_kernel_time(c)) : HCA_E_INVALID;
}

hca_status hca_tile_shape(hca_ctx* c, int rep, int32_t* tx, int32_t* ty, int32_t* tz) {
  return c ? HCA_DISPATCH(c, api_tile_shape(c, rep, tx, ty, tz)) : HCA_E_INVALID;
}

hca_status hca_set_surrogate(hca_ctx* c, const hca_mlp* net, double margin) {
  return c ? HCA_DISPATCH(c, api_set_surrogate(c, net, margin)) : HCA_E_INVALID;
}

hca_status hca_harvest_step(hca_ctx* c, float* X, float* Y, int64_t cap_rows, int64_t* n_rows) {
  return c ? HCA_DISPATCH(c, api_harvest_step(c, X, Y, cap_rows, n_rows)) : HCA_E_INVALID;
}

hca_status hca_synchronize(hca_ctx* c) {
  return c ? HCA_DISPATCH(c, api_synchronize(c)) : HCA_E_INVALID;
}

const char* hca_last_error(const hca_ctx* c) {
  return c ? HCA_DISPATCH(c, api_last_error(c)) : "";
}

void hca_destroy(hca_ctx* c) {
  if (!c) return;
  if (c->precision == 32)
    hca::rt32::api_destroy(c);
  else
    hca::rt64::api_destroy(c);
}

}  // extern "C"
