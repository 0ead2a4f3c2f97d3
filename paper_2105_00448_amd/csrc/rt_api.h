// The context-level entry points of one runtime instance (runtime.cpp,
// compiled once per storage precision into hca::rt64 and hca::rt32); the C
// ABI in capi.cpp forwards each call to the instance that owns the context.
#pragma once

#include "hca.h"
#include "hca_internal.h"

#define HCA_RT_API_DECL(NS)                                                                        \
  namespace hca {                                                                                  \
  namespace NS {                                                                                   \
  hca_status api_init(::hca_ctx** out, const hca_params* p, const hca_replicate* reps, int n_reps, \
                      void* stream);                                                               \
  hca_status api_init_from_state(::hca_ctx** out, const hca_params* p,                             \
                                 const hca_replicate* reps, const void* const* states,             \
                                 const size_t* state_bytes, int n_reps, void* stream);             \
  hca_status api_run_phases(::hca_ctx* c, unsigned mask);                                          \
  hca_status api_step(::hca_ctx* c, int n_steps);                                                  \
  hca_status api_fields(::hca_ctx* c, int rep, hca_field f, void* dst, size_t dst_bytes,           \
                        int dst_is_device);                                                        \
  hca_status api_set_field(::hca_ctx* c, int rep, hca_field f, const void* src, size_t src_bytes,  \
                           int src_is_device);                                                     \
  hca_status api_set_step(::hca_ctx* c, int64_t step);                                             \
  hca_status api_state_bytes(::hca_ctx* c, int rep, size_t* bytes);                                \
  hca_status api_export_state(::hca_ctx* c, int rep, void* dst, size_t dst_bytes,                  \
                              int dst_is_device);                                                  \
  hca_status api_import_state(::hca_ctx* c, int rep, const void* src, size_t src_bytes,            \
                              int src_is_device);                                                  \
  hca_status api_stats(::hca_ctx* c, int rep, hca_stats_t* out);                                   \
  hca_status api_kernel_time(::hca_ctx* c, int kernel, double* ms, int64_t* launches,              \
                             double* bytes_per_launch);                                            \
  hca_status api_set_profile(::hca_ctx* c, int profile);                                           \
  hca_status api_reset_kernel_time(::hca_ctx* c);                                                  \
  hca_status api_tile_shape(::hca_ctx* c, int rep, int32_t* tx, int32_t* ty, int32_t* tz);         \
  hca_status api_set_surrogate(::hca_ctx* c, const hca_mlp* net, double margin);                   \
  hca_status api_harvest_step(::hca_ctx* c, float* X, float* Y, int64_t cap_rows,                  \
                              int64_t* n_rows);                                                    \
  hca_status api_synchronize(::hca_ctx* c);                                                        \
  const char* api_last_error(const ::hca_ctx* c);                                                  \
  void api_destroy(::hca_ctx* c);                                                                  \
  }                                                                                                \
  }

HCA_RT_API_DECL(rt64)
HCA_RT_API_DECL(rt32)
