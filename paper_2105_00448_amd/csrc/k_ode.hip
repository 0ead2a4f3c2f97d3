// Intracellular module over one coupled step for every occupied voxel: the
// plain integrator of ode_dev.h.  FP64; the kernel is bound by the VALU
// (about 120 divides per voxel).
#include "dev_util.h"
#include "ode_dev.h"

namespace hca {

__global__ void __launch_bounds__(kBlock) k_ode(Work w, DevParams p, const uint8_t* __restrict__ L,
                                                const double* __restrict__ K,
                                                double* __restrict__ P,
                                                double* __restrict__ Vc,
                                                double* __restrict__ phi) {
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    const long long off = w.reps[fb.rep].off;
    for (long long li = fb.begin + threadIdx.x; li < fb.end; li += kBlock) {
      const long long i = off + li;
      const uint8_t l = L[i];
      if (l == 0) continue;
      double pv = P[i], vv = Vc[i], ph = phi[i];
      ode_voxel(p, l, K[i], pv, vv, ph);
      P[i] = pv;
      Vc[i] = vv;
      if (l == 1) phi[i] = ph;
    }
  }
}

void launch_ode(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L,
                const double* K, double* P, double* Vc, double* phi) {
  hipLaunchKernelGGL(k_ode, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, L, K,
                     P, Vc, phi);
}

}  // namespace hca
