// Intracellular module over one coupled step for every occupied voxel: the
// plain integrator of ode_dev.h, FP64, bound by the vector ALU (about 120
// divides per voxel).  Each workgroup first lists the occupied voxels of its
// run of the lattice in LDS, so every lane of a wavefront integrates an
// occupied voxel (empty voxels would otherwise idle half the lanes at the
// typical occupancy of one half).
#include "dev_util.h"
#include "ode_dev.h"

namespace hca {

// fin: a deferred solve end, made per run before its listing (K aliases
// fin.x, so K is not restrict-qualified).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ode(Work w, DevParams p, const uint8_t* __restrict__ L,
                                                const T* K,
                                                double* __restrict__ P,
                                                double* __restrict__ Vc,
                                                double* __restrict__ phi,
                                                const CgFinish<T>* __restrict__ fin) {
  __shared__ int list[kFlatChunk];
  __shared__ int wcnt[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    for (long long c0 = fb.begin; c0 < fb.end; c0 += kFlatChunk) {
      const long long off = w.reps[fb.rep].off + c0;
      const int len = (int)min((long long)kFlatChunk, fb.end - c0);
      cg_finish_run(fin, fb.rep, off, len);   // published by the listing's barriers
      int n = 0;
      for (int base = 0; base < len; base += kBlock) {
        const int li = base + (int)threadIdx.x;
        const bool occ = li < len && L[off + li] != 0;
        const unsigned long long bal = __ballot(occ);
        const int rank = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wcnt[wave] = __popcll(bal);
        __syncthreads();
        int woff = 0;
        for (int k = 0; k < wave; ++k) woff += wcnt[k];
        if (occ) list[n + woff + rank] = li;
        n += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        __syncthreads();
      }
      for (int s = threadIdx.x; s < n; s += kBlock) {
        const long long i = off + list[s];
        const uint8_t l = L[i];
        double pv = P[i], vv = Vc[i], ph = phi[i];
        ode_voxel(p, l, K[i], pv, vv, ph);
        P[i] = pv;
        Vc[i] = vv;
        if (l == 1) phi[i] = ph;
      }
      __syncthreads();   // the list is rewritten by the next run
    }
  }
}

template <typename T>
void launch_ode(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L, const T* K,
                double* P, double* Vc, double* phi, const CgFinish<T>* fin) {
  hca_launch(k_ode<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, L, K, P, Vc, phi,
             fin);
}

// The plain integrator on listed voxels only: flat work item it's voxels
// (local indices) at list.cells[first voxel of the item ...], list.item_n[it]
// of them (the surrogate's fallback voxels).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ode_list(Work w, DevParams p, const uint8_t* __restrict__ L,
                                                     const T* __restrict__ K, double* __restrict__ P,
                                                     double* __restrict__ Vc, double* __restrict__ phi,
                                                     CaList list) {
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const int n = list.item_n[it];
    if (n == 0) continue;
    const FlatBlk fb = w.flat[it];
    const RepDev rp = w.reps[fb.rep];
    const long long* slots = list.cells + rp.off + fb.begin;
    for (int k = threadIdx.x; k < n; k += kBlock) {
      const long long i = rp.off + slots[k];
      const uint8_t l = L[i];
      double pv = P[i], vv = Vc[i], ph = phi[i];
      ode_voxel(p, l, K[i], pv, vv, ph);
      P[i] = pv;
      Vc[i] = vv;
      if (l == 1) phi[i] = ph;
    }
  }
}

template <typename T>
void launch_ode_list(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L, const T* K,
                     double* P, double* Vc, double* phi, CaList list) {
  hca_launch(k_ode_list<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, L, K, P, Vc,
             phi, list);
}

template void launch_ode_list<double>(hipStream_t, const Work&, const DevParams&, const uint8_t*,
                                      const double*, double*, double*, double*, CaList);
template void launch_ode_list<float>(hipStream_t, const Work&, const DevParams&, const uint8_t*,
                                     const float*, double*, double*, double*, CaList);
template void launch_ode<double>(hipStream_t, const Work&, const DevParams&, const uint8_t*,
                                 const double*, double*, double*, double*, const CgFinish<double>*);
template void launch_ode<float>(hipStream_t, const Work&, const DevParams&, const uint8_t*,
                                const float*, double*, double*, double*, const CgFinish<float>*);

}  // namespace hca
