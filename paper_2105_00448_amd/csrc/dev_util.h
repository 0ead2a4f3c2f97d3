// Device helpers: fixed-order workgroup reductions, the per-replicate
// "last workgroup finishes the reduction" handshake, work-item decoding and
// the Philox4x64-10 block function.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hca_internal.h"

namespace hca {

// Sum over a 256-thread workgroup in a fixed order (wavefront butterfly, then
// the four wavefront sums in index order).  Every thread returns the total.
__device__ inline double block_sum(double v, double* lds4) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds4[wave] = v;
  __syncthreads();
  double t = ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
  __syncthreads();
  return t;
}

__device__ inline unsigned long long block_sum_u64(unsigned long long v,
                                                   unsigned long long* lds4) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds4[wave] = v;
  __syncthreads();
  unsigned long long t = lds4[0] + lds4[1] + lds4[2] + lds4[3];
  __syncthreads();
  return t;
}

__device__ inline double block_max(double v, double* lds4) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds4[wave] = v;
  __syncthreads();
  double t = fmax(fmax(lds4[0], lds4[1]), fmax(lds4[2], lds4[3]));
  __syncthreads();
  return t;
}

// Persistent launches: G workgroups cover T work items in contiguous chunks.
// Workgroups are dealt to the 8 XCDs round-robin, so logical block
// lb = (b % 8) * (G / 8) + b / 8 gives each XCD one contiguous run of chunks
// (neighbouring tiles, shared halos in that XCD's L2).
__device__ inline void work_range(int T, int& begin, int& end) {
  const int G = gridDim.x, b = blockIdx.x;
  const int lb = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  begin = (int)((long long)lb * T / G);
  end = (int)((long long)(lb + 1) * T / G);
}

// Stencil tiles: with a grid that is a multiple of 8 * kXcdChunk the tiles
// are dealt to the 8 XCDs in runs of kXcdChunk consecutive tiles, round robin
// (run k to XCD k mod 8), one tile per workgroup: neighbouring tiles share
// their frame rows in one XCD's L2 while every system's tiles still spread
// over all XCDs (systems finish at different iterations).  Otherwise as
// work_range.
__device__ inline void tile_range(int T, int& begin, int& end) {
  const int G = gridDim.x, b = blockIdx.x;
  if (G % (8 * kXcdChunk) == 0) {
    const int x = b % 8, j = b / 8;   // j-th workgroup of XCD x
    const int t = ((j / kXcdChunk) * 8 + x) * kXcdChunk + j % kXcdChunk;
    begin = min(t, T);
    end = min(t + 1, T);
    return;
  }
  work_range(T, begin, end);
}

// Fused-smoothing tiles: workgroup b (dispatched to XCD b mod 8) takes a tile
// of the runs of `chunk` consecutive tiles dealt round robin to the XCDs.  A
// run spans about eight rows of tiles of one z-slab, so the tiles whose
// extended planes overlap (x and y neighbours) mostly run on one XCD at the
// same time and share their halo reads in its L2.  Returns -1 past the end.
__device__ inline int ftile_of(int T, int chunk) {
  const int b = blockIdx.x, x = b % 8, j = b / 8;
  const int t = ((j / chunk) * 8 + x) * chunk + j % chunk;
  return t < T ? t : -1;
}

// A workgroup's three partial sums, stored at its work-item slot (3 doubles);
// a later reduce kernel (one workgroup per replicate) sums the slots of a
// replicate in a fixed order.  The kernel boundary orders the two.
__device__ inline void store_partials(double* slot, double a, double b, double c) {
  if (threadIdx.x == 0) {
    slot[0] = a;
    slot[1] = b;
    slot[2] = c;
  }
}

// A deferred solve end (CgFinish: x += alpha p of each field's last CG
// iteration) on the voxels [off, off + len) of replicate rep, len at most
// kFlatChunk.  Thread t takes the voxels t + k kBlock, every load issued
// before the stores; the caller's next barrier publishes the values to the
// rest of the workgroup.
template <typename T>
__device__ inline void cg_finish_run(const CgFinish<T>* __restrict__ finp, int rep, long long off, int len) {
  if (!finp) return;
  const CgFinish<T> fin = *finp;
  constexpr int kPer = kFlatChunk / kBlock;
  for (int f = 0; f < fin.nf; ++f) {
    const SolveScal* ssr = fin.ss + f * fin.nrep + rep;
    const int n = ssr->it;
    if (n == 0) continue;
    const long long base = (long long)f * fin.ntot + off;
    const T* p = (((n - 1) & 1) ? fin.p0 : fin.p1) + base;   // the direction of iteration n - 1
    T* x = fin.x + base;
    const double alpha = ssr->alpha;
    double xv[kPer], pv[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int li = (int)threadIdx.x + k * kBlock;
      xv[k] = li < len ? (double)x[li] : 0.0;
      pv[k] = li < len ? (double)p[li] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int li = (int)threadIdx.x + k * kBlock;
      if (li < len) x[li] = (T)fma(alpha, pv[k], xv[k]);
    }
  }
}

// ---- Philox4x64-10 (Salmon et al., SC'11) ----------------------------------
struct U64x4 {
  uint64_t v[4];
};

__device__ inline U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                      uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U64x4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

__device__ inline double unit53(uint64_t o) { return (double)(o >> 11) * 0x1.0p-53; }

// Moore neighbour d (0..25, ascending gid order) offsets.
__device__ inline void moore_offset(int d, int& dx, int& dy, int& dz) {
  const int e = d < 13 ? d : d + 1;   // skip the centre (13)
  dz = e / 9 - 1;
  dy = (e / 3) % 3 - 1;
  dx = e % 3 - 1;
}

__device__ inline int moore_opposite(int d) { return 25 - d; }

}  // namespace hca
