// Stochastic cellular automaton of the cellular module in three passes whose
// result cannot depend on thread scheduling or tiling (no atomics on the
// state; the only atomic is the position counter of a list whose order does
// not matter):
//
// propose   a cancer cell with phi >= 1 is committed; a scan of the lattice
//           lists the committed cells, and each listed cell decides: one
//           Philox4x64-10 block (key (seed, 0), counter (gid, n+1, KILL, 0))
//           gives one uniform per drug (words 0, 1, and 2 for the third
//           drug); drug i kills with probability I(x_i; 1, b_i) = 1 - (1-x_i)^b_i,
//           x_i = clip(G_i / G_ref_i, 0, 1), the power by repeated products.
//           A surviving cell proposes the empty non-vessel Moore neighbour of
//           highest oxygen (first strict maximum in ascending gid order), else
//           NOSPACE.
// resolve   every proposed site takes, among the neighbours proposing it, the
//           one with the largest phi (Algorithm 2's priority), equal phi ->
//           lowest gid; evaluated by a gather at the site for each of its
//           proposers, which all write the same winner.
// finalize  each voxel applies its own outcome from the codes of the previous
//           passes: killed -> emptied and zeroed; won -> phi = P = Vc = 0;
//           lost or NOSPACE -> phi = 0; daughter site -> cancer with zero state.
//
// Every decision reads the pre-update state (asynchronous rule of the CA
// numerical treatment).  This file is compiled without floating-point
// contraction; decisions use only correctly rounded +, -, *, / and compares.
#include "dev_util.h"

namespace hca {

struct VoxelCoord {
  int x, y, z;
};

__device__ inline VoxelCoord coord_of(long long li, const RepDev& rp) {
  VoxelCoord v;
  if (rp.n <= 0x7fffffffLL) {   // 32-bit arithmetic when the lattice allows it
    const int l = (int)li;
    v.x = l % rp.nx;
    const int t = l / rp.nx;
    v.y = t % rp.ny;
    v.z = t / rp.ny;
    return v;
  }
  v.x = (int)(li % rp.nx);
  const long long t = li / rp.nx;
  v.y = (int)(t % rp.ny);
  v.z = (int)(t / rp.ny);
  return v;
}



__device__ inline bool neighbour(const RepDev& rp, const VoxelCoord& v, int d, long long& nli) {
  int dx, dy, dz;
  moore_offset(d, dx, dy, dz);
  const int x = v.x + dx, y = v.y + dy, z = v.z + dz;
  if (x < 0 || y < 0 || z < 0 || x >= rp.nx || y >= rp.ny || z >= rp.nz) return false;
  nli = x + (long long)rp.nx * (y + (long long)rp.ny * z);
  return true;
}

// Local indices of the 26 Moore neighbours (ascending gid order), -1 outside.
__device__ inline void moore_neighbours(const RepDev& rp, const VoxelCoord& v, long long (&nb)[26]) {
#pragma unroll
  for (int d = 0; d < 26; ++d) {
    long long j;
    nb[d] = neighbour(rp, v, d, j) ? j : -1;
  }
}

// f(rep, replicate, local voxel index) over this workgroup's work items;
// end_item(rep, item) after each item (per-item counter partials).
template <typename F, typename E>
__device__ inline void for_each_voxel_ca(const Work& w, F f, E end_item) {
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    const RepDev rp = w.reps[fb.rep];
    for (long long li = fb.begin + threadIdx.x; li < fb.end; li += kBlock) f(fb.rep, rp, li);
    end_item(fb.rep, it);
  }
}

template <typename F>
__device__ inline void for_each_voxel_ca(const Work& w, F f) {
  for_each_voxel_ca(w, f, [](int, int) {});
}

__device__ inline double kill_probability(double G, double Gref, int b) {
  double x = G / Gref;
  x = x < 0.0 ? 0.0 : x;
  x = x > 1.0 ? 1.0 : x;
  const double y = 1.0 - x;
  double pw = y;
  for (int k = 1; k < b; ++k) pw = pw * y;
  return 1.0 - pw;
}

// Scan: code = win = NONE for every voxel; each work item's committed cancer
// cells (phi >= 1) listed in voxel order in the item's own slots (a
// workgroup prefix sum, no global atomics).  Light, so it runs at full
// occupancy; the gathers of the committed cells' decisions run in the list
// kernels below.
__global__ void __launch_bounds__(kBlock) k_ca_scan(Work w, const uint8_t* __restrict__ L,
                                                    const double* __restrict__ phi,
                                                    uint8_t* __restrict__ code, uint8_t* __restrict__ win,
                                                    CaList list) {
  __shared__ int wcnt[kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    const long long off = w.reps[fb.rep].off;
    long long* slots = list.cells + off + fb.begin;
    int n = 0;
    for (long long base = fb.begin; base < fb.end; base += kBlock) {
      const long long li = base + threadIdx.x;
      bool com = false;
      if (li < fb.end) {
        const long long i = off + li;
        code[i] = kCodeNone;
        win[i] = kCodeNone;
        com = L[i] == 1 && phi[i] >= 1.0;
      }
      const unsigned long long bal = __ballot(com);
      if (lane == 0) wcnt[wave] = __popcll(bal);
      __syncthreads();
      int woff = n;
      for (int k = 0; k < wave; ++k) woff += wcnt[k];
      if (com) slots[woff + __popcll(bal & ((1ull << lane) - 1ull))] = li;
      for (int k = 0; k < kBlock / 64; ++k) n += wcnt[k];
      __syncthreads();
    }
    if (threadIdx.x == 0) list.item_n[it] = n;
  }
}

// The decision of each listed committed cell.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ca_propose_list(Work w, DevParams p,
                                                            const long long* d_step,
                                                            const uint8_t* __restrict__ L,
                                                            const double* __restrict__ vw,
                                                            const T* __restrict__ K,
                                                            const T* __restrict__ G1,
                                                            const T* __restrict__ G2,
                                                            const T* __restrict__ G3,
                                                            CaList list, uint8_t* __restrict__ code) {
  const long long step = d_step[0];
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const int n = list.item_n[it];
    if (n == 0) continue;
    const FlatBlk fb = w.flat[it];
    const RepDev rp = w.reps[fb.rep];
    const long long* slots = list.cells + rp.off + fb.begin;
    for (int k = threadIdx.x; k < n; k += kBlock) {
      const long long li = slots[k];
      const long long i = rp.off + li;
      uint8_t cd;
      const U64x4 o = philox4x64_10((uint64_t)li, (uint64_t)(step + 1), kStreamKill, 0ull, rp.seed, 0ull);
      const double u0 = unit53(o.v[0]), u1 = unit53(o.v[1]);
      const double p1 = kill_probability(G1[i], p.G_ref[0], p.b_int[0]);
      const double p2 = kill_probability(G2[i], p.G_ref[1], p.b_int[1]);
      // the third drug (drug3) draws its trial from the block's third word
      const bool kill3 = p.drug3 && unit53(o.v[2]) < kill_probability(G3[i], p.G_ref3, p.b3);
      if (u0 < p1 || u1 < p2 || kill3) {
        cd = kCodeKill;
      } else {
        const VoxelCoord v = coord_of(li, rp);
        long long nb[26];
        moore_neighbours(rp, v, nb);
        // all neighbour loads issued before any decision (one memory latency)
        uint8_t ln[26];
        double wn[26], kn[26];
  #pragma unroll
        for (int d = 0; d < 26; ++d) {
          const long long j = rp.off + (nb[d] < 0 ? li : nb[d]);
          ln[d] = L[j];
          wn[d] = vw[j];
          kn[d] = K[j];
        }
        double best = -INFINITY;
        cd = kCodeNoSpace;
  #pragma unroll
        for (int d = 0; d < 26; ++d) {
          if (nb[d] < 0 || ln[d] != 0 || wn[d] != 0.0) continue;
          if (kn[d] > best) {
            best = kn[d];
            cd = (uint8_t)d;
          }
        }
      }
      code[i] = cd;
    }
  }
}

// The target site of each listed cell that proposes a daughter: among the
// site's neighbours proposing it, the one with the largest phi (Algorithm 2),
// equal phi -> lowest gid (strict > in ascending gid order).
__global__ void __launch_bounds__(kBlock) k_ca_resolve_list(Work w, const double* __restrict__ phi,
                                                            const uint8_t* __restrict__ code,
                                                            CaList list, uint8_t* __restrict__ win) {
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const int n = list.item_n[it];
    if (n == 0) continue;
    const FlatBlk fb = w.flat[it];
    const RepDev rp = w.reps[fb.rep];
    const long long* slots = list.cells + rp.off + fb.begin;
    for (int k = threadIdx.x; k < n; k += kBlock) {
      const long long li = slots[k];
      const uint8_t cd = code[rp.off + li];
      if (cd >= 26) continue;   // killed or no space
      long long tl = 0;
      neighbour(rp, coord_of(li, rp), cd, tl);   // exists: propose chose it
      long long nb[26];
      moore_neighbours(rp, coord_of(tl, rp), nb);
      uint8_t cn[26];
  #pragma unroll
      for (int d = 0; d < 26; ++d) cn[d] = code[rp.off + (nb[d] < 0 ? tl : nb[d])];
      double best = -INFINITY;
      uint8_t wn = kCodeNone;
  #pragma unroll
      for (int d = 0; d < 26; ++d) {   // ascending parent gid: strict > keeps the lowest
        if (nb[d] < 0 || cn[d] != (uint8_t)moore_opposite(d)) continue;
        const double ph = phi[rp.off + nb[d]];
        if (ph > best) {
          best = ph;
          wn = (uint8_t)d;
        }
      }
      win[rp.off + tl] = wn;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_ca_finalize(Work w, uint8_t* __restrict__ L,
                                                        double* __restrict__ phi,
                                                        double* __restrict__ P,
                                                        double* __restrict__ Vc,
                                                        const uint8_t* __restrict__ code,
                                                        const uint8_t* __restrict__ win,
                                                        unsigned long long* __restrict__ part) {
  __shared__ unsigned long long lds4[4];
  unsigned long long n_com = 0, n_kill = 0, n_div = 0, n_nosp = 0, n_lost = 0;
  for_each_voxel_ca(w, [&](int, const RepDev& rp, long long li) {
    const long long i = rp.off + li;
    const uint8_t cd = code[i];
    const uint8_t wn = win[i];
    if (cd != kCodeNone) {
      ++n_com;
      if (cd == kCodeKill) {
        ++n_kill;
        L[i] = 0;
        phi[i] = 0.0;
        P[i] = 0.0;
        Vc[i] = 0.0;
      } else if (cd == kCodeNoSpace) {
        ++n_nosp;
        phi[i] = 0.0;
      } else {
        const VoxelCoord v = coord_of(li, rp);
        long long nli = 0;
        neighbour(rp, v, cd, nli);
        if (win[rp.off + nli] == (uint8_t)moore_opposite(cd)) {
          ++n_div;
          phi[i] = 0.0;
          P[i] = 0.0;
          Vc[i] = 0.0;
        } else {
          ++n_lost;
          phi[i] = 0.0;
        }
      }
    }
    if (wn != kCodeNone) {
      L[i] = 1;
      phi[i] = 0.0;
      P[i] = 0.0;
      Vc[i] = 0.0;
    }
  }, [&](int, int it) {
    const unsigned long long v[5] = {block_sum_u64(n_com, lds4), block_sum_u64(n_kill, lds4),
                                     block_sum_u64(n_div, lds4), block_sum_u64(n_nosp, lds4),
                                     block_sum_u64(n_lost, lds4)};
    if (threadIdx.x == 0)
      for (int k = 0; k < 5; ++k) part[(size_t)it * kCounterSlots + k] = v[k];
    n_com = n_kill = n_div = n_nosp = n_lost = 0;
  });
}

// Vascular module, Eq. (vascular_module), at the end of the step n -> n+1
// when (n + 1) is a multiple of dv_steps: a vessel whose V lies outside
// [V_low, V_high] is removed with probability p_death; an empty non-vessel
// voxel whose V lies inside becomes a vessel of weight w_new with probability
// birth_per_V V.  One uniform per candidate voxel (Philox key (seed, 0),
// counter (gid, n+1, VESSEL, 0), first word); the event happens when
// u < probability.  The rule is voxel-local and reads the cell map after the
// CA, so the vessel map is updated in place.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_vessel(Work w, DevParams p, const long long* d_step,
                                                   const uint8_t* __restrict__ L,
                                                   const T* __restrict__ V,
                                                   double* __restrict__ vw,
                                                   unsigned long long* __restrict__ part) {
  __shared__ unsigned long long lds4[4];
  const long long step = d_step[0];
  const bool due = (step + 1) % p.dv_steps == 0;
  unsigned long long nb = 0, nd = 0;
  for_each_voxel_ca(w, [&](int, const RepDev& rp, long long li) {
    if (!due) return;
    const long long i = rp.off + li;
    const double wv = vw[i];
    const double v = V[i];
    const bool inside = v >= p.V_low && v <= p.V_high;
    const bool vessel = wv > 0.0;
    const bool candidate = vessel ? !inside : (inside && L[i] == 0);
    if (!candidate) return;
    const U64x4 o = philox4x64_10((uint64_t)li, (uint64_t)(step + 1), kStreamVessel, 0ull, rp.seed, 0ull);
    const double u = unit53(o.v[0]);
    if (vessel) {
      if (u < p.p_death) {
        vw[i] = 0.0;
        ++nd;
      }
    } else if (u < p.birth_per_V * v) {
      vw[i] = p.w_new;
      ++nb;
    }
  }, [&](int, int it) {
    const unsigned long long a = block_sum_u64(nb, lds4), b = block_sum_u64(nd, lds4);
    if (threadIdx.x == 0) {
      part[(size_t)it * kCounterSlots + 0] = a;
      part[(size_t)it * kCounterSlots + 1] = b;
    }
    nb = nd = 0;
  });
}

// Cell-type counts and a non-finite scan of the solved fields (nf x ntot in
// F) and of P, V_c, phi.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_stats(Work w, const uint8_t* __restrict__ L,
                                                  const double* __restrict__ vw,
                                                  const T* __restrict__ F, int nf, long long ntot,
                                                  const double* __restrict__ P,
                                                  const double* __restrict__ Vc,
                                                  const double* __restrict__ phi,
                                                  unsigned long long* __restrict__ part) {
  __shared__ unsigned long long lds4[4];
  unsigned long long nc = 0, ns = 0, ne = 0, nv = 0, bad = 0;
  for_each_voxel_ca(w, [&](int, const RepDev& rp, long long li) {
    const long long i = rp.off + li;
    const uint8_t l = L[i];
    nc += l == 1;
    ns += l == 2;
    ne += l == 0;
    nv += vw[i] != 0.0;
    for (int f = 0; f < nf; ++f) bad += !isfinite(F[i + (long long)f * ntot]);
    bad += !isfinite(P[i]) + !isfinite(Vc[i]) + !isfinite(phi[i]);
  }, [&](int, int it) {
    const unsigned long long v[5] = {block_sum_u64(nc, lds4), block_sum_u64(ns, lds4),
                                     block_sum_u64(ne, lds4), block_sum_u64(nv, lds4),
                                     block_sum_u64(bad, lds4)};
    if (threadIdx.x == 0)
      for (int k = 0; k < 5; ++k) part[(size_t)it * kCounterSlots + k] = v[k];
    nc = ns = ne = nv = bad = 0;
  });
}

// Zero the event counters (events_only) or the state counters.  A kernel,
// not a memset, so the sequence stays safe to capture in a graph.
__global__ void k_zero_counters(Counters* cnt, int nreps, int what) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nreps) return;
  Counters& c = cnt[r];
  if (what == 1) {
    c.committed = c.kills = c.divisions = c.nospace = c.lost = 0;
  } else if (what == 0) {
    c.n_cancer = c.n_stroma = c.n_empty = c.n_vessel = c.nonfinite = 0;
  } else {
    c.sur_voxels = c.sur_fallbacks = 0;
  }
}

// One workgroup per replicate: sums the per-item partials of the
// replicate's flat items in a fixed order into its counters (plain stores, no
// contended atomics; the cumulative totals are added to).
template <int KIND>
__global__ void __launch_bounds__(kBlock) k_counters_reduce(Work w,
                                                            const unsigned long long* __restrict__ part,
                                                            Counters* cnt) {
  __shared__ unsigned long long lds4[4];
  const int rep = blockIdx.x;
  const RepDev rp = w.reps[rep];
  constexpr int K = (KIND == CNT_SUR || KIND == CNT_VESSEL) ? 2 : 5;
  unsigned long long v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0;
  for (int j = threadIdx.x; j < rp.flat_nb; j += kBlock)
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += part[(size_t)(rp.flat_b0 + j) * kCounterSlots + k];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = block_sum_u64(v[k], lds4);
  if (threadIdx.x != 0) return;
  Counters& c = cnt[rep];
  if (KIND == CNT_CA) {
    c.committed = v[0];
    c.kills = v[1];
    c.divisions = v[2];
    c.nospace = v[3];
    c.lost = v[4];
    c.total_kills += v[1];
    c.total_divisions += v[2];
  } else if (KIND == CNT_STATS) {
    c.n_cancer = v[0];
    c.n_stroma = v[1];
    c.n_empty = v[2];
    c.n_vessel = v[3];
    c.nonfinite = v[4];
  } else if (KIND == CNT_VESSEL) {
    c.births = v[0];
    c.deaths = v[1];
    c.total_births += v[0];
    c.total_deaths += v[1];
  } else {
    c.sur_voxels = v[0];
    c.sur_fallbacks = v[1];
  }
}

void launch_counters_reduce(hipStream_t s, const Work& w, const unsigned long long* part,
                            Counters* cnt, int kind) {
  switch (kind) {
    case CNT_CA: hca_launch(k_counters_reduce<CNT_CA>, dim3(w.nreps), dim3(kBlock), 0, s, w, part, cnt); break;
    case CNT_STATS: hca_launch(k_counters_reduce<CNT_STATS>, dim3(w.nreps), dim3(kBlock), 0, s, w, part, cnt); break;
    case CNT_VESSEL: hca_launch(k_counters_reduce<CNT_VESSEL>, dim3(w.nreps), dim3(kBlock), 0, s, w, part, cnt); break;
    default: hca_launch(k_counters_reduce<CNT_SUR>, dim3(w.nreps), dim3(kBlock), 0, s, w, part, cnt); break;
  }
}

__global__ void k_advance(long long* d_step) { d_step[0] += 1; }

// Counts cell codes outside {0,1,2}, cells on vessel voxels and non-finite
// or negative vessel weights of replicate rep.
__global__ void __launch_bounds__(kBlock) k_validate_cells(Work w, const uint8_t* __restrict__ L,
                                                           const double* __restrict__ vw, int rep,
                                                           unsigned long long* bad) {
  unsigned long long nb = 0;
  for_each_voxel_ca(w, [&](int r, const RepDev& rp, long long li) {
    if (r != rep) return;
    const long long i = rp.off + li;
    const uint8_t l = L[i];
    const double wv = vw[i];
    nb += (l > 2) || (l != 0 && wv != 0.0) || !(wv >= 0.0 && isfinite(wv));
  });
  for (int o = 32; o > 0; o >>= 1) nb += __shfl_xor(nb, o, 64);
  if ((threadIdx.x & 63) == 0 && nb) atomicAdd(bad, nb);
}

template <typename T>
void launch_ca_propose(hipStream_t s, const Work& w, const DevParams& p, const long long* d_step,
                       const uint8_t* L, const double* vw, const T* K, const T* G1, const T* G2,
                       const T* G3, const double* phi, uint8_t* code, uint8_t* win, CaList list) {
  hca_launch(k_ca_scan, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, L, phi, code, win, list);
  hca_launch(k_ca_propose_list<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, d_step, L,
             vw, K, G1, G2, G3, list, code);
}

void launch_ca_resolve(hipStream_t s, const Work& w, const double* phi, const uint8_t* code,
                       uint8_t* win, CaList list) {
  hca_launch(k_ca_resolve_list, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, phi, code, list,
             win);
}

void launch_ca_finalize(hipStream_t s, const Work& w, uint8_t* L, double* phi, double* P,
                        double* Vc, const uint8_t* code, const uint8_t* win,
                        unsigned long long* part, Counters* cnt) {
  hca_launch(k_ca_finalize, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, L, phi, P,
             Vc, code, win, part);
  launch_counters_reduce(s, w, part, cnt, CNT_CA);
}

template <typename T>
void launch_vessel(hipStream_t s, const Work& w, const DevParams& p, const long long* d_step,
                   const uint8_t* L, const T* V, double* vw, unsigned long long* part, Counters* cnt) {
  hca_launch(k_vessel<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, d_step, L, V,
             vw, part);
  launch_counters_reduce(s, w, part, cnt, CNT_VESSEL);
}

template <typename T>
void launch_stats(hipStream_t s, const Work& w, const uint8_t* L, const double* vw, const T* F,
                  int nf, long long ntot, const double* P, const double* Vc, const double* phi,
                  unsigned long long* part, Counters* cnt) {
  hca_launch(k_stats<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, L, vw, F, nf,
             ntot, P, Vc, phi, part);
  launch_counters_reduce(s, w, part, cnt, CNT_STATS);
}

void launch_zero_counters(hipStream_t s, Counters* cnt, int nreps, int what) {
  hca_launch(k_zero_counters, dim3((nreps + 63) / 64), dim3(64), 0, s, cnt, nreps, what);
}

void launch_advance(hipStream_t s, long long* d_step) {
  hca_launch(k_advance, dim3(1), dim3(1), 0, s, d_step);
}

void launch_validate_cells(hipStream_t s, const Work& w, const uint8_t* L, const double* vw,
                           int rep, unsigned long long* bad) {
  hca_launch(k_validate_cells, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, L, vw, rep, bad);
}

#define HCA_CA_INST(T)                                                                             \
  template void launch_ca_propose<T>(hipStream_t, const Work&, const DevParams&, const long long*, \
                                     const uint8_t*, const double*, const T*, const T*, const T*,  \
                                     const T*, const double*, uint8_t*, uint8_t*, CaList);         \
  template void launch_vessel<T>(hipStream_t, const Work&, const DevParams&, const long long*,     \
                                 const uint8_t*, const T*, double*, unsigned long long*,           \
                                 Counters*);                                                       \
  template void launch_stats<T>(hipStream_t, const Work&, const uint8_t*, const double*, const T*, \
                                int, long long, const double*, const double*, const double*,       \
                                unsigned long long*, Counters*);
HCA_CA_INST(double)
HCA_CA_INST(float)

}  // namespace hca
