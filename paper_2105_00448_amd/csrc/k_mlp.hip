// ODE surrogate: a 6 -> 64 -> 64 -> 64 -> 3 MLP (GELU, erf form) on BF16
// MFMA with FP32 accumulation, for inference inside the coupled step and for
// training (forward, backward, Adam), plus the kernels that harvest its
// training pairs from the plain integrator.
//
// Formulation: every layer is computed transposed, Y^T = W X^T, with
// v_mfma_f32_32x32x16_bf16: A = weights (rows = output units), B =
// activations (columns = 32 samples), D = next activations.  In D a lane holds
// one sample and rows 8(j/4) + 4h + (j%4) of its column (h = lane/32,
// j = register); registers 8(kb%2)..8(kb%2)+7 of row tile kb/2 are then
// exactly the B operand of k-block kb of the next layer, provided that layer's
// weights are packed with the contraction index in the same order:
//   slot 16 kb + 8h + j  <->  hidden unit 16 kb + 4h + 8(j/4) + (j%4).
// Activations therefore stay in registers through the forward and backward
// passes; the packed A operands (weights for the forward pass, transposed
// weights for the backward pass) are built once per parameter update.
//
// GELU(z) = z Phi(z) with erf from Abramowitz & Stegun 7.1.26 (absolute error
// <= 1.5e-7, far below the bfloat16 rounding of the activations), hardware
// reciprocal and exp2; its derivative Phi(z) + z phi(z) reuses the exponential.
#include <cmath>
#include <type_traits>

#include "dev_util.h"
#include "mlp_dev.h"
#include "ode_dev.h"

namespace hca {

__device__ inline f32x16 mfma16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Output unit of register j of row tile mt in a lane of half h.
__device__ inline int drow(int mt, int j, int h) { return 32 * mt + 8 * (j >> 2) + 4 * h + (j & 3); }

// Hidden unit carried by contraction slot 16 kb + 8h + j.
__device__ inline int perm_slot(int kb, int h, int j) { return 16 * kb + 4 * h + 8 * (j >> 2) + (j & 3); }

template <bool GRAD>
__device__ inline void gelu(float z, float& g, float& dg) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * x);
  const float poly =
      t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  const float e = __builtin_amdgcn_exp2f(z * z * -0.72134752044448170f);   // exp(-z^2/2)
  const float half_erf = 0.5f - 0.5f * poly * e;                          // erf(|z|/sqrt2)/2
  const float Phi = 0.5f + (z < 0.0f ? -half_erf : half_erf);
  g = z * Phi;
  if (GRAD) dg = Phi + z * 0.3989422804014327f * e;
}

// GELU(z) = z Phi(z), Phi interpolated in the LDS copy of the table.
__device__ inline float gelu_lut(const float2* __restrict__ tab, float z) {
  const float u = fminf(fmaxf(fmaf(z, kGeluScale, kGeluOrigin), 0.f), (float)kGeluN);
  const int i = (int)u;
  const float2 e = tab[i];
  return z * fmaf(u - (float)i, e.y, e.x);
}

// Copies the table into LDS (the whole workgroup; synchronise before use).
__device__ inline void load_gelu_table(const float2* __restrict__ g, float2* lds) {
  for (int k = threadIdx.x; k <= kGeluN; k += blockDim.x) lds[k] = g[k];
}

struct Hid {
  __bf16 v[2][16];   // D layout: [row tile][register]
};

__device__ inline bf16x8 bop(const Hid& H, int kb) {
  bf16x8 r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r[j] = H.v[kb >> 1][8 * (kb & 1) + j];
  return r;
}

// ---- packing ----------------------------------------------------------------

// One thread per (MFMA block, lane): the 8 bf16 values lane `lane` feeds as A.
__global__ void k_mlp_pack(const float* __restrict__ th, bf16x8* __restrict__ pk) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= kPackAll) return;
  const int lane = g & 63, m = lane & 31, h = lane >> 5;
  const int blk = g >> 6;
  float v[8];
  if (blk < kPackL2 / 64) {   // W1, row tile blk; contraction over the 6 inputs
    const int o = 32 * blk + m;
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * h + j;
      v[j] = k < kMlpIn ? th[kOW1 + o * kMlpIn + k] : 0.0f;
    }
  } else if (blk < kPackL4 / 64) {   // W2, W3: [row tile][k-block]
    const bool l2 = blk < kPackL3 / 64;
    const int b = blk - (l2 ? kPackL2 : kPackL3) / 64;
    const int mt = b / 4, kb = b % 4, o = 32 * mt + m;
    const float* W = th + (l2 ? kOW2 : kOW3);
    for (int j = 0; j < 8; ++j) v[j] = W[o * kMlpHid + perm_slot(kb, h, j)];
  } else if (blk < kPackFwd / 64) {   // W4: [k-block], rows 0..2 of 32
    const int kb = blk - kPackL4 / 64;
    for (int j = 0; j < 8; ++j) v[j] = m < kMlpOut ? th[kOW4 + m * kMlpHid + perm_slot(kb, h, j)] : 0.0f;
  } else if (blk < kPackL3T / 64) {   // W4^T: [row tile], contraction over the 3 outputs
    const int i = 32 * (blk - kPackL4T / 64) + m;
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * h + j;
      v[j] = k < kMlpOut ? th[kOW4 + k * kMlpHid + i] : 0.0f;
    }
  } else {   // W3^T, W2^T: [row tile][k-block], contraction over the layer's outputs
    const bool l3 = blk < kPackL2T / 64;
    const int b = blk - (l3 ? kPackL3T : kPackL2T) / 64;
    const int mt = b / 4, kb = b % 4, i = 32 * mt + m;
    const float* W = th + (l3 ? kOW3 : kOW2);
    for (int j = 0; j < 8; ++j) v[j] = W[perm_slot(kb, h, j) * kMlpHid + i];
  }
  bf16x8 r;
  for (int j = 0; j < 8; ++j) r[j] = (__bf16)v[j];
  pk[g] = r;
}

__global__ void k_mlp_gelu_table(float2* __restrict__ tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > kGeluN) return;
  auto Phi = [](int k) { return 0.5 * erfc(-((k - (double)kGeluOrigin) / kGeluScale) * 0.70710678118654752); };
  const double a = Phi(i);
  tab[i] = make_float2((float)a, i < kGeluN ? (float)(Phi(i + 1) - a) : 0.f);
}

// ---- forward of one 32-sample tile (one wavefront) ------------------------------

struct Pre {
  f32x16 z[3][2];   // hidden pre-activations (training)
};

// Weight source: A operand of packed block `blk` (kPackL1/64 ...) for this
// lane.  Bias source: accumulator of layer L (0..2), row tile mt, initialised
// with the bias of each D row.
struct GlobalNet {
  const bf16x8* __restrict__ pk;
  const float* __restrict__ th;
  const float2* tab;   // LDS
  int lane;
  __device__ inline float gelu(float z) const { return gelu_lut(tab, z); }
  __device__ inline bf16x8 A(int blk) const { return pk[blk * 64 + lane]; }
  __device__ inline f32x16 bias(int L, int mt) const {
    const float* b = th + (L == 0 ? kOb1 : L == 1 ? kOb2 : kOb3);
    const int h = lane >> 5;
    f32x16 acc;
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = b[drow(mt, j, h)];
    return acc;
  }
  __device__ inline float b4(int o) const { return th[kOb4 + o]; }
};

// The forward operands staged once per workgroup in LDS (22.5 KB of packed
// weights); hidden biases in D-row order, sb[((L*2 + mt)*2 + h)*16 + j].
struct LdsNet {
  const bf16x8* w;     // LDS, kPackFwd
  const float* sb;     // LDS, 192 floats
  const float2* tab;   // LDS
  float ob[kMlpOut];
  int lane;
  __device__ inline float gelu(float z) const { return gelu_lut(tab, z); }
  __device__ inline bf16x8 A(int blk) const { return w[blk * 64 + lane]; }
  __device__ inline f32x16 bias(int L, int mt) const {
    const float4* q = reinterpret_cast<const float4*>(sb + ((L * 2 + mt) * 2 + (lane >> 5)) * 16);
    f32x16 acc;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4 v = q[k];
      acc[4 * k + 0] = v.x;
      acc[4 * k + 1] = v.y;
      acc[4 * k + 2] = v.z;
      acc[4 * k + 3] = v.w;
    }
    return acc;
  }
  __device__ inline float b4(int o) const { return ob[o]; }
};

// xin: layer-1 B operand (lanes of half 0 hold the 6 standardised inputs of
// sample n = lane).  Returns the output accumulator including b4: outputs in
// registers 0..2 of lanes 0..31.
template <bool KEEP, typename NET>
__device__ inline f32x16 mlp_forward_tile(const NET& net, bf16x8 xin, int lane, Pre* pre, Hid* hs) {
  const int h = lane >> 5;
  Hid H;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f32x16 acc = mfma16(net.A(kPackL1 / 64 + mt), xin, net.bias(0, mt));
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (KEEP) pre->z[0][mt][j] = acc[j];
      H.v[mt][j] = (__bf16)net.gelu(acc[j]);
    }
  }
  if (KEEP) hs[0] = H;
#pragma unroll
  for (int L = 1; L < 3; ++L) {
    const int blk = (L == 1 ? kPackL2 : kPackL3) / 64;
    Hid Hn;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      f32x16 acc = net.bias(L, mt);
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) acc = mfma16(net.A(blk + mt * 4 + kb), bop(H, kb), acc);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if (KEEP) pre->z[L][mt][j] = acc[j];
        Hn.v[mt][j] = (__bf16)net.gelu(acc[j]);
      }
    }
    H = Hn;
    if (KEEP) hs[L] = H;
  }
  f32x16 out = {};
  if (h == 0) {
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) out[o] = net.b4(o);
  }
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) out = mfma16(net.A(kPackL4 / 64 + kb), bop(H, kb), out);
  return out;
}

__device__ inline bf16x8 input_operand(const float (&x)[kMlpIn], int h) {
  bf16x8 b;
#pragma unroll
  for (int j = 0; j < 8; ++j) b[j] = (__bf16)((h == 0 && j < kMlpIn) ? x[j] : 0.0f);
  return b;
}

// Network outputs for the 64 samples of a wavefront, sample = lane:
// tile 0 takes lanes 0..31, tile 1 lanes 32..63 (inputs moved down by 32).
template <typename NET>
__device__ inline void forward64(const NET& net, const float (&x)[kMlpIn], int lane,
                                 float (&y)[kMlpOut]) {
  const int h = lane >> 5;
  float x1[kMlpIn];
#pragma unroll
  for (int f = 0; f < kMlpIn; ++f) x1[f] = __shfl(x[f], (lane & 31) + 32, 64);
  const f32x16 o0 = mlp_forward_tile<false>(net, input_operand(x, h), lane, nullptr, nullptr);
  const f32x16 o1 = mlp_forward_tile<false>(net, input_operand(x1, h), lane, nullptr, nullptr);
#pragma unroll
  for (int o = 0; o < kMlpOut; ++o) {
    const float t1 = __shfl(o1[o], lane & 31, 64);
    y[o] = h == 0 ? o0[o] : t1;
  }
}

// Network outputs for one 32-sample tile: sample = lane & 31, inputs taken
// from lanes 0..31, outputs valid in lanes 0..31.
template <typename NET>
__device__ inline void forward32(const NET& net, const float (&x)[kMlpIn], int lane,
                                 float (&y)[kMlpOut]) {
  const f32x16 o = mlp_forward_tile<false>(net, input_operand(x, lane >> 5), lane, nullptr, nullptr);
#pragma unroll
  for (int k = 0; k < kMlpOut; ++k) y[k] = o[k];
}

// ---- surrogate in the coupled step ---------------------------------------------

// Per flat work item, in runs of at most kFlatChunk voxels:
//  0. a deferred solve end (fin) is made on the run's voxels (K, G1 and G2
//     alias fin.x and are not restrict-qualified);
//  1. the item's occupied voxels are listed in LDS, in voxel order;
//  2. each wavefront evaluates the network on 32 listed voxels at a time
//     (one 32-sample MFMA tile; every lane takes part in the GELUs); a voxel
//     takes (P, Vc) += update and, for a cancer cell, phi += update;
//  3. a cancer cell whose predicted phi lands within `margin` of the division
//     threshold 1, or (box mode) a voxel whose inputs leave the training
//     range, is left untouched and listed in fb (slots from the item's first
//     voxel, in any order: voxels are independent); launch_ode_list then
//     advances those by the plain integrator.
// The weights and biases stay in LDS and are re-read on every pass (the
// empty asm with a memory clobber keeps the compiler from hoisting them
// into registers for the whole loop, which took the kernel to one wavefront
// per SIMD); with them in LDS the kernel runs at four.
template <typename T>
__global__ void __launch_bounds__(kBlock, 4) k_mlp_apply(Work w, MlpDev net,
                                                         const uint8_t* __restrict__ L,
                                                         const T* K, const T* G1, const T* G2,
                                                         double* __restrict__ P,
                                                         double* __restrict__ Vc,
                                                         double* __restrict__ phi,
                                                         unsigned long long* __restrict__ part,
                                                         CaList fbl,
                                                         const CgFinish<T>* __restrict__ fin) {
  __shared__ unsigned long long lds4[4];
  __shared__ int list[kFlatChunk];
  __shared__ int wcnt[4];
  __shared__ int n_fb_s;
  __shared__ __attribute__((aligned(16))) float sbias[192];
  __shared__ float2 stab[kGeluN + 1];
  __shared__ bf16x8 sw[kPackFwd];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  load_gelu_table(net.gelu_tab, stab);
  for (int k = threadIdx.x; k < kPackFwd; k += kBlock) sw[k] = net.packed[k];
  for (int k = threadIdx.x; k < 192; k += kBlock) {
    const int j = k & 15, h = (k >> 4) & 1, mt = (k >> 5) & 1, Ly = k >> 6;
    const int ob = Ly == 0 ? kOb1 : Ly == 1 ? kOb2 : kOb3;
    sbias[k] = net.theta[ob + drow(mt, j, h)];
  }
  LdsNet R;
  R.w = sw;
#pragma unroll
  for (int o = 0; o < kMlpOut; ++o) R.ob[o] = net.theta[kOb4 + o];
  R.sb = sbias;
  R.tab = stab;
  R.lane = lane;
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    const long long roff = w.reps[fb.rep].off;
    long long* const slots = fbl.cells + roff + fb.begin;
    unsigned long long n_sur = 0;
    if (threadIdx.x == 0) n_fb_s = 0;
    // the item in runs of at most kFlatChunk voxels (the LDS list size)
    for (long long c0 = fb.begin; c0 < fb.end; c0 += kFlatChunk) {
      const long long off = roff + c0;
      const int len = (int)min((long long)kFlatChunk, fb.end - c0);
      cg_finish_run(fin, fb.rep, off, len);   // 0. published by the listing's barriers
      // 1. list the occupied voxels (index within the run), in order
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
      // 2. network pass, 32 listed voxels per wavefront step (lanes 0..31)
      for (int s0 = 32 * wave; s0 < n; s0 += 32 * (kBlock / 64)) {
        asm volatile("" ::: "memory");   // network operands re-read from LDS per pass
        const int si = s0 + (lane & 31);
        const bool act = si < n && lane < 32;
        const int li = act ? list[si] : 0;
        const long long i = off + li;
        double raw[kMlpIn] = {0, 0, 0, 0, 0, 0};
        uint8_t l = 0;
        if (act) {
          l = L[i];
          raw[0] = K[i];
          raw[1] = G1[i];
          raw[2] = G2[i];
          raw[3] = P[i];
          raw[4] = Vc[i];
          raw[5] = phi[i];
        }
        float x[kMlpIn];
        bool inbox = true;
#pragma unroll
        for (int f = 0; f < kMlpIn; ++f) {
          const float r = (float)raw[f];
          inbox = inbox && r >= net.in_lo[f] && r <= net.in_hi[f];
          x[f] = act ? (r - net.in_mean[f]) * net.in_scale[f] : 0.0f;
        }
        float y[kMlpOut];
        forward32(R, x, lane, y);
        if (!act) continue;
        // the state again (cached) rather than held in registers over the pass
        asm volatile("" ::: "memory");
        const double p0 = P[i], v0 = Vc[i], f0 = phi[i];
        const double dphi = (double)(y[2] * net.out_scale[2] + net.out_mean[2]);
        const bool fallback =
            (net.box && !inbox) || (l == 1 && fabs(f0 + dphi - 1.0) < net.margin);
        if (fallback) {
          slots[atomicAdd(&n_fb_s, 1)] = c0 + li;
        } else {
          P[i] = p0 + (double)(y[0] * net.out_scale[0] + net.out_mean[0]);
          Vc[i] = v0 + (double)(y[1] * net.out_scale[1] + net.out_mean[1]);
          if (l == 1) phi[i] = f0 + dphi;
          ++n_sur;
        }
      }
      __syncthreads();   // the list is rewritten by the next run
    }
    const unsigned long long a = block_sum_u64(n_sur, lds4);
    if (threadIdx.x == 0) {
      const int nfb = n_fb_s;
      fbl.item_n[it] = nfb;
      part[(size_t)it * kCounterSlots + 0] = a;
      part[(size_t)it * kCounterSlots + 1] = (unsigned long long)nfb;
    }
  }
}

// ---- training pairs from the plain integrator -------------------------------------

__global__ void __launch_bounds__(kBlock) k_mlp_count(Work w, const uint8_t* __restrict__ L,
                                                      int* __restrict__ item_cnt) {
  __shared__ unsigned long long lds4[4];
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    const long long off = w.reps[fb.rep].off;
    unsigned long long n = 0;
    for (long long li = fb.begin + threadIdx.x; li < fb.end; li += kBlock) n += L[off + li] != 0;
    const unsigned long long t = block_sum_u64(n, lds4);
    if (threadIdx.x == 0) item_cnt[it] = (int)t;
  }
}

// Exclusive prefix sum of n counts into off[0..n] (off[n] = total), one
// workgroup: each thread sums a contiguous run, the run totals are scanned by
// thread 0 in order, then every run is written.
__global__ void __launch_bounds__(1024) k_mlp_scan(int n, const int* __restrict__ cnt,
                                                   long long* __restrict__ off) {
  __shared__ long long run[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int a = min(n, t * per), b = min(n, a + per);
  long long s = 0;
  for (int i = a; i < b; ++i) s += cnt[i];
  run[t] = s;
  __syncthreads();
  if (t == 0) {
    long long acc = 0;
    for (int k = 0; k < 1024; ++k) {
      const long long v = run[k];
      run[k] = acc;
      acc += v;
    }
    off[n] = acc;
  }
  __syncthreads();
  long long acc = run[t];
  for (int i = a; i < b; ++i) {
    off[i] = acc;
    acc += cnt[i];
  }
}

__global__ void __launch_bounds__(kBlock) k_mlp_save_state(Work w, const double* __restrict__ P,
                                                           const double* __restrict__ Vc,
                                                           const double* __restrict__ phi,
                                                           double* __restrict__ before) {
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    const long long off = w.reps[fb.rep].off;
    for (long long li = fb.begin + threadIdx.x; li < fb.end; li += kBlock) {
      const long long i = off + li;
      before[3 * i + 0] = P[i];
      before[3 * i + 1] = Vc[i];
      before[3 * i + 2] = phi[i];
    }
  }
}

// After the plain ODE phase: row (K, G1, G2, P, Vc, phi)_before ->
// (dP, dVc, dphi) for every occupied voxel, rows in voxel order.  dphi is the
// cycle-clock increment a cancer cell receives at this oxygen (stroma carries
// no clock, but shares the same (K, P, Vc) dynamics, so its rows teach the
// same map).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_mlp_harvest(Work w, DevParams p,
                                                        const uint8_t* __restrict__ L,
                                                        const T* __restrict__ K,
                                                        const T* __restrict__ G1,
                                                        const T* __restrict__ G2,
                                                        const double* __restrict__ P,
                                                        const double* __restrict__ Vc,
                                                        const double* __restrict__ before,
                                                        const long long* __restrict__ item_off,
                                                        float* __restrict__ X, float* __restrict__ Y) {
  __shared__ int wcnt[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    const long long off = w.reps[fb.rep].off;
    long long row0 = item_off[it];
    for (long long base = fb.begin; base < fb.end; base += kBlock) {
      const long long li = base + threadIdx.x;
      const long long i = off + li;
      const bool occ = li < fb.end && L[i] != 0;
      const unsigned long long bal = __ballot(occ);
      const int rank = __popcll(bal & ((1ull << lane) - 1ull));
      if (lane == 0) wcnt[wave] = __popcll(bal);
      __syncthreads();
      int woff = 0;
      for (int k = 0; k < wave; ++k) woff += wcnt[k];
      const int total = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
      __syncthreads();
      if (occ) {
        const long long r = row0 + woff + rank;
        const double kk = K[i];
        float* x = X + r * kMlpIn;
        x[0] = (float)kk;
        x[1] = (float)G1[i];
        x[2] = (float)G2[i];
        x[3] = (float)before[3 * i + 0];
        x[4] = (float)before[3 * i + 1];
        x[5] = (float)before[3 * i + 2];
        float* y = Y + r * kMlpOut;
        y[0] = (float)(P[i] - before[3 * i + 0]);
        y[1] = (float)(Vc[i] - before[3 * i + 1]);
        y[2] = (float)cycle_increment(p.dt, kk, p.T_cycle, p.K_phi);
      }
      row0 += total;
    }
  }
}

// ---- training-set statistics and standardisation ---------------------------------

constexpr int kMomCols = kMlpIn + kMlpOut;
constexpr int kMomRowsPerBlock = 4096;

int mlp_moments_blocks(long long n) {
  long long b = (n + kMomRowsPerBlock - 1) / kMomRowsPerBlock;
  return (int)(b < 1 ? 1 : b > 1024 ? 1024 : b);
}

// Block b: rows [b n / G, (b+1) n / G); per column sum, sum of squares, max
// and max of the negated value (FP64, fixed-order block reductions).
__global__ void __launch_bounds__(kBlock) k_mlp_moments_part(const float* __restrict__ X,
                                                             const float* __restrict__ Y,
                                                             long long n, double* __restrict__ part) {
  __shared__ double lds4[4];
  const long long a = blockIdx.x * n / gridDim.x, b = (blockIdx.x + 1) * n / gridDim.x;
  for (int c = 0; c < kMomCols; ++c) {
    double s = 0.0, s2 = 0.0, mx = -INFINITY, mn = -INFINITY;
    for (long long r = a + threadIdx.x; r < b; r += kBlock) {
      const double v = c < kMlpIn ? X[r * kMlpIn + c] : Y[r * kMlpOut + c - kMlpIn];
      s += v;
      s2 += v * v;
      mx = fmax(mx, v);
      mn = fmax(mn, -v);
    }
    s = block_sum(s, lds4);
    s2 = block_sum(s2, lds4);
    mx = block_max(mx, lds4);
    mn = block_max(mn, lds4);
    if (threadIdx.x == 0) {
      double* o = part + ((size_t)blockIdx.x * kMomCols + c) * 4;
      o[0] = s;
      o[1] = s2;
      o[2] = mx;
      o[3] = mn;
    }
  }
}

__global__ void k_mlp_moments_fin(const double* __restrict__ part, int nblk, long long n,
                                  float* __restrict__ st) {
  const int c = threadIdx.x;
  if (c >= kMomCols) return;
  double s = 0.0, s2 = 0.0, mx = -INFINITY, mn = -INFINITY;
  for (int k = 0; k < nblk; ++k) {
    const double* o = part + ((size_t)k * kMomCols + c) * 4;
    s += o[0];
    s2 += o[1];
    mx = fmax(mx, o[2]);
    mn = fmax(mn, o[3]);
  }
  const double mean = s / (double)n;
  const double var = fmax(s2 / (double)n - mean * mean, 0.0);
  double sd = sqrt(var);
  if (!(sd > 1e-12 * fmax(1.0, fabs(mean)))) sd = 1.0;
  if (c < kMlpIn) {
    st[kStInMean + c] = (float)mean;
    st[kStInScale + c] = (float)(1.0 / sd);
    st[kStInLo + c] = (float)(-mn);
    st[kStInHi + c] = (float)mx;
  } else {
    st[kStOutMean + c - kMlpIn] = (float)mean;
    st[kStOutScale + c - kMlpIn] = (float)sd;
  }
}

__global__ void k_mlp_standardize(const float* __restrict__ X, const float* __restrict__ Y, long long n,
                                  const float* __restrict__ st, float* __restrict__ Xs,
                                  float* __restrict__ Ys) {
  const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int f = 0; f < kMlpIn; ++f)
    Xs[r * kMlpIn + f] = (X[r * kMlpIn + f] - st[kStInMean + f]) * st[kStInScale + f];
  for (int o = 0; o < kMlpOut; ++o)
    Ys[r * kMlpOut + o] = (Y[r * kMlpOut + o] - st[kStOutMean + o]) / st[kStOutScale + o];
}

// ---- initialisation and minibatch sampling ----------------------------------------

// Weights ~ U(-sqrt(3/fan_in), sqrt(3/fan_in)) from Philox counter
// (p, 0, 2, 0), key (seed, 0); biases 0.
__global__ void k_mlp_init(uint64_t seed, float* __restrict__ th) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpNparam) return;
  int fan = 0;
  if (p < kOb1) fan = kMlpIn;
  else if ((p >= kOW2 && p < kOb2) || (p >= kOW3 && p < kOb3) || (p >= kOW4 && p < kOb4)) fan = kMlpHid;
  if (fan == 0) {
    th[p] = 0.0f;
    return;
  }
  const U64x4 r = philox4x64_10((uint64_t)p, 0, 2, 0, seed, 0);
  const double lim = sqrt(3.0 / fan);
  th[p] = (float)((2.0 * unit53(r.v[0]) - 1.0) * lim);
}

// Minibatch t: row indices drawn with replacement, Philox counter
// (j, t, 3, 0), key (seed, 0), reduced modulo n.
__global__ void k_mlp_sample(uint64_t seed, long long t, long long n, int batch, int* __restrict__ idx) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= batch) return;
  const U64x4 r = philox4x64_10((uint64_t)j, (uint64_t)t, 3, 0, seed, 0);
  idx[j] = (int)(r.v[0] % (uint64_t)n);
}

// ---- training: forward + backward of 64 samples per workgroup ------------------

constexpr int kTS = 64;   // samples per workgroup (two wavefronts of 32)

// LDS tiles are [unit][sample] bf16 with 64 samples per row.
__device__ inline void lds_store_tile(__bf16* base, const Hid& H, int lane, int col0) {
  const int h = lane >> 5, n = lane & 31;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int j = 0; j < 16; ++j) base[drow(mt, j, h) * kTS + col0 + n] = H.v[mt][j];
}

__device__ inline bf16x8 lds_row8(const __bf16* base, int row, int col) {
  return *reinterpret_cast<const bf16x8*>(base + row * kTS + col);
}

// Sum over the workgroup's 64 samples of dZ[o][s] H[i][s] for output row
// tile mt and input column tile nt: A = dZ, B = H^T, 4 k-blocks of samples.
__device__ inline f32x16 wgrad_tile(const __bf16* dZ, int nrow_dz, const __bf16* Hm, int nrow_h,
                                    int mt, int nt, int lane) {
  const int h = lane >> 5, m = lane & 31;
  const bf16x8 zero8 = {};
  f32x16 acc = {};
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    const int o = 32 * mt + m, i = 32 * nt + m, col = 16 * kb + 8 * h;
    const bf16x8 a = o < nrow_dz ? lds_row8(dZ, o, col) : zero8;
    const bf16x8 b = i < nrow_h ? lds_row8(Hm, i, col) : zero8;
    acc = mfma16(a, b, acc);
  }
  return acc;
}

// Per-workgroup gradient of the summed loss over samples idx[64 wg .. 64 wg + 63]
// (already divided by 3 x batch), and the workgroup's summed squared error.
// Row indices are clamped to [0, n).
__global__ void __launch_bounds__(128) k_mlp_grad(const bf16x8* __restrict__ pk,
                                                  const float* __restrict__ th,
                                                  const float2* __restrict__ tab,
                                                  const float* __restrict__ Xs,
                                                  const float* __restrict__ Ys,
                                                  const int* __restrict__ idx, int batch,
                                                  long long nrows, float* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) __bf16 sH[3][kMlpHid * kTS];
  __shared__ __attribute__((aligned(16))) __bf16 sX[8 * kTS];
  __shared__ __attribute__((aligned(16))) __bf16 sdZ[3][kMlpHid * kTS];
  __shared__ __attribute__((aligned(16))) __bf16 sdZ4[kMlpOut * kTS];
  __shared__ float sloss[2];
  __shared__ float2 stab[kGeluN + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, n = lane & 31;
  load_gelu_table(tab, stab);
  __syncthreads();
  const int col0 = 32 * wave;
  const long long row = min(max((long long)idx[blockIdx.x * kTS + col0 + n], 0LL), nrows - 1);
  float x[kMlpIn];
#pragma unroll
  for (int f = 0; f < kMlpIn; ++f) x[f] = Xs[row * kMlpIn + f];
  if (h == 0) {
#pragma unroll
    for (int f = 0; f < 8; ++f) sX[f * kTS + col0 + n] = (__bf16)(f < kMlpIn ? x[f] : 0.0f);
  }
  Pre pre;
  Hid hs[3];
  const GlobalNet gnet{pk, th, stab, lane};
  const f32x16 out = mlp_forward_tile<true>(gnet, input_operand(x, h), lane, &pre, hs);
#pragma unroll
  for (int L = 0; L < 3; ++L) lds_store_tile(sH[L], hs[L], lane, col0);
  // dL/dy on the lanes of half 0 (sample n); loss = mean over batch and outputs
  const float inv = 2.0f / (float)(kMlpOut * batch);
  float dy[kMlpOut];
  float l2 = 0.0f;
#pragma unroll
  for (int o = 0; o < kMlpOut; ++o) {
    const float d = out[o] - Ys[row * kMlpOut + o];
    dy[o] = h == 0 ? d * inv : 0.0f;
    l2 += h == 0 ? d * d : 0.0f;
  }
  if (h == 0) {
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) sdZ4[o * kTS + col0 + n] = (__bf16)dy[o];
  }
  bf16x8 bdy;
#pragma unroll
  for (int j = 0; j < 8; ++j) bdy[j] = (__bf16)(j < kMlpOut ? dy[j] : 0.0f);
  // dZ3 = (W4^T dy) * GELU'(z3), then dZ_L = (W_{L+1}^T dZ_{L+1}) * GELU'(z_L)
  Hid dz;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f32x16 acc = {};
    acc = mfma16(pk[kPackL4T + mt * 64 + lane], bdy, acc);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      float g, dg;
      gelu<true>(pre.z[2][mt][j], g, dg);
      dz.v[mt][j] = (__bf16)(acc[j] * dg);
    }
  }
  lds_store_tile(sdZ[2], dz, lane, col0);
#pragma unroll
  for (int L = 2; L >= 1; --L) {
    const int blk = L == 2 ? kPackL3T : kPackL2T;
    Hid nd;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      f32x16 acc = {};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) acc = mfma16(pk[blk + (mt * 4 + kb) * 64 + lane], bop(dz, kb), acc);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        float g, dg;
        gelu<true>(pre.z[L - 1][mt][j], g, dg);
        nd.v[mt][j] = (__bf16)(acc[j] * dg);
      }
    }
    dz = nd;
    lds_store_tile(sdZ[L - 1], dz, lane, col0);
  }
  for (int o = 32; o > 0; o >>= 1) l2 += __shfl_xor(l2, o, 64);
  if (lane == 0) sloss[wave] = l2;
  __syncthreads();
  float* pg = partial + (size_t)blockIdx.x * kPartialStride;
  {   // W4 (3 x 64): wave w takes input column tile w
    const f32x16 acc = wgrad_tile(sdZ4, kMlpOut, sH[2], kMlpHid, 0, wave, lane);
    if (h == 0) {
#pragma unroll
      for (int j = 0; j < kMlpOut; ++j) pg[kOW4 + j * kMlpHid + 32 * wave + n] = acc[j];
    }
  }
#pragma unroll
  for (int L = 2; L >= 1; --L) {   // W3 = dZ3 H2^T, W2 = dZ2 H1^T: wave w takes row tile w
    const int ow = L == 2 ? kOW3 : kOW2;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const f32x16 acc = wgrad_tile(sdZ[L], kMlpHid, sH[L - 1], kMlpHid, wave, nt, lane);
#pragma unroll
      for (int j = 0; j < 16; ++j) pg[ow + drow(wave, j, h) * kMlpHid + 32 * nt + n] = acc[j];
    }
  }
  {   // W1 = dZ1 X^T (64 x 6)
    const f32x16 acc = wgrad_tile(sdZ[0], kMlpHid, sX, kMlpIn, wave, 0, lane);
    if (n < kMlpIn) {
#pragma unroll
      for (int j = 0; j < 16; ++j) pg[kOW1 + drow(wave, j, h) * kMlpIn + n] = acc[j];
    }
  }
  // biases: sums of the dZ rows over the samples
  for (int r = threadIdx.x; r < 3 * kMlpHid + kMlpOut; r += 128) {
    const __bf16* src = r < 3 * kMlpHid ? sdZ[r / kMlpHid] + (r % kMlpHid) * kTS
                                        : sdZ4 + (r - 3 * kMlpHid) * kTS;
    float acc = 0.0f;
    for (int c = 0; c < kTS; ++c) acc += (float)src[c];
    const int ob = r < kMlpHid       ? kOb1 + r
                   : r < 2 * kMlpHid ? kOb2 + r - kMlpHid
                   : r < 3 * kMlpHid ? kOb3 + r - 2 * kMlpHid
                                     : kOb4 + r - 3 * kMlpHid;
    pg[ob] = acc;
  }
  if (threadIdx.x == 0) pg[kMlpNparam] = sloss[0] + sloss[1];
}

// Sums the workgroup partials in workgroup order; with `update`, an Adam step
// with the bias corrections bc1 = 1/(1 - b1^t), bc2 = 1/(1 - b2^t) of step t
// (from the launcher, in FP64: 1 - b2^t evaluated in FP32 would lose about
// 2^-24 / (1 - b2^t) of its relative accuracy to cancellation).  Slot kMlpNparam is the batch's summed
// squared error, reported as the mean loss.
__global__ void k_mlp_adam(float* __restrict__ th, float* __restrict__ m1, float* __restrict__ m2,
                           const float* __restrict__ partial, int nwg, float bc1, float bc2, float lr,
                           float b1, float b2, float eps, int update, float* __restrict__ grad_out,
                           float* __restrict__ loss_out, int batch) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpNparam) return;
  float g = 0.0f;
  for (int k = 0; k < nwg; ++k) g += partial[(size_t)k * kPartialStride + p];
  if (p == kMlpNparam) {
    if (loss_out) *loss_out = g / (float)(kMlpOut * batch);
    return;
  }
  if (grad_out) grad_out[p] = g;
  if (!update) return;
  const float a = b1 * m1[p] + (1.0f - b1) * g;
  const float v = b2 * m2[p] + (1.0f - b2) * g * g;
  m1[p] = a;
  m2[p] = v;
  const float ah = a * bc1;
  const float vh = v * bc2;
  th[p] -= lr * ah / (sqrtf(vh) + eps);
}

// Forward over n rows, 64 per wavefront.  raw = 1: X and Y are model values
// (standardised with the statistics st); raw = 0: standardised values.
__global__ void __launch_bounds__(kBlock) k_mlp_eval(const bf16x8* __restrict__ pk,
                                                     const float* __restrict__ th,
                                                     const float2* __restrict__ tab,
                                                     const float* __restrict__ st,
                                                     const float* __restrict__ X, long long n,
                                                     int raw, float* __restrict__ Y) {
  __shared__ float2 stab[kGeluN + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  load_gelu_table(tab, stab);
  __syncthreads();
  const long long r = (blockIdx.x * 4LL + wave) * 64 + lane;
  float x[kMlpIn];
#pragma unroll
  for (int f = 0; f < kMlpIn; ++f) {
    const float v = r < n ? X[r * kMlpIn + f] : 0.0f;
    x[f] = raw ? (v - st[kStInMean + f]) * st[kStInScale + f] : v;
  }
  float y[kMlpOut];
  const GlobalNet gnet{pk, th, stab, lane};
  forward64(gnet, x, lane, y);
  if (r < n) {
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o)
      Y[r * kMlpOut + o] = raw ? y[o] * st[kStOutScale + o] + st[kStOutMean + o] : y[o];
  }
}

// ---- launchers --------------------------------------------------------------------

void launch_mlp_gelu_table(hipStream_t s, float2* tab) {
  hca_launch(k_mlp_gelu_table, dim3((kGeluN + 1 + 255) / 256), dim3(256), 0, s, tab);
}

void launch_mlp_pack(hipStream_t s, const float* theta, bf16x8* packed) {
  hca_launch(k_mlp_pack, dim3((kPackAll + 255) / 256), dim3(256), 0, s, theta, packed);
}

template <typename T>
void launch_mlp_apply(hipStream_t s, const Work& w, const DevParams& p, const MlpDev& net,
                      const uint8_t* L, const T* K, const T* G1, const T* G2, double* P,
                      double* Vc, double* phi, unsigned long long* part, Counters* cnt, CaList fb,
                      const CgFinish<T>* fin) {
  hca_launch(k_mlp_apply<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, net, L,
             K, G1, G2, P, Vc, phi, part, fb, fin);
  launch_ode_list(s, w, p, L, K, P, Vc, phi, fb);
  launch_counters_reduce(s, w, part, cnt, CNT_SUR);
}

void launch_mlp_count(hipStream_t s, const Work& w, const uint8_t* L, int* item_cnt) {
  hca_launch(k_mlp_count, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, L,
                     item_cnt);
}

void launch_mlp_scan(hipStream_t s, int n, const int* cnt, long long* off) {
  hca_launch(k_mlp_scan, dim3(1), dim3(1024), 0, s, n, cnt, off);
}

void launch_mlp_save_state(hipStream_t s, const Work& w, const double* P, const double* Vc,
                           const double* phi, double* before) {
  hca_launch(k_mlp_save_state, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w,
                     P, Vc, phi, before);
}

template <typename T>
void launch_mlp_harvest(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L,
                        const T* K, const T* G1, const T* G2, const double* P, const double* Vc,
                        const double* before, const long long* item_off, float* X, float* Y) {
  hca_launch(k_mlp_harvest<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p,
                     L, K, G1, G2, P, Vc, before, item_off, X, Y);
}

void launch_mlp_moments(hipStream_t s, const float* X, const float* Y, long long n, double* part,
                        int nblk, float* stats) {
  hca_launch(k_mlp_moments_part, dim3(nblk), dim3(kBlock), 0, s, X, Y, n, part);
  hca_launch(k_mlp_moments_fin, dim3(1), dim3(64), 0, s, part, nblk, n, stats);
}

void launch_mlp_standardize(hipStream_t s, const float* X, const float* Y, long long n,
                            const float* stats, float* Xs, float* Ys) {
  hca_launch(k_mlp_standardize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, Y, n,
                     stats, Xs, Ys);
}

void launch_mlp_init(hipStream_t s, uint64_t seed, float* theta) {
  hca_launch(k_mlp_init, dim3((kMlpNparam + 255) / 256), dim3(256), 0, s, seed, theta);
}

void launch_mlp_sample(hipStream_t s, uint64_t seed, long long t, long long n, int batch, int* idx) {
  hca_launch(k_mlp_sample, dim3((batch + 255) / 256), dim3(256), 0, s, seed, t, n, batch, idx);
}

void launch_mlp_grad(hipStream_t s, const bf16x8* pk, const float* th, const float2* tab,
                     const float* Xs, const float* Ys, const int* idx, int batch, long long nrows,
                     float* partial) {
  hca_launch(k_mlp_grad, dim3(batch / kTS), dim3(128), 0, s, pk, th, tab, Xs, Ys, idx, batch,
                     nrows, partial);
}

void launch_mlp_adam(hipStream_t s, float* th, float* m1, float* m2, const float* partial, int nwg,
                     int t, float lr, float b1, float b2, float eps, int update, float* grad_out,
                     float* loss_out, int batch) {
  const float bc1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)t)));
  const float bc2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)t)));
  hca_launch(k_mlp_adam, dim3((kMlpNparam + 1 + 255) / 256), dim3(256), 0, s, th, m1, m2,
                     partial, nwg, bc1, bc2, lr, b1, b2, eps, update, grad_out, loss_out, batch);
}

void launch_mlp_eval(hipStream_t s, const bf16x8* pk, const float* th, const float2* tab,
                     const float* stats, const float* X, long long n, int raw, float* Y) {
  hca_launch(k_mlp_eval, dim3((unsigned)((n + 255) / 256)), dim3(kBlock), 0, s, pk, th, tab,
                     stats, X, n, raw, Y);
}

#define HCA_MLP_INST(T)                                                                            \
  template void launch_mlp_apply<T>(hipStream_t, const Work&, const DevParams&, const MlpDev&,     \
                                    const uint8_t*, const T*, const T*, const T*, double*,         \
                                    double*, double*, unsigned long long*, Counters*, CaList,      \
                                    const CgFinish<T>*);                                           \
  template void launch_mlp_harvest<T>(hipStream_t, const Work&, const DevParams&, const uint8_t*,  \
                                      const T*, const T*, const T*, const double*, const double*,  \
                                      const double*, const long long*, float*, float*);
HCA_MLP_INST(double)
HCA_MLP_INST(float)

}  // namespace hca
