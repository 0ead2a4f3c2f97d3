// Plasma kinetics, coefficient / right-hand-side setup of the implicit-Euler
// systems, and the cell-state initialisation of Algorithm 1.
//
// Every implicit-Euler update of Eqs. (oxygen) and (chemo) on the voxel
// lattice is   c_i u_i - a (Lap u)_i = b_i   with a = D/h^2 and the
// zero-flux 7-point Laplacian; these kernels produce c and b per voxel.
#include "dev_util.h"

namespace hca {

// G_{i,0}(t^{n+1}) of both drugs for every replicate: a_m G_ref e^{-k (t - t_m)}
// for the latest bolus t_m <= t (reset at each dose), 0 before the first dose.
// One-compartment linear elimination (Eq. intrachemo3; the fluorouracil model
// in its linear regime).
__global__ void k_plasma(int nreps, const RepDev* reps, DevParams p, const long long* d_step,
                         const double* dose_t, const double* dose_a, double* g0) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nreps) return;
  const double t = (double)(d_step[0] + 1) * p.dt;
  const RepDev rp = reps[r];
  for (int i = 0; i < 2; ++i) {
    double g = 0.0;
    double tm = -1.0;
    for (int k = 0; k < rp.ndose[i]; ++k) {
      const double td = dose_t[rp.dose_off + i * HCA_MAX_DOSES + k];
      if (td <= t && td >= tm) {
        tm = td;
        g = dose_a[rp.dose_off + i * HCA_MAX_DOSES + k] * p.G_ref[i];
      }
    }
    if (tm >= 0.0) g = g * exp(-p.k_pk[i] * (t - tm));
    g0[2 * r + i] = g;
  }
}

template <typename F>
__device__ inline void for_each_voxel(const Work& w, F f) {
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    const RepDev rp = w.reps[fb.rep];
    for (long long i = fb.begin + threadIdx.x; i < fb.end; i += kBlock) f(fb.rep, rp, rp.off + i);
  }
}

// Oxygen, Eq. (oxygen) linearised as in the paper: the uptake
// phi_K K/(K1 + K) becomes phi_K K^{n+1}/(K1 + K^n).  chi = [L != 0] marks the
// cell delta functions, w weights the vessel sources.
//   step:   c = 1/dt + r_k w + phi_K chi/(K1 + K^n),   b = K^n/dt + r_k w K0
//   steady: c =        r_k w + phi_K chi/(K1 + K),     b =        r_k w K0
__global__ void __launch_bounds__(kBlock) k_setup_o2(Work w, DevParams p, const uint8_t* L,
                                                     const double* vw, const double* K,
                                                     double* c, double* b, int steady) {
  for_each_voxel(w, [&](int, const RepDev&, long long g) {
    const double k = K[g];
    const double wv = vw[g];
    const double chi = L[g] != 0 ? 1.0 : 0.0;
    const double up = p.phi_K * chi / (p.K1 + k);
    if (steady) {
      c[g] = p.r_k * wv + up;
      b[g] = p.r_k * wv * p.K0;
    } else {
      c[g] = p.inv_dt + p.r_k * wv + up;
      b[g] = k * p.inv_dt + p.r_k * wv * p.K0;
    }
  });
}

// Drug i, Eq. (chemo): c = 1/dt + psi_G + kappa_G w,  b = G^n/dt + kappa_G w G_{i,0}.
__global__ void __launch_bounds__(kBlock) k_setup_drug(Work w, DevParams p, int drug,
                                                       const double* vw, const double* G,
                                                       const double* g0, double* c, double* b) {
  for_each_voxel(w, [&](int rep, const RepDev&, long long g) {
    const double wv = vw[g];
    const double gp = g0[2 * rep + drug];
    c[g] = p.inv_dt + p.psi_G + p.kappa_G * wv;
    b[g] = G[g] * p.inv_dt + p.kappa_G * wv * gp;
  });
}

// The three systems of one coupled step (oxygen and both drugs, see above)
// in one pass; F = [K | G1 | G2], c and b in the same 3 x ntot layout.
__global__ void __launch_bounds__(kBlock) k_setup_step(Work w, DevParams p, long long ntot,
                                                       const uint8_t* __restrict__ L,
                                                       const double* __restrict__ vw,
                                                       const double* __restrict__ F,
                                                       const double* __restrict__ g0,
                                                       double* __restrict__ c,
                                                       double* __restrict__ b) {
  for_each_voxel(w, [&](int rep, const RepDev&, long long g) {
    const double wv = vw[g];
    const double k = F[g];
    const double chi = L[g] != 0 ? 1.0 : 0.0;
    c[g] = p.inv_dt + p.r_k * wv + p.phi_K * chi / (p.K1 + k);
    b[g] = k * p.inv_dt + p.r_k * wv * p.K0;
    const double cg = p.inv_dt + p.psi_G + p.kappa_G * wv;
    for (int i = 0; i < 2; ++i) {
      const long long j = g + (i + 1) * ntot;
      c[j] = cg;
      b[j] = F[j] * p.inv_dt + p.kappa_G * wv * g0[2 * rep + i];
    }
  });
}

// Algorithm 1 initialisation of the cell state at the initial oxygen K^0:
// P, V_c at the steady states of Eqs. (odep53), (odevegf) on occupied voxels,
// phi ~ U(0,1) for cancer cells (Philox counter (gid, 0, INIT, 0), key (seed, 0)).
__global__ void __launch_bounds__(kBlock) k_init_cells(Work w, DevParams p, const uint8_t* L,
                                                       const double* K, double* P, double* Vc,
                                                       double* phi) {
  for_each_voxel(w, [&](int, const RepDev& rp, long long g) {
    const uint8_t l = L[g];
    double pv = 0.0, vv = 0.0, ph = 0.0;
    if (l != 0) {
      const double k = K[g];
      const double lam = p.k1p * k / (p.K_p53 + k);
      pv = p.k1 / lam;
      const double mu = p.k2p * k / (p.K_V + k);
      const double beta = p.k2 + p.k2pp * pv - mu * p.J5;
      const double disc = sqrt(beta * beta + 4.0 * mu * p.k2 * p.J5);
      // positive root of mu V^2 - beta V - k2 J5 = 0, in the cancellation-free form
      vv = beta >= 0.0 ? (beta + disc) / (2.0 * mu) : (2.0 * p.k2 * p.J5) / (disc - beta);
    }
    if (l == 1) {
      const uint64_t gid = (uint64_t)(g - rp.off);
      const U64x4 o = philox4x64_10(gid, 0ull, kStreamInit, 0ull, rp.seed, 0ull);
      ph = unit53(o.v[0]);
    }
    P[g] = pv;
    Vc[g] = vv;
    phi[g] = ph;
  });
}

void launch_plasma(hipStream_t s, const Work& w, const DevParams& p, const long long* d_step,
                   const double* dose_t, const double* dose_a, double* g0) {
  const int nb = (w.nreps + 63) / 64;
  hca_launch(k_plasma, dim3(nb), dim3(64), 0, s, w.nreps, w.reps, p, d_step, dose_t,
                     dose_a, g0);
}

void launch_setup_o2(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L,
                     const double* vw, const double* K, double* c, double* b, int steady) {
  hca_launch(k_setup_o2, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, L, vw, K, c, b, steady);
}

void launch_setup_drug(hipStream_t s, const Work& w, const DevParams& p, int drug,
                       const double* vw, const double* G, const double* g0, double* c,
                       double* b) {
  hca_launch(k_setup_drug, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, drug, vw, G, g0, c, b);
}

void launch_setup_step(hipStream_t s, const Work& w, const DevParams& p, long long ntot,
                       const uint8_t* L, const double* vw, const double* F, const double* g0,
                       double* c, double* b) {
  hca_launch(k_setup_step, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, ntot, L, vw, F, g0, c,
                     b);
}

void launch_init_cells(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L,
                       const double* K, double* P, double* Vc, double* phi) {
  hca_launch(k_init_cells, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, L, K, P, Vc, phi);
}

}  // namespace hca
