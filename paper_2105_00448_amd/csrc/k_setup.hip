// Plasma kinetics, coefficient / right-hand-side setup of the implicit
// systems, and the cell-state initialisation of Algorithm 1.
//
// The fields advance over a coupled step dt in m substeps of tau = dt/m (one
// by default; Algorithm 1's PDE step is 1 min), each a theta-scheme update of
// Eqs. (oxygen) and (chemo): for u_t = -R u + a Lap u + S,
//     (1/tau + theta R) u' - theta a Lap u'
//         = (1/tau - (1 - theta) R) u + (1 - theta) a Lap u + theta S' + (1 - theta) S,
// theta = 1 backward Euler, 1/2 Crank-Nicolson.  On the voxel lattice every
// such update is  c_i u_i - a' (Lap u)_i = b_i  with the solver coupling
// a' = theta a and the zero-flux 7-point Laplacian; these kernels produce c
// and b per voxel.
#include <algorithm>

#include "dev_util.h"

namespace hca {

// Principal-branch Lambert W of x = e^lx (x >= 0, the solution w >= 0 of
// w e^w = x): Halley's iteration w <- w - f / (e^w (w + 1) - (w + 2) f / (2w + 2)),
// f = w e^w - x, from w = log1p(x) >= W(x) (cubic convergence); where e^lx
// would overflow, Newton's iteration on w + ln w = lx from lx - ln lx.
__device__ inline double lambert_w_exp(double lx) {
  if (lx < 700.0) {
    const double x = exp(lx);
    double w = log1p(x);
    for (int k = 0; k < 30; ++k) {
      const double ew = exp(w);
      const double f = w * ew - x;
      const double w1 = w + 1.0;
      const double dw = f / (ew * w1 - (w + 2.0) * f / (2.0 * w1));
      w -= dw;
      if (!(fabs(dw) > 1e-16 * w)) break;
    }
    return w;
  }
  double w = lx - log(lx);
  for (int k = 0; k < 50; ++k) {
    const double dw = (w + log(w) - lx) / (1.0 + 1.0 / w);
    w -= dw;
    if (!(fabs(dw) > 1e-16 * w)) break;
  }
  return w;
}

// Drug i's plasma level at time t (intravascular module): reset to a_m G_ref
// at the latest bolus t_m <= t (0 before the first dose), then the
// elimination: one-compartment linear, G e^{-k (t - t_m)} (Eq. intrachemo3;
// fluorouracil in its linear regime); or, for fluorouracil with pk_mm, the exact
// Michaelis-Menten decay, separable into k_m ln(G/G_m) + G - G_m = -v_max (t - t_m),
// i.e. G = k_m W((G_m/k_m) e^{(G_m - v_max (t - t_m))/k_m}).
__device__ inline double plasma_level(const RepDev& rp, const DevParams& p, const double* dose_t,
                                      const double* dose_a, int i, double t) {
  double g = 0.0;
  double tm = -1.0;
  for (int k = 0; k < rp.ndose[i]; ++k) {
    const double td = dose_t[rp.dose_off + i * HCA_MAX_DOSES + k];
    if (td <= t && td >= tm) {
      tm = td;
      g = dose_a[rp.dose_off + i * HCA_MAX_DOSES + k] * p.G_ref[i];
    }
  }
  if (tm < 0.0 || g == 0.0) return tm < 0.0 ? 0.0 : g;
  if (i == 1 && p.pk_mm)
    return p.mm_km * lambert_w_exp(log(g / p.mm_km) + (g - p.mm_vmax * (t - tm)) / p.mm_km);
  return g * exp(-p.k_pk[i] * (t - tm));
}

// x <- exp(M dt) x for the three-compartment state, M = S diag(lam) S^-1.
__device__ inline void epi_propagate(const DevParams& p, double (&x)[3], double dt) {
  double y[3];
  for (int i = 0; i < 3; ++i)
    y[i] = (p.epi_Si[3 * i] * x[0] + p.epi_Si[3 * i + 1] * x[1] + p.epi_Si[3 * i + 2] * x[2]) *
           exp(p.epi_lam[i] * dt);
  for (int i = 0; i < 3; ++i) x[i] = p.epi_S[3 * i] * y[0] + p.epi_S[3 * i + 1] * y[1] + p.epi_S[3 * i + 2] * y[2];
}

// The third drug's (epirubicin's) plasma level at t: from an empty state,
// each bolus t_k <= t (ascending) resets the plasma compartment to
// a_k G_ref3 after the state has followed the three-compartment model from
// the previous bolus; 0 before the first.
__device__ inline double epi_level(const RepDev& rp, const DevParams& p, const double* dose_t,
                                   const double* dose_a, double t) {
  double x[3] = {0.0, 0.0, 0.0};
  double tc = 0.0;
  bool any = false;
  for (int k = 0; k < rp.ndose[2]; ++k) {
    const double td = dose_t[rp.dose_off + 2 * HCA_MAX_DOSES + k];
    if (td > t) break;
    if (any) epi_propagate(p, x, td - tc);
    x[0] = dose_a[rp.dose_off + 2 * HCA_MAX_DOSES + k] * p.G_ref3;
    tc = td;
    any = true;
  }
  if (!any) return 0.0;
  epi_propagate(p, x, t - tc);
  return x[0];
}

// Levels at the end (t^n + (j+1) tau; t^{n+1} for a single substep) and the
// start (t^n + j tau) of field substep j.
__global__ void k_plasma(int nreps, const RepDev* reps, DevParams p, const long long* d_step, int j,
                         const double* dose_t, const double* dose_a, double* g0) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nreps) return;
  const double t_old = (double)d_step[0] * p.dt + (double)j * p.tau;
  const double t_new = p.nsub_pde == 1 ? (double)(d_step[0] + 1) * p.dt : t_old + p.tau;
  const RepDev rp = reps[r];
  for (int i = 0; i < 2; ++i) {
    g0[3 * r + i] = plasma_level(rp, p, dose_t, dose_a, i, t_new);
    g0[3 * nreps + 3 * r + i] = plasma_level(rp, p, dose_t, dose_a, i, t_old);
  }
  if (p.drug3) {
    g0[3 * r + 2] = epi_level(rp, p, dose_t, dose_a, t_new);
    g0[3 * nreps + 3 * r + 2] = epi_level(rp, p, dose_t, dose_a, t_old);
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
// cell delta functions, w weights the vessel sources.  Below K = 0, which
// only a Crank-Nicolson-type substep's oscillation can reach, the uptake is
// continued linearly with its slope at 0, phi_K K/K1: every denominator is
// K1 + max(K, 0), so every oxygen system stays an M-matrix.
//   step:   c = 1/dt + r_k w + phi_K chi/(K1 + K^n),   b = K^n/dt + r_k w K0
//   steady: c =        r_k w + phi_K chi/(K1 + K),     b =        r_k w K0,
//           both times theta (the solver's coupling is theta a_K)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_setup_o2(Work w, DevParams p, const uint8_t* L,
                                                     const double* vw, const T* K, T* c, T* b,
                                                     int steady) {
  for_each_voxel(w, [&](int, const RepDev&, long long g) {
    const double k = K[g];
    const double wv = vw[g];
    const double chi = L[g] != 0 ? 1.0 : 0.0;
    const double up = p.phi_K * chi / (p.K1 + fmax(k, 0.0));
    if (steady) {
      c[g] = (T)(p.theta * (p.r_k * wv + up));
      b[g] = (T)(p.theta * (p.r_k * wv * p.K0));
    } else {
      c[g] = (T)(p.inv_dt + p.r_k * wv + up);
      b[g] = (T)(k * p.inv_dt + p.r_k * wv * p.K0);
    }
  });
}

// All systems of one field substep in one pass (the pointwise terms of the
// theta scheme above; the explicit Laplacian of a theta < 1 substep is added
// by k_rhs_lap); F = [K | G1 | G2 (| G3) (| V)], c and b in the same
// nf x ntot layout.
//   oxygen: R = r_k w + phi_K chi/(K1 + K) (uptake linearised at the substep's
//           start), S = r_k w K0 constant;
//   drugs:  R = psi_G + kappa_G w, S = kappa_G w g0(t) with the plasma level
//           at the substep's end (weight theta) and start (1 - theta); the
//           third drug (drug3) likewise in field 3;
//   VEGF (vegf): R = psi_V, S = sec_V V_c chi, Eq. (vac_v) with no Avastin,
//           V_c of the coupled step's start at both ends of every substep.
// With one backward-Euler substep these are the coupled step's systems
// c = 1/dt + R, b = u/dt + S.  The fields but oxygen have a c that depends on
// the vessel map and the constants only: keep_c leaves the c already stored
// for them.
template <bool X, typename T>
__global__ void __launch_bounds__(kBlock) k_setup_step(Work w, DevParams p, long long ntot,
                                                       const uint8_t* __restrict__ L,
                                                       const double* __restrict__ vw,
                                                       T* __restrict__ F,
                                                       const double* __restrict__ Vc,
                                                       const double* __restrict__ g0,
                                                       T* __restrict__ c, T* __restrict__ b,
                                                       const T* Fprev, T* Fprev_out, unsigned xmask,
                                                       int xmode, int keep_c) {
  const double th = p.theta, th1 = 1.0 - p.theta;
  // X: the solves' initial guess as k_extrapolate forms it, from the value u
  // just read for b (fields of xmask); u goes to Fprev_out (Fprev itself, or
  // the buffer that takes Fprev's role after the step's history rotation)
  auto guess = [&](int f, long long j, double u) {
    if (X && ((xmask >> f) & 1u)) {
      const double up = Fprev[j];
      Fprev_out[j] = (T)u;
      if (xmode == 1) {
        F[j] = (T)(u + (u - up));
      } else if (up > 0.0 && u > 0.0 && u < up) {   // geometric, decaying values only
        F[j] = (T)(u * (u / up));
      }
    }
  };
  for_each_voxel(w, [&](int rep, const RepDev&, long long g) {
    const double wv = vw[g];
    const double k = F[g];
    const double chi = L[g] != 0 ? 1.0 : 0.0;
    const double rw = p.r_k * wv;
    const double up = p.phi_K * chi / (p.K1 + fmax(k, 0.0));
    c[g] = (T)(p.inv_tau + th * rw + th * up);
    b[g] = (T)(k * (p.inv_tau - th1 * (rw + up)) + rw * p.K0);
    guess(0, g, k);
    const double kw = p.kappa_G * wv;
    const double cg = p.inv_tau + th * p.psi_G + th * kw;
    const double rg = p.psi_G + kw;
    for (int i = 0; i < 2 + p.drug3; ++i) {   // drug i in field i + 1
      const long long j = g + (i + 1) * ntot;
      const double u = F[j];
      if (!keep_c) c[j] = (T)cg;
      b[j] = (T)(u * (p.inv_tau - th1 * rg) +
                 kw * (th * g0[3 * rep + i] + th1 * g0[3 * w.nreps + 3 * rep + i]));
      guess(i + 1, j, u);
    }
    if (p.vegf) {
      const long long j = g + (long long)p.fV * ntot;
      const double u = F[j];
      if (!keep_c) c[j] = (T)(p.inv_tau + th * p.psi_V);
      b[j] = (T)(u * (p.inv_tau - th1 * p.psi_V) + p.sec_V * Vc[g] * chi);
      guess(p.fV, j, u);
    }
  });
}

// Newton step on the implicit oxygen update with the uptake at the new value,
//   (1/tau + theta r_k w) K' + theta phi_K chi K'/(K1 + K') - theta a_K Lap K' = b_lin,
// linearised at the iterate K:
//   c = 1/tau + theta r_k w + theta phi_K chi K1/(K1 + K)^2,
//   b = b_lin - theta phi_K chi K^2/(K1 + K)^2;
// with the linear continuation below K = 0 (K+ = max(K, 0)):
//   c = ... K1/(K1 + K+)^2,  b = b_lin - theta phi_K chi K K+/(K1 + K+)^2.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_setup_o2_newton(Work w, DevParams p,
                                                            const uint8_t* __restrict__ L,
                                                            const double* __restrict__ vw,
                                                            const T* __restrict__ K,
                                                            const T* __restrict__ b_lin,
                                                            T* __restrict__ c, T* __restrict__ b) {
  for_each_voxel(w, [&](int, const RepDev&, long long g) {
    const double k = K[g];
    const double kp = fmax(k, 0.0);
    const double chi = L[g] != 0 ? 1.0 : 0.0;
    const double d = p.K1 + kp;
    c[g] = (T)(p.inv_tau + p.theta * (p.r_k * vw[g]) + p.theta * (p.phi_K * chi * p.K1 / (d * d)));
    b[g] = (T)((double)b_lin[g] - p.theta * (p.phi_K * chi * k * kp / (d * d)));
  });
}

// b += (1 - theta) a Lap F for the nf fields (theta < 1): the explicit half
// of a Crank-Nicolson-type substep, Lap the zero-flux 7-point Laplacian
// (neighbours in the order -x, +x, -y, +y, -z, +z).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_rhs_lap(Work w, DevParams p, long long ntot,
                                                    const T* __restrict__ F, T* __restrict__ b) {
  const double sK = (1.0 - p.theta) * p.aK, sG = (1.0 - p.theta) * p.aG,
               sV = (1.0 - p.theta) * p.aV;
  for_each_voxel(w, [&](int, const RepDev& rp, long long g) {
    const long long i = g - rp.off;
    const int x = (int)(i % rp.nx);
    const long long q = i / rp.nx;
    const int y = (int)(q % rp.ny);
    const int z = (int)(q / rp.ny);
    const long long sy = rp.nx, sz = (long long)rp.nx * rp.ny;
    for (int f = 0; f < p.nf; ++f) {
      const T* u = F + (long long)f * ntot;
      const double uc = u[g];
      double lap = 0.0;
      if (x > 0) lap += (double)u[g - 1] - uc;
      if (x + 1 < rp.nx) lap += (double)u[g + 1] - uc;
      if (y > 0) lap += (double)u[g - sy] - uc;
      if (y + 1 < rp.ny) lap += (double)u[g + sy] - uc;
      if (z > 0) lap += (double)u[g - sz] - uc;
      if (z + 1 < rp.nz) lap += (double)u[g + sz] - uc;
      const long long j = g + (long long)f * ntot;
      b[j] = (T)((double)b[j] + (f == 0 ? sK : (p.vegf && f == p.fV) ? sV : sG) * lap);
    }
  });
}

// Extrapolation in time of the solved fields as the solver's initial guess,
// the previous solve's value kept in Fprev: mode 1 linear, u + (u - u_prev);
// mode 2 geometric, u (u / u_prev), on positive decaying values only (a
// drug field between boluses decays nearly geometrically), else u.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_extrapolate(Work w, long long ntot, int nf, unsigned fmask,
                                                        int mode, T* __restrict__ F,
                                                        T* __restrict__ Fprev) {
  for_each_voxel(w, [&](int, const RepDev&, long long g) {
    for (int f = 0; f < nf; ++f) {
      if (!((fmask >> f) & 1u)) continue;
      const long long j = g + (long long)f * ntot;
      const double u = F[j];
      const double up = Fprev[j];
      Fprev[j] = (T)u;
      if (mode == 1) {
        F[j] = (T)(u + (u - up));
      } else if (up > 0.0 && u > 0.0 && u < up) {   // geometric, decaying values only
        F[j] = (T)(u * (u / up));
      }
    }
  });
}

// Algorithm 1 initialisation of the cell state at the initial oxygen K^0:
// P, V_c at the steady states of Eqs. (odep53), (odevegf) on occupied voxels,
// phi ~ U(0,1) for cancer cells (Philox counter (gid, 0, INIT, 0), key (seed, 0)).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_init_cells(Work w, DevParams p, const uint8_t* L,
                                                       const T* K, double* P, double* Vc,
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
                   int j, const double* dose_t, const double* dose_a, double* g0) {
  const int nb = (w.nreps + 63) / 64;
  hca_launch(k_plasma, dim3(nb), dim3(64), 0, s, w.nreps, w.reps, p, d_step, j, dose_t, dose_a, g0);
}

template <typename T>
void launch_setup_o2(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L,
                     const double* vw, const T* K, T* c, T* b, int steady) {
  hca_launch(k_setup_o2<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, L, vw, K,
             c, b, steady);
}

template <typename T>
void launch_setup_step(hipStream_t s, const Work& w, const DevParams& p, long long ntot,
                       const uint8_t* L, const double* vw, T* F, const double* Vc,
                       const double* g0, T* c, T* b, const T* Fprev, T* Fprev_out, unsigned xmask,
                       int xmode, int keep_c) {
  if (Fprev)
    hca_launch(k_setup_step<true, T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, ntot,
               L, vw, F, Vc, g0, c, b, Fprev, Fprev_out, xmask, xmode, keep_c);
  else
    hca_launch(k_setup_step<false, T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, ntot,
               L, vw, F, Vc, g0, c, b, Fprev, Fprev_out, xmask, xmode, keep_c);
}

template <typename T>
void launch_setup_o2_newton(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L,
                            const double* vw, const T* K, const T* b_lin, T* c, T* b) {
  hca_launch(k_setup_o2_newton<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, L,
             vw, K, b_lin, c, b);
}

template <typename T>
void launch_rhs_lap(hipStream_t s, const Work& w, const DevParams& p, long long ntot, const T* F,
                    T* b) {
  hca_launch(k_rhs_lap<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, ntot, F, b);
}

template <typename T>
void launch_extrapolate(hipStream_t s, const Work& w, long long ntot, int nf, unsigned fmask, int mode,
                        T* F, T* Fprev) {
  hca_launch(k_extrapolate<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, ntot, nf,
             fmask, mode, F, Fprev);
}

template <typename T>
void launch_init_cells(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L,
                       const T* K, double* P, double* Vc, double* phi) {
  hca_launch(k_init_cells<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, p, L, K, P,
             Vc, phi);
}

template <typename S, typename D>
__global__ void __launch_bounds__(kBlock) k_convert(const S* __restrict__ src, D* __restrict__ dst,
                                                    long long n) {
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
    dst[i] = (D)src[i];
}

void launch_convert(hipStream_t s, const float* src, double* dst, long long n) {
  const long long nb = std::min<long long>((n + kBlock - 1) / kBlock, 65536);
  hca_launch(k_convert<float, double>, dim3((unsigned)std::max<long long>(nb, 1)), dim3(kBlock), 0, s,
             src, dst, n);
}

void launch_convert(hipStream_t s, const double* src, float* dst, long long n) {
  const long long nb = std::min<long long>((n + kBlock - 1) / kBlock, 65536);
  hca_launch(k_convert<double, float>, dim3((unsigned)std::max<long long>(nb, 1)), dim3(kBlock), 0, s,
             src, dst, n);
}

#define HCA_SETUP_INST(T)                                                                          \
  template void launch_setup_o2<T>(hipStream_t, const Work&, const DevParams&, const uint8_t*,     \
                                   const double*, const T*, T*, T*, int);                          \
  template void launch_setup_step<T>(hipStream_t, const Work&, const DevParams&, long long,        \
                                     const uint8_t*, const double*, T*, const double*,             \
                                     const double*, T*, T*, const T*, T*, unsigned, int, int);     \
  template void launch_setup_o2_newton<T>(hipStream_t, const Work&, const DevParams&,              \
                                          const uint8_t*, const double*, const T*, const T*, T*,   \
                                          T*);                                                     \
  template void launch_rhs_lap<T>(hipStream_t, const Work&, const DevParams&, long long, const T*, \
                                  T*);                                                             \
  template void launch_extrapolate<T>(hipStream_t, const Work&, long long, int, unsigned, int, T*, \
                                      T*);                                                         \
  template void launch_init_cells<T>(hipStream_t, const Work&, const DevParams&, const uint8_t*,   \
                                     const T*, double*, double*, double*);
HCA_SETUP_INST(double)
HCA_SETUP_INST(float)

}  // namespace hca
