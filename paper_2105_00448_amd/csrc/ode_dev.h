// Per-voxel plain integrator of the intracellular module over one coupled
// step: Eqs. (odep53), (odevegf), (cellcycle), oxygen frozen at K^{n+1}.
// Shared by the ODE kernel and the surrogate's fallback path.
//
// * p53 is linear with constant coefficients while K is frozen, so it is
//   advanced exactly (the paper's explicit form):
//     lam = k1' K/(K_p53 + K),  P(t) = P0 e^{-lam t} + k1 t phi1(lam t),
//     phi1(z) = (1 - e^{-z})/z = -expm1(-z)/z.
// * V_c: classical RK4 with the fixed step h = dt/nsub (1 min, the paper's
//   VODE maximum step), the exact P(t) at the stage times, advanced along the
//   half-step grid by products and sums of positive terms.
// * phi (cancer cells only): phi += dt K / (T (K_phi + K)), evaluated without
//   contraction so it rounds exactly like the plain expression.
#pragma once

#include "hca_internal.h"

namespace hca {

__device__ inline double cycle_increment(double dt, double K, double T, double Kphi) {
#pragma clang fp contract(off)
  const double num = dt * K;
  const double den = T * (Kphi + K);
  return num / den;
}

__device__ inline double add_nocontract(double a, double b) {
#pragma clang fp contract(off)
  return a + b;
}

// 1/x for finite x > 0: the hardware reciprocal estimate refined by two
// Newton steps for f(r) = 1/r - x, r <- r + r (1 - x r) (each step squares the
// relative error), so the result is within an ulp or two of the rounded
// quotient at about half the instructions of the IEEE division sequence.
__device__ inline double recip_pos(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// J5 + V > 0 (J5 > 0, V >= 0).
__device__ inline double vegf_rhs(double V, double Pt, double mu, const DevParams& p) {
  return p.k2 + p.k2pp * Pt * V * recip_pos(p.J5 + V) - mu * V;
}

// Advances (P, Vc, phi) of one occupied voxel (cell code l) with oxygen kk,
// seen as max(kk, 0) (a negative value can only come from the oscillation of
// a Crank-Nicolson-type field substep).
__device__ inline void ode_voxel(const DevParams& p, uint8_t l, double kk, double& P, double& Vc,
                                 double& phi) {
  kk = fmax(kk, 0.0);
  const double h = p.dt / p.nsub;
  const double P0 = P;
  const double lam = p.k1p * kk / (p.K_p53 + kk);
  const double mu = p.k2p * kk / (p.K_V + kk);
  // Along the half-step grid: E(t) = e^{-lam t} and
  // Gi(t) = int_0^t e^{-lam s} ds = t phi1(lam t), so P(t) = P0 E + k1 Gi.
  // Both advance by products and sums of positive terms (no cancellation):
  //   E(t + h/2) = E eh,   Gi(t + h/2) = Gi + E gh,
  //   eh = e^{-lam h/2},   gh = -expm1(-lam h/2)/lam  (h/2 when lam = 0).
  const double zh = lam * 0.5 * h;
  const double eh = exp(-zh);
  const double gh = zh > 0.0 ? -expm1(-zh) / lam : 0.5 * h;
  double E = 1.0, Gi = 0.0;
  double V = Vc;
  for (int s = 0; s < p.nsub; ++s) {
    const double Pa = P0 * E + p.k1 * Gi;
    const double Gm = Gi + E * gh;
    const double Em = E * eh;
    const double Pm = P0 * Em + p.k1 * Gm;
    Gi = Gm + Em * gh;
    E = Em * eh;
    const double Pb = P0 * E + p.k1 * Gi;
    const double s1 = vegf_rhs(V, Pa, mu, p);
    const double s2 = vegf_rhs(V + 0.5 * h * s1, Pm, mu, p);
    const double s3 = vegf_rhs(V + 0.5 * h * s2, Pm, mu, p);
    const double s4 = vegf_rhs(V + h * s3, Pb, mu, p);
    V = V + (h / 6.0) * (s1 + 2.0 * s2 + 2.0 * s3 + s4);
  }
  const double z = lam * p.dt;
  const double ph1 = z > 0.0 ? -expm1(-z) / z : 1.0;
  P = P0 * exp(-z) + p.k1 * p.dt * ph1;
  Vc = V;
  if (l == 1) phi = add_nocontract(phi, cycle_increment(p.dt, kk, p.T_cycle, p.K_phi));
}

}  // namespace hca
