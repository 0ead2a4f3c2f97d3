"""Intracellular module: Eqs. (odep53), (odevegf) and (cellcycle).

Test infrastructure only.  All functions are vectorised over voxels, FP64.

Oxygen K is frozen over the coupled step at the value just solved for
(Algorithm 1 computes K first, then the ODEs "using K"); the cells see
max(K, 0) (a negative value is an artifact of a Crank-Nicolson-type field
substep's oscillation, not an oxygen level).

* p53 (Eq. odep53) is linear in P with constant coefficients while K is
  frozen, so the paper's explicit form is exact:
      lam = k1' K / (K_p53 + K)
      P(t) = P0 exp(-lam t) + k1 t phi1(lam t),   phi1(z) = (1 - e^-z)/z.
* Cell cycle (Eq. cellcycle): phi(t) = phi0 + t K / (T (K_phi + K)).
* Intracellular VEGF (Eq. odevegf) has no closed form; the paper integrates it
  with VODE (implicit Adams, maximum step 1 min).  The oracle takes classical
  RK4 with the fixed step h = dt/substeps (1 min), feeding the exact P(t) at
  the stage times.
* Initial P, V_c (Algorithm 1, initialisation) are the steady states of the
  two ODEs at the initial oxygen: P_ss = k1/lam and the positive root of
  mu V^2 - beta V - k2 J5 = 0 with mu = k2' K/(K_V + K),
  beta = k2 + k2'' P_ss - mu J5.
"""
import numpy as np


def p53_rate(K, p):
    return p.k1p * K / (p.K_p53 + K)


def phi1(z):
    z = np.asarray(z, dtype=np.float64)
    out = np.ones_like(z)
    nz = z != 0.0
    out[nz] = -np.expm1(-z[nz]) / z[nz]
    return out


def p53_exact(P0, K, t, p):
    lam = p53_rate(K, p)
    return P0 * np.exp(-lam * t) + p.k1 * t * phi1(lam * t)


def vegf_rhs(V, P, K, p):
    mu = p.k2p * K / (p.K_V + K)
    return p.k2 + p.k2pp * P * V / (p.J5 + V) - mu * V


def vegf_rk4(V0, P0, K, dt, nsub, p):
    h = dt / nsub
    V = np.array(V0, dtype=np.float64, copy=True)
    for j in range(nsub):
        t0 = j * h
        Pa = p53_exact(P0, K, t0, p)
        Pm = p53_exact(P0, K, t0 + 0.5 * h, p)
        Pb = p53_exact(P0, K, t0 + h, p)
        s1 = vegf_rhs(V, Pa, K, p)
        s2 = vegf_rhs(V + 0.5 * h * s1, Pm, K, p)
        s3 = vegf_rhs(V + 0.5 * h * s2, Pm, K, p)
        s4 = vegf_rhs(V + h * s3, Pb, K, p)
        V = V + (h / 6.0) * (s1 + 2.0 * s2 + 2.0 * s3 + s4)
    return V


def cycle_increment(K, dt, p):
    return dt * K / (p.T_cycle * (p.K_phi + K))


def ode_step(L, K, P, Vc, phi, p):
    """Advance P, V_c (occupied voxels) and phi (cancer voxels) over dt.

    Returns new (P, Vc, phi); empty voxels are left as they are.
    """
    K = np.maximum(K, 0.0)
    occ = L != 0
    can = L == 1
    Pn, Vn, phin = P.copy(), Vc.copy(), phi.copy()
    Ko, Po, Vo = K[occ], P[occ], Vc[occ]
    Pn[occ] = p53_exact(Po, Ko, p.dt_min, p)
    Vn[occ] = vegf_rk4(Vo, Po, Ko, p.dt_min, p.ode_substeps, p)
    phin[can] = phi[can] + cycle_increment(K[can], p.dt_min, p)
    return Pn, Vn, phin


def steady_p53(K, p):
    return p.k1 / p53_rate(K, p)


def steady_vegf(K, P, p):
    mu = p.k2p * K / (p.K_V + K)
    beta = p.k2 + p.k2pp * P - mu * p.J5
    return (beta + np.sqrt(beta * beta + 4.0 * mu * p.k2 * p.J5)) / (2.0 * mu)
