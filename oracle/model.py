"""Algorithm 1 of the paper: initialisation and the coupled time step.

Test infrastructure only.

State at t^n = n dt:  L (uint8 cell map), K, G1, G2, P, Vc, phi (float64),
with the perfusion map w (0 = no vessel, > 0 = perfusion weight), static
unless the VEGF option is on; then the state also holds the extracellular
VEGF V and its own w, which the vessel birth-death update changes.

One coupled step n -> n+1 (loop body of Algorithm 1, with the implicit Euler
step dt of the cell-cycle update):

1. plasma concentrations G_{i,0}(t^{n+1}) (intravascular module, closed form);
   (steps 1-3 optionally in m theta-scheme substeps, see ``solve_fields``);
2. oxygen, Eq. (oxygen) with s_K = 1, linearised as the paper does: the
   uptake phi_K K/(K1 + K) becomes phi_K K^{n+1}/(K1 + K^n):
       (1/dt + r_k w + phi_K chi_c/(K1 + K^n)) K^{n+1} - a_K Lap K^{n+1}
           = K^n/dt + r_k w K0,
   chi_c = [L != 0] the cell indicator (Eq. delta_function with one unit
   delta per occupied voxel), w the vessel indicator weighted by perfusion;
3. each drug, Eq. (chemo):
       (1/dt + psi_G + kappa_G w) G^{n+1} - a_G Lap G^{n+1}
           = G^n/dt + kappa_G w G_{i,0}(t^{n+1});
   Below K = 0, reachable only through the oscillation of a theta < 1
   substep, the uptake is continued linearly with its slope at 0,
   phi_K K/K1 (``uptake_den``): every oxygen system stays an M-matrix;
4. intracellular ODEs with K^{n+1} frozen;
5. cellular automaton on the state after 4.
With ``p.vegf``: V^{n+1} from Eq. (vac_v) without Avastin (the V_c source of
the state at t^n, see ``vegf_substep_system``) alongside steps 2-3, and after
step 5 the vessel birth-death update (``vascular.vessel_update``) when due.

Initialisation (Algorithm 1 before the loop): K^0 solves Eq. (oxygen) with
s_K = 0 (Picard iteration on the uptake coefficient from K = K0 until the
max-norm relative change is below ``picard_tol``); P, V_c are the ODE steady
states at K^0 on occupied voxels; phi_0 ~ U(0, 1) for cancer cells from
Philox stream INIT at counter (gid, 0, 0, 0); G = 0.
"""
from dataclasses import dataclass, field

import numpy as np

from . import ca, lattice, ode, philox, pk, vascular
from .constants import CANCER, STREAM_INIT


@dataclass
class Schedule:
    """Dose times (min) and amounts (multiples of G_ref) per drug (a third
    entry for the third drug)."""
    times: tuple = ((), ())
    amts: tuple = ((), ())


@dataclass
class State:
    L: np.ndarray
    K: np.ndarray
    G1: np.ndarray
    G2: np.ndarray
    P: np.ndarray
    Vc: np.ndarray
    phi: np.ndarray
    step: int = 0
    V: np.ndarray = None        # extracellular VEGF (VEGF option)
    w: np.ndarray = None        # the state's own vessel map (VEGF option)
    G3: np.ndarray = None       # third drug in the tissue (third-drug option)

    def copy(self):
        cp = lambda a: None if a is None else a.copy()
        return State(self.L.copy(), self.K.copy(), self.G1.copy(), self.G2.copy(),
                     self.P.copy(), self.Vc.copy(), self.phi.copy(), self.step,
                     cp(self.V), cp(self.w), cp(self.G3))


def plasma_pair(t, sched, p):
    g1 = pk.plasma(t, sched.times[0], sched.amts[0], p.k_pk[0], p.G_ref[0])
    if p.pk_mm:
        g2 = pk.plasma_mm(t, sched.times[1], sched.amts[1], p.mm_vmax, p.mm_km, p.G_ref[1])
    else:
        g2 = pk.plasma(t, sched.times[1], sched.amts[1], p.k_pk[1], p.G_ref[1])
    return g1, g2


def uptake_den(K, p):
    """Denominator K1 + max(K, 0) of the oxygen uptake phi_K K/(K1 + K), which
    for K < 0 continues the uptake by its tangent at 0."""
    return p.K1 + np.maximum(K, 0.0)


def o2_system(L, w, K_old, p):
    chi = (L != 0).astype(np.float64)
    c = 1.0 / p.dt_min + p.r_k * w + p.phi_K * chi / uptake_den(K_old, p)
    b = K_old / p.dt_min + p.r_k * w * p.K0
    return c, b


def drug_system(w, G_old, g0, p):
    c = 1.0 / p.dt_min + p.psi_G + p.kappa_G * w
    b = G_old / p.dt_min + p.kappa_G * w * g0
    return c, b


def o2_substep_system(L, w, K_old, p, tau, theta):
    """One theta-scheme substep of length tau of Eq. (oxygen), the uptake
    linearised at the substep's old value as in the coupled step:
        (1/tau + theta R) K' - theta a_K Lap K'
            = (1/tau - (1 - theta) R) K + (1 - theta) a_K Lap K + r_k w K0,
    R = r_k w + phi_K chi/(K1 + K) (the source r_k w K0 is constant in time).
    theta = 1: backward Euler (with tau = dt exactly the coupled step's
    system); theta = 1/2: Crank-Nicolson.  Returns (c, b) of the system with
    coupling theta a_K."""
    chi = (L != 0).astype(np.float64)
    rw = p.r_k * w
    up = p.phi_K * chi / uptake_den(K_old, p)
    c = 1.0 / tau + theta * rw + theta * up
    b = K_old * (1.0 / tau - (1.0 - theta) * (rw + up)) + rw * p.K0
    if theta < 1.0:
        b = b + (1.0 - theta) * p.a_K * lattice.laplacian_apply(K_old)
    return c, b


def drug_substep_system(w, G_old, g_old, g_new, p, tau, theta):
    """One theta-scheme substep of Eq. (chemo) with the plasma level at the
    substep's ends:
        (1/tau + theta R) G' - theta a_G Lap G'
            = (1/tau - (1 - theta) R) G + (1 - theta) a_G Lap G
              + kappa_G w (theta g_new + (1 - theta) g_old),
    R = psi_G + kappa_G w.  Returns (c, b) of the system with coupling theta a_G."""
    kw = p.kappa_G * w
    c = 1.0 / tau + theta * p.psi_G + theta * kw
    b = G_old * (1.0 / tau - (1.0 - theta) * (p.psi_G + kw)) + kw * (theta * g_new + (1.0 - theta) * g_old)
    if theta < 1.0:
        b = b + (1.0 - theta) * p.a_G * lattice.laplacian_apply(G_old)
    return c, b


def vegf_substep_system(L, V_old, Vc, p, tau, theta):
    """One theta-scheme substep of Eq. (vac_v) with no Avastin (A = C = 0, so
    the binding terms vanish): V_t = D_V Lap V + a V_c chi - psi_V V, the
    secretion a V_c chi (chi = [L != 0]: cancer and stroma cells release
    VEGF) taken from the cell state at the start of the coupled step, so it is
    the same at both ends of every substep:
        (1/tau + theta psi_V) V' - theta a_V Lap V'
            = (1/tau - (1 - theta) psi_V) V + (1 - theta) a_V Lap V + a V_c chi.
    Returns (c, b) of the system with coupling theta a_V."""
    chi = (L != 0).astype(np.float64)
    c = np.full(L.shape, 1.0 / tau + theta * p.psi_V)
    b = V_old * (1.0 / tau - (1.0 - theta) * p.psi_V) + p.sec_V * Vc * chi
    if theta < 1.0:
        b = b + (1.0 - theta) * p.a_V * lattice.laplacian_apply(V_old)
    return c, b


def solve_vegf(s, p, method="cg"):
    """V^{n+1}: ``p.pde_substeps`` theta-scheme substeps of Eq. (vac_v) over
    the coupled step (one backward-Euler solve by default)."""
    m, theta = p.pde_substeps, p.pde_theta
    tau = p.dt_min / m
    V = s.V if s.V is not None else np.zeros(s.L.shape)
    for _ in range(m):
        c, b = vegf_substep_system(s.L, V, s.Vc, p, tau, theta)
        V = lattice.solve(c, theta * p.a_V, b, x0=V, method=method)
    return V


def solve_drug3(s, w, sched, p, method="cg"):
    """G3^{n+1}: the third drug (epirubicin) by the drugs' Eq. (chemo) in
    ``p.pde_substeps`` theta-scheme substeps, its vessel source from the
    three-compartment plasma level at the substep ends."""
    m, theta = p.pde_substeps, p.pde_theta
    tau = p.dt_min / m
    G = s.G3 if s.G3 is not None else np.zeros(s.L.shape)
    for j in range(m):
        t_old = s.step * p.dt_min + j * tau
        t_new = (s.step + 1) * p.dt_min if m == 1 else t_old + tau
        g_old = pk.plasma_epi(t_old, sched.times[2], sched.amts[2], p)
        g_new = pk.plasma_epi(t_new, sched.times[2], sched.amts[2], p)
        c, b = drug_substep_system(w, G, g_old, g_new, p, tau, theta)
        G = lattice.solve(c, theta * p.a_G, b, x0=G, method=method)
    return G


def o2_newton_system(L, w, K_it, b_lin, p, tau, theta):
    """One Newton step on the implicit oxygen update with the uptake kept
    nonlinear, phi_K K'/(K1 + K') at the new value:
        (1/tau + theta r_k w) K' + theta phi_K chi K'/(K1 + K') - theta a_K Lap K' = b_lin,
    b_lin the linearised substep's right-hand side (its explicit part uses the
    old value in the uptake exactly as the nonlinear form does).  Linearised
    at the iterate K_it the step solves
        (1/tau + theta r_k w + theta phi_K chi K1/(K1 + K_it)^2) K'
            - theta a_K Lap K' = b_lin - theta phi_K chi K_it^2/(K1 + K_it)^2;
    below K = 0 the uptake's linear continuation phi_K K/K1 gives, with
    K+ = max(K_it, 0), the diagonal term K1/(K1 + K+)^2 and the right-hand
    side term K_it K+/(K1 + K+)^2 (the same expressions for K_it >= 0)."""
    chi = (L != 0).astype(np.float64)
    kp = np.maximum(K_it, 0.0)
    d = p.K1 + kp
    c = 1.0 / tau + theta * (p.r_k * w) + theta * (p.phi_K * chi * p.K1 / (d * d))
    b = b_lin - theta * (p.phi_K * chi * K_it * kp / (d * d))
    return c, b


def steady_o2_system(L, w, K_iter, p):
    chi = (L != 0).astype(np.float64)
    c = p.r_k * w + p.phi_K * chi / uptake_den(K_iter, p)
    b = p.r_k * w * p.K0
    return c, b


def steady_oxygen(L, w, p, picard_tol=1e-13, maxit=200, method="cg"):
    K = np.full(L.shape, p.K0)
    for it in range(maxit):
        c, b = steady_o2_system(L, w, K, p)
        Kn = lattice.solve(c, p.a_K, b, x0=K, method=method)
        change = np.max(np.abs(Kn - K)) / np.max(np.abs(Kn))
        K = Kn
        if change < picard_tol:
            return K, it + 1
    raise RuntimeError("steady oxygen Picard iteration did not converge")


def init_state(L, w, seed, p, method="cg"):
    L = L.astype(np.uint8)
    K, _ = steady_oxygen(L, w, p, method=method)
    occ = L != 0
    P = np.zeros(L.shape)
    Vc = np.zeros(L.shape)
    P[occ] = ode.steady_p53(K[occ], p)
    Vc[occ] = ode.steady_vegf(K[occ], P[occ], p)
    phi = np.zeros(L.shape)
    gids = np.flatnonzero(L == CANCER)
    o0, _, _, _ = philox.block_vec(gids.astype(np.uint64), 0, STREAM_INIT, 0, (seed, 0))
    phi.ravel()[gids] = philox.to_unit_vec(o0)
    z = np.zeros(L.shape)
    s = State(L, K, z.copy(), z.copy(), P, Vc, phi, 0)
    if p.vegf:   # V(., 0) = 0 (Algorithm 1) and the state's own vessel map
        s.V, s.w = z.copy(), np.array(w, dtype=np.float64)
    if p.drug3:
        s.G3 = z.copy()
    return s


def solve_fields(s, w, sched, p, method="cg"):
    """Steps 1-3: returns (K^{n+1}, G1^{n+1}, G2^{n+1}).

    With the defaults (one backward-Euler substep) this is one implicit solve
    per field over the coupled step.  With ``p.pde_substeps = m`` the fields
    advance by m substeps of dt/m (Algorithm 1's PDE step; m = 30 gives its
    1-min step), each a theta-scheme solve (``p.pde_theta``: 1 backward
    Euler, 1/2 Crank-Nicolson) with the plasma levels at the substep's ends
    and the oxygen uptake linearised at the substep's start; with
    ``p.o2_newton = k`` the oxygen update then takes k Newton steps on the
    uptake at the new value (the nonlinear form the paper linearises)."""
    m, theta = p.pde_substeps, p.pde_theta
    if m == 1 and theta == 1.0 and p.o2_newton == 0:
        t1 = (s.step + 1) * p.dt_min
        g0 = plasma_pair(t1, sched, p)
        c, b = o2_system(s.L, w, s.K, p)
        K = lattice.solve(c, p.a_K, b, x0=s.K, method=method)
        c, b = drug_system(w, s.G1, g0[0], p)
        G1 = lattice.solve(c, p.a_G, b, x0=s.G1, method=method)
        c, b = drug_system(w, s.G2, g0[1], p)
        G2 = lattice.solve(c, p.a_G, b, x0=s.G2, method=method)
        return K, G1, G2
    tau = p.dt_min / m
    K, G = s.K, [s.G1, s.G2]
    for j in range(m):
        t_old = s.step * p.dt_min + j * tau
        g_old = plasma_pair(t_old, sched, p)
        g_new = plasma_pair(t_old + tau, sched, p)
        c, b = o2_substep_system(s.L, w, K, p, tau, theta)
        K = lattice.solve(c, theta * p.a_K, b, x0=K, method=method)
        for _ in range(p.o2_newton):   # the uptake at the new value (Newton)
            cn, bn = o2_newton_system(s.L, w, K, b, p, tau, theta)
            K = lattice.solve(cn, theta * p.a_K, bn, x0=K, method=method)
        for i in range(2):
            c, b = drug_substep_system(w, G[i], g_old[i], g_new[i], p, tau, theta)
            G[i] = lattice.solve(c, theta * p.a_G, b, x0=G[i], method=method)
    return K, G[0], G[1]


def step(s, w, sched, seed, p, method="cg"):
    """One coupled step; returns (new state, CA event counts).  The vessel
    map is ``s.w`` when the state holds one, else ``w``.  With ``p.vegf`` the
    new state holds V^{n+1} and the vessel map after the birth-death update
    (events "births", "deaths")."""
    if s.w is not None:
        w = s.w
    K, G1, G2 = solve_fields(s, w, sched, p, method)
    V = solve_vegf(s, p, method) if p.vegf else s.V
    G3 = solve_drug3(s, w, sched, p, method) if p.drug3 else s.G3
    P, Vc, phi = ode.ode_step(s.L, K, s.P, s.Vc, s.phi, p)
    Ln, phin, Pn, Vn, ev, _, _ = ca.ca_update(s.L, w, K, G1, G2, phi, P, Vc,
                                              s.step, seed, p, G3 if p.drug3 else None)
    w_out = s.w
    if p.vegf:
        w_out, nb, nd = vascular.vessel_update(Ln, w, V, s.step, seed, p)
        ev = dict(ev, births=nb, deaths=nd)
    return State(Ln, K, G1, G2, Pn, Vn, phin, s.step + 1, V, w_out, G3), ev
