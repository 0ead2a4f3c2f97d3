"""Model constants of the oracle (Table 1 of the paper) and the readings taken
where the paper is silent, ambiguous or garbled.

Test infrastructure only.  The HIP library carries its own transcription of
the same table; a CPU test compares the two field by field.
"""
from dataclasses import dataclass, field, replace

MIN_PER_DAY = 1440.0


@dataclass(frozen=True)
class Params:
    # lattice and coupled step ------------------------------------------------
    h_um: float = 20.0          # voxel edge (the paper's 2-D lattice uses 10 um)
    dt_min: float = 30.0        # Table 1 "time interval of cell cycle update"
    # oxygen, Eq. (oxygen), Table 1 -----------------------------------------
    D_K: float = 1.05e5         # um^2/min
    r_k: float = 1.88e4         # supply rate per unit perfusion weight, 1/min
    K0: float = 20.0            # blood oxygen, mmHg
    phi_K: float = 900.0        # consumption rate per occupied voxel
    K1: float = 2.5             # half-maximal consumption, mmHg
    # chemotherapies, Eq. (chemo), Table 1 ------------------------------------
    D_G: float = 9.6e3          # um^2/min
    psi_G: float = 1.0e-2       # decay, 1/min
    kappa_G: float = 0.1        # vessel transfer per unit perfusion weight, 1/min
    # plasma elimination: drug 1 cyclophosphamide cl_3/u, drug 2 fluorouracil
    # in its linear regime v_max/k_m (Table 1)
    k_pk: tuple = (3.93e3 / 2430e3, 1.75 / 27.0)
    G_ref: tuple = (1.0, 1.0)   # normalisation of the kill probability
    b_int: tuple = (1, 1)       # Table 1 "FEC dose-response shape" alpha = 1
    # intracellular module, Eqs. (odep53), (odevegf), (cellcycle), Table 1 ----
    k1: float = 4.0e-4
    k1p: float = 1.0e-2
    K_p53: float = 1.0e-2
    k2: float = 2.0e-3
    k2p: float = 1.0e-2
    k2pp: float = -2.0e-4
    J5: float = 4.0e-2
    K_V: float = 1.0e-2
    K_phi: float = 1.4
    T_cycle: float = 3.74 * MIN_PER_DAY
    ode_substeps: int = 30      # V_c sub-steps of 1 min (the paper's VODE max step)
    # time stepping of Eqs. (oxygen) and (chemo) inside one coupled step ------
    pde_substeps: int = 1       # implicit substeps per coupled step (Algorithm 1's
                                # 1-min PDE step is 30)
    pde_theta: float = 1.0      # theta scheme: 1 = backward Euler, 1/2 = Crank-Nicolson
    o2_newton: int = 0          # Newton iterations on the nonlinear oxygen uptake after
                                # the linearised solve (0: the paper's linearisation)
    # drug 2 (fluorouracil) plasma elimination: 0 its linear regime (rate k_pk[1]),
    # 1 the exact Michaelis-Menten model with v_max, k_m (Table 1)
    pk_mm: int = 0
    mm_vmax: float = 1.75       # ug/mL/min
    mm_km: float = 27.0         # ug/mL
    # extracellular VEGF, Eq. (vac_v) with no Avastin (A = C = 0), and the
    # vascular module, Eq. (vascular_module); off by default ----------------
    vegf: int = 0               # 1: solve V with the other fields and run the vessel
                                # birth-death update every dv_min
    D_V: float = 3.52e3         # diffusion, um^2/min (Table 1)
    psi_V: float = 1.0e-2       # decay, 1/min (Table 1)
    sec_V: float = 6.66e-6      # secretion slope a: source a V_c per occupied voxel, 1/min
    dv_min: float = 720.0       # vessel update interval (Table 1), a multiple of dt_min
    V_low: float = 1.0e-6       # lower viability threshold, ug/mL (Table 1)
    V_high: float = 1.0e-4      # upper threshold: missing from Table 1, chosen
    p_death: float = 0.05       # death probability per update outside the window (chosen)
    birth_per_V: float = 100.0  # birth probability per update = birth_per_V * V inside
                                # the window, mL/ug (chosen: 0.01 at V_high)
    w_new: float = 1.0          # perfusion weight of a new vessel
    # third drug, epirubicin: three-compartment plasma kinetics (Table 1's
    # volumes in mL; its clearances, printed in garbled units, read as mL/min),
    # its own tissue field G3 (Eq. chemo with the drugs' D_G, psi_G, kappa_G)
    # and a third kill trial; off by default -------------------------------
    drug3: int = 0
    epi_w1: float = 18.0e3      # plasma compartment volume, mL
    epi_w2: float = 957.0e3     # peripheral compartment volumes, mL
    epi_w3: float = 25.0e3
    epi_q2: float = 0.918e3     # intercompartmental clearances, mL/min
    epi_q3: float = 0.25e3
    epi_cl: float = 0.983e3     # elimination clearance, mL/min
    G_ref3: float = 1.0         # kill-probability normalisation
    b_int3: int = 1             # dose-response shape (Table 1 alpha = 1)

    @property
    def a_K(self):
        """Face coupling D_K/h^2 of the oxygen Laplacian, 1/min."""
        return self.D_K / (self.h_um * self.h_um)

    @property
    def a_G(self):
        """Face coupling D_G/h^2 of the drug Laplacian, 1/min."""
        return self.D_G / (self.h_um * self.h_um)

    @property
    def a_V(self):
        """Face coupling D_V/h^2 of the VEGF Laplacian, 1/min."""
        return self.D_V / (self.h_um * self.h_um)

    @property
    def dv_steps(self):
        """Coupled steps per vessel update."""
        return int(round(self.dv_min / self.dt_min))

    def with_(self, **kw):
        return replace(self, **kw)


DEFAULT = Params()

# Philox stream identifiers (third counter word)
STREAM_INIT = 0
STREAM_KILL = 1
STREAM_VESSEL = 4   # (2 and 3 draw the surrogate trainer's weights and minibatches)

# cell codes of the cellular module
EMPTY, CANCER, STROMA = 0, 1, 2

# CA proposal codes: 0..25 = Moore direction, then these
CODE_NOSPACE = 26
CODE_KILL = 27
CODE_NONE = 255
