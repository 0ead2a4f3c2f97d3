/*
 * hca.h - C ABI of the MI355X (gfx950) coupled time step of the stochastic
 * hybrid cellular automaton (HCA) of Lai et al., "A scalable solver for a
 * stochastic, hybrid cellular automaton model of personalized breast cancer
 * therapy".
 *
 * The library advances, for one or many independent replicates, the state
 *   L   uint8 cell map (0 empty, 1 cancer, 2 stroma)      (cellular module)
 *   K   oxygen pressure, mmHg                              (Eq. oxygen)
 *   G1  drug 1 (cyclophosphamide-like) concentration       (Eq. chemo)
 *   G2  drug 2 (fluorouracil-like, linear regime)          (Eq. chemo)
 *   P   intracellular p53                                  (Eq. odep53)
 *   Vc  intracellular VEGF                                 (Eq. odevegf)
 *   phi cell-cycle clock                                   (Eq. cellcycle)
 * on a cubic voxel lattice with a perfusion map w (0 = no vessel), by the
 * coupled step of Algorithm 1: implicit reaction-diffusion solves of oxygen
 * and the drugs, the intracellular ODEs, then the cellular automaton.
 * Options (hca_params): a third drug G3 (epirubicin), the extracellular VEGF
 * V with the vessel birth-death update (w then changes), field substeps with
 * a theta scheme, Newton steps on the oxygen uptake, exact Michaelis-Menten
 * fluorouracil kinetics.
 *
 * Layout: every per-voxel array is x-fastest, gid = x + nx*(y + ny*z),
 * FP64 for fields and uint8 for the cell map.  All replicates live in one
 * device allocation per field, concatenated in replicate order.
 *
 * Errors: every call returns an hca_status; nothing is thrown across the ABI.
 * A failed hca_step / hca_run_phases marks the context failed: further steps
 * return HCA_E_INVALID, while hca_fields, hca_stats, hca_last_error and
 * hca_destroy still work.  Contexts are independent and not thread-safe; one
 * context issues all its work on one HIP stream.
 */
#ifndef HCA_H
#define HCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HCA_ABI_VERSION 1
#define HCA_MAX_DOSES 64          /* per drug and replicate */

typedef enum hca_status {
  HCA_OK = 0,
  HCA_E_INVALID = -1,    /* bad argument, bad input data, or failed context   */
  HCA_E_NOMEM = -2,      /* device or host allocation failed                  */
  HCA_E_DEVICE = -3,     /* a HIP runtime call failed                         */
  HCA_E_NOCONV = -4,     /* a linear solve hit cg_maxit above cg_rtol         */
  HCA_E_NONFINITE = -5,  /* a field became NaN or Inf                         */
  HCA_E_SINGULAR = -6,   /* steady oxygen has no vessel source                */
  HCA_E_RANGE = -7       /* replicate index or buffer size out of range       */
} hca_status;

typedef enum hca_field {
  HCA_F_O2 = 0, HCA_F_DRUG1 = 1, HCA_F_DRUG2 = 2, HCA_F_CELL = 3 /* uint8 */,
  HCA_F_P53 = 4, HCA_F_VEGF_IC = 5, HCA_F_PHI = 6, HCA_F_VESSEL_W = 7,
  HCA_F_VEGF = 8 /* extracellular VEGF V; only with params.vegf */,
  HCA_F_DRUG3 = 9 /* third drug (epirubicin) in the tissue; only with params.drug3 */
} hca_field;

/* Phases of one coupled step n -> n+1 (loop body of Algorithm 1). */
enum {
  HCA_PH_O2 = 1u << 0,      /* plasma kinetics + oxygen solve                 */
  HCA_PH_DRUGS = 1u << 1,   /* plasma kinetics + the drug solves (two; three
                               with params.drug3)                            */
  HCA_PH_ODE = 1u << 2,     /* intracellular ODEs with the current K          */
  HCA_PH_CA = 1u << 3,      /* cellular automaton propose/resolve/finalize,
                               then (params.vegf) the vessel update when due  */
  HCA_PH_STATS = 1u << 4,   /* counts and non-finite check                    */
  HCA_PH_ADVANCE = 1u << 5, /* n := n + 1 at the end                          */
  HCA_PH_VEGF = 1u << 6,    /* extracellular VEGF solve (params.vegf; batched
                               with the O2 and drug solves of the same call)  */
  HCA_PH_ALL = 127u
};

/* Model constants (Table 1) and numerical settings.  Fill with
 * hca_default_params() and override as needed. */
typedef struct hca_params {
  double h_um;         /* voxel edge, um (20)                                   */
  double dt_min;       /* coupled step, min (Table 1 cell-cycle update, 30)     */
  /* oxygen, Eq. (oxygen) */
  double D_K;          /* diffusion, um^2/min                                   */
  double r_k;          /* vessel supply per unit perfusion weight, 1/min        */
  double K0;           /* blood oxygen, mmHg                                    */
  double phi_K;        /* uptake rate per occupied voxel, mmHg/min              */
  double K1;           /* half-maximal uptake, mmHg                             */
  /* drugs, Eq. (chemo) */
  double D_G;          /* diffusion, um^2/min                                   */
  double psi_G;        /* decay, 1/min                                          */
  double kappa_G;      /* vessel transfer per unit perfusion weight, 1/min      */
  double k_pk[2];      /* plasma elimination rates, 1/min                       */
  double G_ref[2];     /* kill-probability normalisation of each drug           */
  int32_t b_int[2];    /* dose-response shape b of I(x; 1, b), integer >= 1     */
  /* intracellular module, Eqs. (odep53), (odevegf), (cellcycle) */
  double k1, k1p, K_p53, k2, k2p, k2pp, J5, K_V, K_phi, T_cycle;
  int32_t ode_substeps;    /* RK4 sub-steps of V_c per coupled step (30)        */
  /* linear solver */
  int32_t precond;         /* 0 = Jacobi, 1 = geometric multigrid V-cycle       */
  double cg_rtol;          /* stop when ||r||_2 <= cg_rtol ||b||_2              */
  int32_t cg_maxit;        /* per solve                                          */
  int32_t mg_smooth;       /* Jacobi sweeps before and after the coarse grid;
                              must be 2 (the fused smoothers)                    */
  int32_t mg_coarse_max;   /* levels with at most this many voxels (and whose
                              LDS block fits one workgroup) are solved in one
                              workgroup; default 4096                            */
  /* initialisation */
  double init_rtol;        /* steady oxygen: Picard until the nonlinear residual
                              is below init_rtol ||b||                          */
  int32_t init_maxit;      /* Picard iterations                                  */
  int32_t profile;         /* time kernels with HIP events (hca_kernel_time):
                              0 off, 1 every kernel class, k + 2 class k only  */
  int32_t graphs;          /* 1: replay captured HIP graphs of CG iterations
                              (only while profile = 0); 0: direct launches     */
  int32_t autotune;        /* 1: pick the stencil tiling of the batch by
                              timing candidates at init (hca_tile_shape);
                              0: fixed heuristic from each lattice's size
                              (bit-identical alone or in any batch)           */
  /* time stepping of the fields inside a coupled step (Algorithm 1 solves the
     PDEs with a 1-min step, i.e. 30 substeps of the 30-min coupled step) */
  int32_t pde_substeps;    /* m >= 1 implicit substeps of dt_min/m (1)          */
  double pde_theta;        /* theta scheme in [1/2, 1]: 1 backward Euler (1),
                              1/2 Crank-Nicolson; plasma levels at both ends
                              of a substep, O2 uptake linearised at its start;
                              theta < 1 can oscillate below K = 0 after a
                              vessel change, where the uptake is continued by
                              its tangent phi_K K/K1 and the ODEs see 0        */
  int32_t o2_newton;       /* 0: the paper's linearised O2 uptake (0); k > 0:
                              then k Newton steps per substep on the uptake
                              phi_K K/(K1 + K) at the new value (each one more
                              O2 solve), 0 <= k <= 20                           */
  /* drug 2 (fluorouracil) plasma elimination */
  int32_t pk_mm;           /* 0: linear regime, rate k_pk[1] (0); 1: the exact
                              Michaelis-Menten model dG/dt = -v_max G/(k_m + G)  */
  double mm_vmax;          /* v_max, ug/mL/min (1.75)                           */
  double mm_km;            /* k_m, ug/mL (27)                                   */
  /* extracellular VEGF, Eq. (vac_v) with no Avastin, and the vascular module,
     Eq. (vascular_module).  With vegf = 1 the state gains the field V
     (HCA_F_VEGF, 0 at init), solved in every coupled step with the source
     sec_V V_c on occupied voxels (V_c of the step's start), and every dv_min
     the vessel map changes: a vessel whose V is outside [V_low, V_high] is
     removed with probability p_death; an empty non-vessel voxel with V inside
     becomes a vessel of weight w_new with probability birth_per_V V (one
     uniform per voxel: Philox counter (gid, n+1, 4, 0), key (seed, 0); an
     event when u < probability). */
  int32_t vegf;            /* 0 off (0), 1 on                                   */
  double D_V;              /* diffusion, um^2/min (3.52e3)                      */
  double psi_V;            /* decay, 1/min (1e-2)                               */
  double sec_V;            /* secretion slope a, 1/min (6.66e-6)                */
  double dv_min;           /* vessel update interval, min (720); a whole
                              multiple of dt_min                                */
  double V_low, V_high;    /* viability window, ug/mL (1e-6, 1e-4)             */
  double p_death;          /* in [0, 1] (0.05)                                  */
  double birth_per_V;      /* mL/ug, birth_per_V * V_high <= 1 (100)           */
  double w_new;            /* perfusion weight of a new vessel, > 0 (1)         */
  /* third drug, epirubicin: three-compartment plasma kinetics with the
     plasma level G0 and two peripheral compartments (amounts over the plasma
     volume w1), k10 = cl/w1, k12 = q2/w1, k21 = q2/w2, k13 = q3/w1, k31 = q3/w3:
       G0' = -(k10 + k12 + k13) G0 + k21 G1 + k31 G2, G1' = k12 G0 - k21 G1,
       G2' = k13 G0 - k31 G2;
     a bolus (hca_replicate.dose_*3) resets G0 to amount x G_ref3, the
     peripheral compartments keep their content.  With drug3 = 1 the tissue
     field G3 (HCA_F_DRUG3, 0 at init) follows Eq. (chemo) with D_G, psi_G,
     kappa_G, and a committed cell draws a third kill trial
     I(G3/G_ref3; 1, b_int3) with the third word of its kill Philox block. */
  int32_t drug3;           /* 0 off (0), 1 on                                   */
  double epi_w1, epi_w2, epi_w3;   /* compartment volumes, mL (18e3, 957e3, 25e3) */
  double epi_q2, epi_q3;   /* intercompartmental clearances, mL/min (918, 250)  */
  double epi_cl;           /* elimination clearance, mL/min (983)               */
  double G_ref3;           /* kill-probability normalisation (1)                */
  int32_t b_int3;          /* dose-response shape, 1..64 (1)                     */
  /* initial guess of each field solve, from the field's value u at this
     solve and u_prev at the previous solve of the same field (a value written
     with hca_set_field restarts it): 0 u; 1 the linear extrapolation
     2u - u_prev; 2 the geometric one u (u / u_prev) where the voxel's value
     is positive and decaying (0 < u < u_prev), else u; 3 (default) for the
     fields other than oxygen, per system, the best (smallest residual
     ||b - A x0|| for this solve's system) of the geometric guess and the
     least-squares fits x0 = c1 u + c2 (u - u_prev) + c3 (u_prev - u_prev2)
     (c3 = 0 too), u_prev2 the value at the solve before u_prev's; oxygen as
     2.  The stopping rule, hence the solve's accuracy, is the same for all
     four; the guess changes the iteration counts. */
  int32_t x0_extrapolate;
  /* storage precision of the solved fields (K, G1, G2, G3, V), their solver
     arrays and their guess history: 64 (default) FP64; 32 FP32, half the
     bytes of the solves (the arithmetic stays FP64; a value is rounded to
     FP32 where it is stored).  The solves then stop at a relative residual of
     max(cg_rtol, 1e-8), FP32 storage bounding what they can attain, and the
     steady-oxygen initialisation runs in FP64 (its operator amplifies
     residuals about 1e4-fold) before the state is rounded to FP32.  P, V_c,
     phi, the vessel map and the cellular automaton are FP64 either way;
     hca_fields, hca_set_field and the state blobs stay FP64 (converted). */
  int32_t precision;
  /* multigrid smoothing (precond = 1): 1 (default) runs level 0's three
     sweeps before the coarse-grid correction and the restriction as one pass
     over the lattice, and its three sweeps after it as another (the
     intermediate iterates stay on chip); a coarser level whose cells are all
     full 2^k-cubes and which holds at least 2 M cells over all systems does
     the same with its two sweeps per side; 0 one kernel per sweep.  The two
     compute the same V-cycle up to the rounding order of the neighbour
     sums. */
  int32_t mg_fuse;
} hca_params;

/* One replicate's inputs.  hca_init deep-copies every array; the caller keeps
 * ownership.  Host pointers. */
typedef struct hca_replicate {
  int32_t nx, ny, nz;          /* lattice, each >= 1 (nz = 1: the paper's 2-D) */
  uint64_t seed;               /* Philox key word 0                            */
  const uint8_t* cell;         /* nx*ny*nz codes in {0,1,2}                    */
  const double* vessel_w;      /* nx*ny*nz, finite, >= 0; no cell where w > 0  */
  int32_t n_doses[2];          /* doses per drug, <= HCA_MAX_DOSES             */
  const double* dose_t_min[2]; /* dose times (min), ascending                  */
  const double* dose_amt[2];   /* dose amounts, multiples of G_ref             */
  int32_t n_doses3;            /* third drug (read only with params.drug3)      */
  const double* dose_t_min3;
  const double* dose_amt3;
} hca_replicate;

typedef struct hca_stats_s {
  int64_t step;                /* index n of the current state                 */
  int64_t n_cancer, n_stroma, n_empty, n_vessel;
  /* cellular-automaton events of the last step */
  int64_t committed, divisions, kills, nospace, lost;
  /* cumulative since init */
  int64_t total_divisions, total_kills;
  /* last solve per field (O2, drug 1, drug 2) */
  int32_t cg_iters[3];
  double cg_relres[3];
  int32_t nonfinite;           /* 1 if a NaN/Inf was seen by the last stats pass */
  int32_t init_picard_iters;
  /* last ODE phase with a surrogate set: occupied voxels advanced by the
   * network, and by the plain integrator (threshold margin or range) */
  int64_t sur_voxels, sur_fallbacks;
  /* VEGF option: the last V solve, and the vessel events of the last step
   * (0 between update times) and since init */
  int32_t cg_iters_vegf;
  double cg_relres_vegf;
  int64_t vessel_births, vessel_deaths, total_births, total_deaths;
  /* third-drug option: its last solve */
  int32_t cg_iters_drug3;
  double cg_relres_drug3;
} hca_stats_t;

typedef struct hca_ctx hca_ctx;

/* ---- ODE surrogate --------------------------------------------------------
 * A 6 -> 64 -> 64 -> 64 -> 3 perceptron with GELU (erf form) after each
 * hidden layer that maps a voxel's (K, G1, G2, P, Vc, phi) before the
 * intracellular substep to the substep's update (dP, dVc, dphi), dphi being
 * the clock increment of a cancer cell (Eq. cellcycle).  It evaluates in
 * bfloat16 on the matrix cores with FP32 accumulation. */
#define HCA_MLP_NIN 6
#define HCA_MLP_NHID 64
#define HCA_MLP_NOUT 3
#define HCA_MLP_NPARAM 8963

typedef struct hca_mlp {
  /* HCA_MLP_NPARAM FP32 values: W1 (64x6, row-major, row = output unit), b1,
   * W2 (64x64), b2, W3 (64x64), b3, W4 (3x64), b4.  Host or device memory
   * (theta_is_device); hca_set_surrogate copies it. */
  const float* theta;
  int32_t theta_is_device;
  float in_mean[HCA_MLP_NIN], in_scale[HCA_MLP_NIN];     /* x_s = (x - mean) * scale */
  float out_mean[HCA_MLP_NOUT], out_scale[HCA_MLP_NOUT]; /* y = y_s * scale + mean   */
  float in_lo[HCA_MLP_NIN], in_hi[HCA_MLP_NIN];          /* training input range     */
  int32_t box_check;   /* 1: voxels with inputs outside [in_lo, in_hi] use the
                          plain integrator                                      */
} hca_mlp;

/* Table 1 of the paper plus the readings of its silent passages. */
hca_status hca_default_params(hca_params* out);

/* Algorithm 1 initialisation for n_reps replicates: uploads the inputs, solves
 * Eq. (oxygen) with s_K = 0 by Picard iteration, sets P and V_c to the ODE
 * steady states at that oxygen on occupied voxels, draws phi ~ U(0,1) for
 * cancer cells (Philox counter (gid, 0, 0, 0), key (seed, 0)) and sets both
 * drugs to 0.  `stream` is a hipStream_t (NULL: the library creates one).
 * On success *out owns all device memory of the context. */
hca_status hca_init(hca_ctx** out, const hca_params* p, const hca_replicate* reps,
                    int n_reps, void* stream);

/* n_steps full coupled steps (all phases, advancing n each time).  Returns
 * after enqueuing and synchronising the context's stream. */
hca_status hca_step(hca_ctx* c, int n_steps);

/* The selected phases of the step n -> n+1, in Algorithm 1 order
 * (O2, drugs, ODE, CA, stats); n advances only with HCA_PH_ADVANCE. */
hca_status hca_run_phases(hca_ctx* c, unsigned mask);

/* Copy replicate `rep`'s field into dst (host or device).  dst_bytes must be
 * >= nx*ny*nz*elem (elem 1 for HCA_F_CELL, else 8): else HCA_E_RANGE. */
hca_status hca_fields(hca_ctx* c, int rep, hca_field f, void* dst, size_t dst_bytes,
                      int dst_is_device);

/* Overwrite replicate `rep`'s state field (checkpoint restore, tests).  A
 * cell map with codes outside {0,1,2} or cells on vessel voxels, and a vessel
 * map with non-finite or negative weights or vessels on cells, give
 * HCA_E_INVALID and leave the state unchanged.  HCA_F_VEGF needs vegf = 1. */
hca_status hca_set_field(hca_ctx* c, int rep, hca_field f, const void* src,
                         size_t src_bytes, int src_is_device);

/* Set the step index n of the current state (resume from a checkpoint). */
hca_status hca_set_step(hca_ctx* c, int64_t step);

/* ---- checkpoint and resume ----------------------------------------------------
 * A replicate's complete state as one self-describing blob, so that a run
 * continued from a saved state is bit-identical to the uninterrupted run (the
 * reproducibility the paper asks of its random numbers, here of the whole
 * state): the cell map, the vessel map, every solved field (K, G1, G2, and G3
 * / V with their options), P, V_c, phi, the solves' initial-guess history
 * (each field at its previous solve, and with x0_extrapolate = 3 at the solve
 * before that), the step index, the seed and the
 * cumulative event counts.  Layout: a 96-byte header (magic "HCASTATE",
 * version 1, option flags, nx, ny, nz, field count, step, seed, cumulative
 * counts), then the uint8 cell map padded to 8 bytes and FP64 arrays, all
 * x-fastest.  A context advances its replicates together, so replicates of
 * one context share the step index. */
/* Bytes of replicate rep's state blob. */
hca_status hca_state_bytes(hca_ctx* c, int rep, size_t* bytes);
/* Write replicate rep's state into dst (host or device, dst_is_device);
 * HCA_E_RANGE if dst_bytes is too small. */
hca_status hca_export_state(hca_ctx* c, int rep, void* dst, size_t dst_bytes, int dst_is_device);
/* Overwrite replicate rep's state with a blob of hca_export_state (host or
 * device).  The blob must have the replicate's lattice and seed and the
 * context's options (third drug, VEGF), and in a context of several
 * replicates the context's step; its maps are validated as hca_set_field
 * does.  Violations give HCA_E_INVALID (HCA_E_RANGE for a short buffer) and
 * leave the state unchanged.  A blob without guess history restarts the
 * extrapolation from the restored fields.  The last step's event counts
 * restart at 0. */
hca_status hca_import_state(hca_ctx* c, int rep, const void* src, size_t src_bytes,
                            int src_is_device);
/* Algorithm 1's time loop resumed from saved states instead of its
 * initialisation: like hca_init, but replicate r's cell and vessel maps, fields,
 * cell state, guess history, step and counts come from states[r] (a host
 * blob of state_bytes[r] bytes from hca_export_state), and reps[r] supplies
 * the seed, which must match, and the dose lists (its cell and vessel_w are
 * ignored).  All states must be at the same step.  No steady-oxygen solve is
 * run. */
hca_status hca_init_from_state(hca_ctx** out, const hca_params* p, const hca_replicate* reps,
                               const void* const* states, const size_t* state_bytes, int n_reps,
                               void* stream);

hca_status hca_stats(hca_ctx* c, int rep, hca_stats_t* out);

/* With params.profile set: accumulated device time (ms) and launch count of
 * kernel class `kernel` (see hca_kernel_name) since the last reset. */
hca_status hca_kernel_time(hca_ctx* c, int kernel, double* ms, int64_t* launches,
                           double* bytes_per_launch);
const char* hca_kernel_name(int kernel);
int hca_num_kernels(void);
hca_status hca_reset_kernel_time(hca_ctx* c);
/* Change params.profile of a live context (0 off, 1 every kernel class,
 * k + 2 class k only), e.g. to time a few steps after an untimed run. */
hca_status hca_set_profile(hca_ctx* c, int profile);


/* Replace the plain integrator of the ODE phase (Eqs. odep53, odevegf,
 * cellcycle) by the surrogate network: every occupied voxel takes the
 * network's update, except that a cancer cell whose updated phi would lie
 * within `margin` of the division threshold phi = 1 (cellular module), and
 * with box_check any voxel whose inputs leave the training range, is
 * advanced by the plain integrator.  net = NULL restores the plain
 * integrator.  Non-finite statistics, a zero scale or a negative margin give
 * HCA_E_INVALID and leave the setting unchanged. */
hca_status hca_set_surrogate(hca_ctx* c, const hca_mlp* net, double margin);

/* One full coupled step with the plain integrator (whether or not a
 * surrogate is set) that also records one training pair per occupied voxel of
 * every replicate, replicate-major and in gid order within a replicate:
 * X row = (K^{n+1}, G1^{n+1}, G2^{n+1}, P^n, Vc^n, phi^n) (FP32, 6 per row) and
 * Y row = (P^{n+1} - P^n, Vc^{n+1} - Vc^n, cancer-clock increment) (3 per
 * row).  X and Y are device buffers of cap_rows rows; more occupied voxels
 * than cap_rows gives HCA_E_RANGE before any work.  *n_rows = rows written. */
hca_status hca_harvest_step(hca_ctx* c, float* X, float* Y, int64_t cap_rows, int64_t* n_rows);

/* ---- surrogate training -----------------------------------------------------
 * A trainer holds a standardised copy of n_rows training pairs (X: n x 6,
 * Y: n x 3, FP32 device arrays, row-major, the caller keeps them), the
 * per-column statistics (mean and standard deviation over the set; a column
 * with zero spread gets scale 1), the parameters, and the Adam moments
 * (beta1 0.9, beta2 0.999, eps 1e-8).  Parameters start as
 * U(-sqrt(3/fan_in), sqrt(3/fan_in)) weights from Philox key (seed, 0) and
 * zero biases.  Loss: mean squared error over the batch and the three
 * standardised outputs.  One trainer per stream; not thread-safe. */
typedef struct hca_mlp_trainer hca_mlp_trainer;

hca_status hca_mlp_trainer_create(hca_mlp_trainer** out, const float* X, const float* Y,
                                  int64_t n_rows, uint64_t seed, void* stream);
/* Overwrite the parameters (host or device, HCA_MLP_NPARAM) and reset Adam. */
hca_status hca_mlp_trainer_set_params(hca_mlp_trainer* t, const float* theta, int is_device);
hca_status hca_mlp_trainer_params(hca_mlp_trainer* t, float* theta, int is_device);
/* The standardised training set (device buffers of n x 6 and n x 3). */
hca_status hca_mlp_trainer_data(hca_mlp_trainer* t, float* Xs, float* Ys);
/* Fill *out for hca_set_surrogate: statistics, range, theta = the trainer's
 * device parameters (valid until the next update or destroy), box_check 0. */
hca_status hca_mlp_trainer_export(hca_mlp_trainer* t, hca_mlp* out);
/* Gradient (device, HCA_MLP_NPARAM) and loss (host) of the batch of rows
 * idx[0..batch) (device int32, clamped to [0, n_rows)); batch a positive
 * multiple of 64, at most 65536, else HCA_E_RANGE.  No update. */
hca_status hca_mlp_gradient(hca_mlp_trainer* t, const int32_t* idx, int batch, float* grad,
                            float* loss);
/* n_steps Adam steps on minibatches drawn with replacement (Philox counter
 * (j, step, 3, 0), key (seed, 0)); losses[k] (host, may be NULL) = loss of
 * step k's batch before its update. */
hca_status hca_mlp_train(hca_mlp_trainer* t, int n_steps, int batch, float lr, float* losses);
/* One Adam step (the trainer's next step t, bias-corrected, the moments and
 * constants of hca_mlp_train) from a caller's gradient of HCA_MLP_NPARAM
 * values (host or device, is_device), e.g. one reduced over several trainers'
 * hca_mlp_gradient results.  lr > 0 and finite, else HCA_E_INVALID.  Adam
 * as defined by Kingma and Ba: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), in FP32. */
hca_status hca_mlp_apply_gradient(hca_mlp_trainer* t, const float* grad, int is_device, float lr);
/* Network outputs for n rows of X (device) into Y (device): raw = 1 takes
 * and returns model values, raw = 0 standardised ones. */
hca_status hca_mlp_eval(hca_mlp_trainer* t, const float* X, int64_t n, int raw, float* Y);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, training or serving loops that forbid hipMalloc): the gradient and
 * loss of hca_mlp_gradient without a trainer and without any allocation.
 * theta (HCA_MLP_NPARAM), Xs (n_rows x 6) and Ys (n_rows x 3, standardised
 * rows as hca_mlp_trainer_data returns them) and idx (batch int32 row
 * indices, clamped to [0, n_rows)) are device inputs; grad (HCA_MLP_NPARAM)
 * and loss (one float, may be NULL: the batch's mean squared error) are
 * device outputs.  batch must be a positive multiple of 64 of at most
 * HCA_MLP_NOALLOC_MAX_BATCH, else HCA_E_RANGE before any work.  The work is
 * only enqueued on `stream` (NULL: the null stream); the caller synchronises.
 * The scratch (about 2.4 MB: packed operands, GELU table, per-64-sample
 * partials) is one static device array per GPU, held until the process ends
 * and shared by every call on that GPU: calls that overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller. */
#define HCA_MLP_NOALLOC_MAX_BATCH 4096
hca_status hca_mlp_gradient_noalloc(const float* theta, const float* Xs, const float* Ys,
                                    int64_t n_rows, const int32_t* idx, int batch, float* grad,
                                    float* loss, void* stream);
const char* hca_mlp_trainer_last_error(const hca_mlp_trainer* t);
void hca_mlp_trainer_destroy(hca_mlp_trainer* t);

/* Stencil tile of replicate `rep`: tx x ty voxel columns, tz planes deep
 * (the autotuner's choice with params.autotune = 1). */
hca_status hca_tile_shape(hca_ctx* c, int rep, int32_t* tx, int32_t* ty, int32_t* tz);

/* Block the host until all work of the context has finished. */
hca_status hca_synchronize(hca_ctx* c);

/* Human-readable reason of the context's last failure ("" if none). */
const char* hca_last_error(const hca_ctx* c);

/* Frees every resource of the context (NULL is allowed). */
void hca_destroy(hca_ctx* c);

#ifdef __cplusplus
}
#endif
#endif /* HCA_H */
