// Internal declarations shared by the HIP translation units of libhca.
// Device-side parameter block, replicate / work tables and the launchers
// each kernel file exports to the runtime.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hca.h"

// What every context starts with: the storage precision of its solved
// fields (64 or 32), which selects the runtime instance that owns it.
struct hca_ctx {
  int precision;
};

namespace hca {

// Start/stop events for the next kernel launched through hca_launch: they
// then bracket that kernel's own execution (the packet processor stamps
// them), not the dispatch gap before it.  Set by the runtime's kernel timer,
// consumed by one launch.
struct KernelEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local KernelEvents g_kernel_events;

template <typename F, typename... Args>
inline void hca_launch(F kernel, dim3 grid, dim3 block, unsigned shmem, hipStream_t s,
                       Args... args) {
  if (g_kernel_events.start) {
    const KernelEvents e = g_kernel_events;
    g_kernel_events = KernelEvents{};
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, e.start, e.stop, 0u, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
  }
}

constexpr int kBlock = 256;        // threads per workgroup (all kernels but the two below)
constexpr int kF3Block = 512;      // level 0's fused smoothing passes (tiles tx x 512/tx)
constexpr int kFlatChunk = 1024;   // voxels per flat work item (4 per thread)
constexpr int kMaxFlatBlocksPerRep = 2048;

// CA proposal codes: 0..25 Moore direction (ascending gid order), then:
constexpr uint8_t kCodeNoSpace = 26;
constexpr uint8_t kCodeKill = 27;
constexpr uint8_t kCodeNone = 255;

constexpr uint64_t kStreamInit = 0;
constexpr uint64_t kStreamKill = 1;
constexpr uint64_t kStreamVessel = 4;   // (2, 3: the surrogate trainer's draws)

// Model constants as the kernels use them.
struct DevParams {
  double dt, inv_dt;
  double aK, aG;              // D/h^2 of oxygen and drugs
  double r_k, K0, phi_K, K1;
  double psi_G, kappa_G;
  double k_pk[2], G_ref[2];
  int b_int[2];
  double k1, k1p, K_p53, k2, k2p, k2pp, J5, K_V, K_phi, T_cycle;
  int nsub;
  // the field solves: nsub_pde theta-scheme substeps of tau = dt / nsub_pde
  int nsub_pde;
  double tau, inv_tau, theta;
  // drug 2 plasma: exact Michaelis-Menten elimination when pk_mm
  int pk_mm;
  double mm_vmax, mm_km;
  // extracellular VEGF (field 3 of the solver arrays) and the vessel update
  int vegf;
  int nf;                     // fields solved per replicate: 3, or 4 with vegf
  double aV, psi_V, sec_V;
  long long dv_steps;         // coupled steps per vessel update
  double V_low, V_high, p_death, birth_per_V, w_new;
  // third drug (field 3 of the solver arrays): three-compartment plasma
  // propagator exp(M t) = S diag(e^{lam t}) S^-1 (row-major 3x3), its kill
  // trial; fV = the VEGF field's index (3 + drug3)
  int drug3, fV;
  double epi_lam[3], epi_S[9], epi_Si[9];
  double G_ref3;
  int b3;
};

// One replicate on the device, or (in the solver's tables) one linear system:
// system s = field * nreps + rep, field 0 oxygen, 1 and 2 the drugs, then
// the third drug (drug3 option) and the extracellular VEGF (vegf option), its
// unknowns at [off, off + n) of the nf x total-voxel solver arrays.
struct RepDev {
  int nx, ny, nz, pad0;
  long long off;              // first voxel in the concatenated arrays
  long long n;                // nx*ny*nz
  unsigned long long seed;
  int flat_b0, flat_nb;       // range in the flat block table
  int tile_b0, tile_nb;       // range in the stencil tile table
  int ftile_b0, ftile_nb;     // systems: range in level 0's fused-smoothing tile table
  int ndose[3];
  int dose_off;               // into the dose arrays (3*HCA_MAX_DOSES per rep)
  int tx;                     // stencil tile width (tile = tx x (kBlock/tx) columns)
  double a;                   // systems: face coupling D/h^2 of the field
};

// Work item of the flat kernels: voxels [begin, end) of one lattice.
struct FlatBlk {
  int rep, pad;
  long long begin, end;
};

// Work item of the stencil kernels: a TX x TY column tile over [z0, z1).
struct Tile {
  int rep;
  short x0, y0;
  short z0, z1;
  int pad;
};

// Per-replicate scalars of one conjugate-gradient solve.
struct SolveScal {
  double bb;        // ||b||^2
  double rr;        // ||r||^2
  double rz;        // r.z of the current direction
  double rzo;       // r_new . z_old (flexible CG)
  double rzn;       // r_new . z_new
  double pq;        // p.Ap
  double alpha, beta;
  double rr0;       // ||r_0||^2 of this solve
  // The multigrid works in FP32 on r sc (r32 = r sc) and returns z sc: sc is a
  // power of two near 1/rms(r), so the scaling is exact and keeps a decayed
  // field's tiny residual inside FP32's range; isc = 1/sc unscales z in FP64
  // (isc_prev: the scale of the previous z).
  double sc, isc, isc_prev;
  int it, done, conv, first;
};

// Per-replicate event counters (integers: order-independent sums).
struct Counters {
  unsigned long long committed, kills, divisions, nospace, lost;
  unsigned long long n_cancer, n_stroma, n_empty, n_vessel;
  unsigned long long nonfinite;
  unsigned long long total_divisions, total_kills;
  unsigned long long sur_voxels, sur_fallbacks;   // ODE phase with the surrogate
  unsigned long long births, deaths;              // vessel update of the last step
  unsigned long long total_births, total_deaths;
};

struct Work {
  int nreps;
  const RepDev* reps;
  const FlatBlk* flat;
  int nflat;
  const Tile* tiles;
  int ntiles;
  int max_blocks;             // persistent grid size (multiple of 8)
};

// Launch shape of the work-item kernels (process-wide, set once from the
// tuning knobs): with xcd_remap the grid is a multiple of 8 and work_range
// deals each XCD one contiguous run of work items; otherwise the grid is not
// a multiple of 8 and workgroup b takes run b.
extern int g_xcd_remap;

// Tile kernels: runs of kXcdChunk consecutive tiles per XCD (tile_range)
// when g_tile_remap is set; the grid is then n rounded up to 8 * kXcdChunk.
constexpr int kXcdChunk = 16;
extern int g_tile_remap;
inline int grid_tiles(int n, int max_blocks) {
  if (g_tile_remap && n <= max_blocks) return (n + 8 * kXcdChunk - 1) / (8 * kXcdChunk) * (8 * kXcdChunk);
  int g = n < max_blocks ? n : max_blocks;
  if (g < 1) g = 1;
  if (g % (8 * kXcdChunk) == 0) g += 1;
  if (g_xcd_remap)
    g = (g + 7) / 8 * 8;
  else if (g % 8 == 0)
    g += 1;
  return g;
}

// Grid of a launch over the n fused-smoothing tiles: one workgroup per tile,
// a multiple of 8 runs of `chunk` tiles (see ftile_of).
inline int grid_ftiles(int n, int chunk) {
  const int r = 8 * chunk;
  return (n + r - 1) / r * r;
}

// Grid of a launch over n work items, at most max_blocks workgroups.
inline int grid_for(int n, int max_blocks) {
  int g = n < max_blocks ? n : max_blocks;
  if (g < 1) g = 1;
  if (g_xcd_remap)
    g = (g + 7) / 8 * 8;
  else if (g % 8 == 0)
    g += 1;
  return g;
}

// ---- launchers (defined in the .hip files) --------------------------------
// setup / init / plasma kinetics (k_setup.hip)
// Plasma levels at the ends of field substep j: g0[3 rep + drug] at the end,
// g0[3 nreps + 3 rep + drug] at the start (drug 2, the third, with drug3).
void launch_plasma(hipStream_t s, const Work& w, const DevParams& p, const long long* d_step,
                   int j, const double* dose_t, const double* dose_a, double* g0);
// Field storage: T = double (precision 64) or float (precision 32) for the
// solved fields, their solver arrays and their guess history; arithmetic is
// FP64 in both (a value is rounded to T when it is stored).  P, V_c, phi and
// the vessel map are FP64 in both.
template <typename T>
void launch_setup_o2(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L,
                     const double* vw, const T* K, T* c, T* b, int steady);
// All systems of a field substep at once: F = [K | G1 | G2] (3 x ntot), then
// G3 (drug3) and V (vegf, its source from Vc); c and b of the same layout.
// With Fprev, the same pass also forms the solves' initial guess of the
// fields in xmask as launch_extrapolate does (mode xmode; theta = 1 only:
// a theta < 1 right-hand side still reads F afterwards), the value it
// extrapolates from going to Fprev_out (Fprev, or the buffer that takes its
// role when the history rotates).  keep_c: the c of the fields but oxygen (a
// function of the vessel map and the constants) is already stored and is
// not written again.
template <typename T>
void launch_setup_step(hipStream_t s, const Work& w, const DevParams& p, long long ntot,
                       const uint8_t* L, const double* vw, T* F, const double* Vc,
                       const double* g0, T* c, T* b, const T* Fprev, T* Fprev_out, unsigned xmask,
                       int xmode, int keep_c);
// Newton step on the oxygen uptake at the new value: c, b of the oxygen
// systems (the first ntot entries) from the iterate K and the linearised
// substep's right-hand side b_lin.
template <typename T>
void launch_setup_o2_newton(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L,
                            const double* vw, const T* K, const T* b_lin, T* c, T* b);
// Crank-Nicolson-type substeps (theta < 1): b += (1 - theta) a Lap F per field.
template <typename T>
void launch_rhs_lap(hipStream_t s, const Work& w, const DevParams& p, long long ntot, const T* F,
                    T* b);
// Initial guess of the solves of the fields in fmask (mode 1: F <- 2F - Fprev;
// mode 2: F <- F (F / Fprev) where 0 < F < Fprev) and Fprev <- F (the values
// at the previous solve of each field).
template <typename T>
void launch_extrapolate(hipStream_t s, const Work& w, long long ntot, int nf, unsigned fmask, int mode,
                        T* F, T* Fprev);
template <typename T>
void launch_init_cells(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L,
                       const T* K, double* P, double* Vc, double* phi);
// dst[i] = src[i] for i < n between the two storage types (hca_fields and
// the state blobs are FP64 at the boundary).
void launch_convert(hipStream_t s, const float* src, double* dst, long long n);
void launch_convert(hipStream_t s, const double* src, float* dst, long long n);

// solver (k_solver.hip)
template <typename T>
struct SolverBufsT {
  T *r, *z, *p0, *p1, *q;        // z: Jacobi preconditioner only
  float* z32;                    // z of the multigrid preconditioner (FP32 result)
  float* r32;                    // FP32 copy of r for the multigrid's fine level
  T* dinv;                    // 1/diag(A), written by the start kernel (Jacobi)
  int jacobi;                 // 1: Jacobi preconditioner inside the update kernel
  double* partial;            // per work item
  unsigned* counter;          // per replicate
  SolveScal* ss;              // per replicate
  int* ndone;                 // replicates finished
};
// Systems whose field (s / nrep) is not in field_mask are marked finished.
template <typename T>
void launch_cg_start(hipStream_t s, const Work& w, double rtol, int maxit, const T* c, const T* b,
                     const T* x, const SolverBufsT<T>& sb, unsigned field_mask, int nrep);
// Reduce kernels (one workgroup per replicate) that follow the kernels
// producing partial sums: start (b.b, r.r, r.z), apply (p.q), update
// (r.r, r.z_old, r.z'), and the preconditioner's r.z'.
// RED_RZ sums partials per stencil tile, RED_RZF per fused-smoothing tile.
enum ReduceKind { RED_START = 0, RED_APPLY = 1, RED_UPDATE = 2, RED_RZ = 3, RED_RZF = 4 };
template <typename T>
void launch_cg_reduce(hipStream_t s, const Work& w, const SolverBufsT<T>& sb, int kind, double rtol,
                      int maxit, unsigned field_mask = 7u, int nrep = 1);
// One iteration is launch_cg_apply (with the iteration's parity: the
// direction p alternates between p0 and p1) then launch_cg_update.  The apply
// also makes the previous iteration's x += alpha p (x: the solved field), so
// a solve ends with launch_cg_finish for the last one.
template <typename T>
void launch_cg_apply(hipStream_t s, const Work& w, const T* c, T* x, const SolverBufsT<T>& sb, int parity);
// The apply kernel alone (no reduce), for the tile autotuner.
template <typename T>
void launch_cg_apply_kernel(hipStream_t s, const Work& w, const T* c, T* x, const SolverBufsT<T>& sb,
                            int parity);
template <typename T>
void launch_cg_update(hipStream_t s, const Work& w, double rtol, int maxit, const SolverBufsT<T>& sb);
template <typename T>
void launch_cg_finish(hipStream_t s, const Work& w, T* x, const SolverBufsT<T>& sb);
// The solves' initial guess (x0_extrapolate = 3) for the systems of the
// fields in fmask: F <- the best (smallest residual for this solve's system)
// of the least-squares fits in span(A F, A (F - Fprev), A (Fprev - Fprev2))
// and the geometric extrapolation; Fprev2 <- Fprev, Fprev <- F, or with
// rotate Fprev2 <- F alone (the caller then swaps the two buffers' roles: one
// stored value per voxel fewer).  part: kGuessPartsPerTile doubles per tile
// of w; alpha: 4 per system.
constexpr int kGuessPartsPerTile = 12;
template <typename T>
void launch_guess_projection(hipStream_t s, const Work& w, const T* c, const T* b, T* F, T* Fprev, T* Fprev2,
                             double* part, double* alpha, unsigned fmask, int nrep, int rotate);

// ---- geometric multigrid (k_mg.hip) ---------------------------------------
constexpr int kMaxLevels = 16;
constexpr int kCoarseThreads = 1024;
constexpr int kCoarseMaxCellsPerThread = 8;
// LDS floats per cell of a coarse-solve level: two iterates, r, D^-1, gx, gy, gz
constexpr int kCoarseLdsPerCell = 7;

// One replicate at one multigrid level.  Level k cell I covers fine cells
// [I 2^k, min((I+1) 2^k, n0)) per axis; dims n_k = ceil(n_{k-1} / 2).
struct MgRep {
  int nx, ny, nz;
  int k;
  int n0x, n0y, n0z;
  int active;               // 1: level smoothed by the global kernels (k < kc)
  long long off;            // first cell of this replicate in the level arrays
  int tile_b0, tile_nb;     // smoothing tiles (active levels)
  int rtile_b0, rtile_nb;   // tiles of the cells this level receives by restriction
  int tx;
  float a;                  // face coupling D/h^2 of the system's field
};

struct MgLevel {
  const MgRep* reps;        // [nreps]
  const Tile* tiles;        // smoothing tiles, reps with k < kc
  int ntiles;
  const Tile* rtiles;       // restriction-target tiles, reps with 1 <= k <= kc
  int nrtiles;
  const Tile* ftiles;       // level 0: tiles of the fused smoothing passes (deeper in z)
  int nftiles;
  int fchunk;               // level 0: fused tiles per XCD run (about eight rows of tiles)
  float *c, *dinv, *r, *u, *ualt;
};

// The levels kc.. of one replicate, solved by one workgroup in LDS.
struct MgCoarseRep {
  int nlev;                 // LDS levels (kc .. kc+nlev-1), the last has one cell
  int kc;
  int n0[3];
  int dims[kMaxLevels][3];
  // LDS: the system's precomputed block (pre_len floats, as in coarse_pre),
  // then each level's (ua, ub, r) block at pre_len + lds_off[j]
  int lds_off[kMaxLevels];
  long long off_kc;         // replicate offset in the level-kc arrays
  long long pre_off;        // this system's block in MgBufs::coarse_pre (a multiple of 4)
  int pre_lev[kMaxLevels];  // level j's [D^-1 | gx | gy | gz] within the block
  int pre_len;              // floats in the block (a multiple of 4)
  const float* r_kc;        // this system's level-kc r and u (level arrays + off_kc)
  float* u_kc;
  float a;
};

struct MgBufs {
  MgLevel lev[kMaxLevels];
  int nlev_glob;            // max over replicates of kc
  const MgCoarseRep* coarse;
  float* coarse_pre;        // per solve: couplings and D^-1 of the coarse-solve levels
  int coarse_lds_bytes;
  float w_a, w_b;            // Jacobi weights: pre-sweeps (w_a, w_b), post-sweeps (w_b, w_a)
  float w0[3];              // level 0: pre-sweeps (w0[0], w0[1], w0[2]), post-sweeps reversed
  int fused;                // fused smoothing passes (k_mg_prefused, k_mg_postfused): level 0, and
                            // the coarser levels with ftiles
  float** lev_c;            // device arrays of the per-level pointers
  float** lev_r;
  float** lev_u;
};

// Allow the coarse-solve kernels `bytes` of dynamic LDS (above 64 KiB).
hipError_t mg_set_coarse_lds(int bytes);
template <typename T>
void launch_mg_prepare(hipStream_t s, const Work& w, const MgBufs& mg, const T* c);
// One V-cycle on the residual sb.r, result in sb.z; finishes the flexible-CG
// scalars (r.z, beta) with a RED_RZ reduce.
// `hook(ctx, segment, begin)` brackets the launches of each segment (for
// kernel timing); segments: see MgSegment.
enum MgSegment { MG_PRE0 = 0, MG_RESTRICT0, MG_DOWN, MG_COARSE, MG_UP, MG_POST1_0, MG_POST2_0, MG_SWEEP0,
                 MG_PRE3_0, MG_POST3_0 };
typedef void (*MgHook)(void* ctx, int segment, int begin);
template <typename T>
void launch_mg_vcycle(hipStream_t s, const Work& w, const MgBufs& mg, const SolverBufsT<T>& sb,
                      MgHook hook, void* hook_ctx);

// The last CG iteration's x += alpha p of a solve of every field (the systems
// f * nrep + r of SolverBufsT, f < nf), left to the first kernel that reads
// the fields after the solve: the ODE phase, which streams every voxel once
// anyway and is bound by its arithmetic.  Kernels take it by a pointer to
// device memory (null: nothing left to make), read per run of voxels, so its
// fields hold no registers over the kernel.
template <typename T>
struct CgFinish {
  T* x;                 // the field array: nf fields of ntot voxels
  const T* p0;          // the double-buffered directions (same layout)
  const T* p1;
  const SolveScal* ss;  // per system: it (0: no iteration to finish), alpha
  long long ntot;
  int nf, nrep;
};

// ODE (k_ode.hip); fin (device memory, or null): a deferred solve end, made
// for each run of voxels before the run's fields are read.
template <typename T>
void launch_ode(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L, const T* K,
                double* P, double* Vc, double* phi, const CgFinish<T>* fin);

// CA and stats (k_ca.hip)
// The committed cancer cells (phi >= 1) of a step, listed by the propose
// pass's scan per flat work item: item it's cells (local voxel indices, in
// voxel order) at cells[first voxel of the item ...], item_n[it] of them.
struct CaList {
  long long* cells;   // one slot per voxel
  int* item_n;        // per flat work item
};
// The plain integrator (as launch_ode) on the voxels listed per flat work
// item, list.item_n[it] of them at list.cells[first voxel of the item ...].
template <typename T>
void launch_ode_list(hipStream_t s, const Work& w, const DevParams& p, const uint8_t* L, const T* K,
                     double* P, double* Vc, double* phi, CaList list);
// code = win = NONE everywhere, the committed cells listed, then each listed
// cell's decision (kill, NOSPACE or the daughter's direction) into code.
template <typename T>
void launch_ca_propose(hipStream_t s, const Work& w, const DevParams& p, const long long* d_step,
                       const uint8_t* L, const double* vw, const T* K, const T* G1, const T* G2,
                       const T* G3, const double* phi, uint8_t* code, uint8_t* win, CaList list);
// For each listed cell that proposes a daughter site: the winner among the
// site's proposing neighbours into win (every proposer of a site writes the
// same value).
void launch_ca_resolve(hipStream_t s, const Work& w, const double* phi, const uint8_t* code,
                       uint8_t* win, CaList list);
// Event and census counts: each flat work item stores kCounterSlots partials
// (part[item * kCounterSlots + k]); a one-workgroup-per-replicate reduce
// then writes the replicate's counters.
constexpr int kCounterSlots = 8;
enum CounterKind { CNT_CA = 0, CNT_STATS = 1, CNT_SUR = 2, CNT_VESSEL = 3 };
void launch_counters_reduce(hipStream_t s, const Work& w, const unsigned long long* part,
                            Counters* cnt, int kind);
void launch_ca_finalize(hipStream_t s, const Work& w, uint8_t* L, double* phi, double* P,
                        double* Vc, const uint8_t* code, const uint8_t* win,
                        unsigned long long* part, Counters* cnt);
// The non-finite scan covers the nf solved fields (F, nf x ntot) and P, V_c, phi.
template <typename T>
void launch_stats(hipStream_t s, const Work& w, const uint8_t* L, const double* vw, const T* F,
                  int nf, long long ntot, const double* P, const double* Vc, const double* phi,
                  unsigned long long* part, Counters* cnt);
// Vessel birth-death update of the step n -> n+1 when (n + 1) is a multiple
// of dv_steps (else only zero event counts), from V and the cell map after
// the CA; updates vw in place.
template <typename T>
void launch_vessel(hipStream_t s, const Work& w, const DevParams& p, const long long* d_step,
                   const uint8_t* L, const T* V, double* vw, unsigned long long* part, Counters* cnt);
// what: 1 CA events, 0 census and non-finite count, 2 surrogate counts.
void launch_zero_counters(hipStream_t s, Counters* cnt, int nreps, int what);
void launch_advance(hipStream_t s, long long* d_step);
// Counts, in replicate rep, cell codes outside {0,1,2}, cells on vessel
// voxels and non-finite or negative vessel weights.
void launch_validate_cells(hipStream_t s, const Work& w, const uint8_t* L, const double* vw,
                           int rep, unsigned long long* bad);

}  // namespace hca
