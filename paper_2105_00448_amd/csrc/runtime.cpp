// Host runtime of libhca: context, device memory, replicate / system work
// tables, the per-step phase sequence of Algorithm 1, the CG driver and the
// C ABI.
//
// The implicit solves of a step (oxygen, the two drugs, and with the options
// the third drug and the extracellular VEGF) are independent given the state
// at t^n, so they run as one batch of nf x nreps linear systems (system
// s = field * nreps + rep) through the same launches; the fields live in one
// allocation [K | G1 | G2 (| G3) (| V)] and the solver arrays have the same
// nf x total-voxel layout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hca.h"
#include "hca_internal.h"
#include "mlp_dev.h"

// This file is compiled twice: with HCA_REAL = double into namespace
// hca::rt64 (precision 64, the primary instance, which also defines the
// process-wide knobs and the precision-independent C entry points) and with
// HCA_REAL = float into hca::rt32 (precision 32: the solved fields, their
// solver arrays and guess history stored in FP32).  capi.cpp dispatches each
// call to the instance that owns the context.
#ifndef HCA_REAL
#define HCA_REAL double
#define HCA_RT_NS rt64
#define HCA_RT_PRIMARY 1
#endif
#ifndef HCA_RT_PRIMARY
#define HCA_RT_PRIMARY 0
#endif

#include "rt_api.h"

using namespace hca;

#if HCA_RT_PRIMARY
namespace hca {
thread_local KernelEvents g_kernel_events;
int g_xcd_remap = 0;    // flat kernels: measured slower (HCA_XCD_REMAP=1 to enable)
int g_tile_remap = 1;   // tile kernels: measured 4-8 % faster (HCA_TILE_REMAP=0 to disable)
}  // namespace hca
#endif

namespace hca {
namespace HCA_RT_NS {

using Real = HCA_REAL;
using SolverBufs = SolverBufsT<Real>;
constexpr int kPrecision = sizeof(Real) == 8 ? 64 : 32;
// precision 32: FP32 storage limits the attainable relative residual, so the
// solves stop at no less than this
constexpr double kRtolFloor = sizeof(Real) == 8 ? 0.0 : 1e-8;

namespace {

enum KernelClass {
  KC_PLASMA = 0, KC_SETUP, KC_CG_START, KC_CG_APPLY, KC_CG_UPDATE, KC_ODE,
  KC_CA_PROPOSE, KC_CA_RESOLVE, KC_CA_FINALIZE, KC_STATS,
  KC_MG_PREP, KC_MG_PRE0, KC_MG_RESTRICT0, KC_MG_LEVELS, KC_MG_COARSE, KC_MG_POST1_0,
  KC_MG_POST2_0, KC_MLP_APPLY, KC_VESSEL, KC_MG_SWEEP0, KC_MG_PRE3_0, KC_MG_POST3_0, KC_CG_FINISH,
  KC_GUESS, KC_COUNT
};

[[maybe_unused]] const char* kKernelNames[KC_COUNT] = {
    "k_plasma", "k_setup_step", "k_cg_start", "k_cg_apply", "k_cg_update",
    "k_ode", "k_ca_propose", "k_ca_resolve", "k_ca_finalize", "k_stats",
    "k_mg_prep0+k_mg_coarsen", "k_mg_pre<L0>", "k_mg_restrict<L0>", "mg levels >= 1 (global)",
    "k_mg_coarse", "k_mg_post1<L0>", "k_mg_post2<L0>", "k_mlp_apply", "k_vessel", "k_mg_sweep<L0>",
    "k_mg_prefused<L0>", "k_mg_postfused<L0>", "k_cg_finish", "k_guess (fit)"};

// Compulsory (algorithmic) HBM bytes per voxel of each kernel class; solver
// classes per voxel of each active system (0: not priced, latency-bound).
// e = bytes of a stored field value (8, or 4 in precision 32); the cell map
// is 1 byte, P, V_c, phi and the vessel map 8, the multigrid arrays 4.
constexpr double kE = sizeof(Real);
const double kBytesPerVoxel[KC_COUNT] = {
    0.0,            // plasma: per replicate only
    9.0 + 9 * kE,   // setup_step: read L, w, K, G1, G2; write c, b of three systems
    5 * kE,         // cg_start: read x, c, b; write r, (Jacobi: dinv, z)
    4.0 + 6 * kE,   // cg_apply, multigrid: read z (4), p_old, c, x; write p_new, q, x (the
                    // previous iteration's x += alpha p; a solve's first apply: 4 + 4 e)
    6 * kE,         // cg_update, Jacobi: read r, q, z, dinv; write r, z
    49.0 + kE,      // ode: read L, K, P, Vc, phi; write P, Vc, phi
    11.0,           // ca_propose: scan (read L, phi; write code, win); the list's decisions
                    // gather per committed cell, not per voxel
    0.0,            // ca_resolve: gathers per proposing cell only
    2.0,            // ca_finalize: read code, win (writes only where cells change)
    33.0 + 3 * kE,  // stats: read L, w, K, G1, G2, P, Vc, phi
    13.0 + kE,      // mg prepare: read c; write dinv0 (4); level 1: read c, write c1, dinv1
    12.0,           // mg pre L0: read r (FP32 copy, 4), dinv (4); write ualt (4)
    12.5,           // mg restrict L0: read u, r (4), dinv; write r1 (1/8 of 4)
    0.0,            // coarser global levels
    0.0,            // coarse workgroup levels
    16.5,           // mg post1 L0: read u, e (1/8), r (4), dinv; write ualt
    12.0 + kE,      // mg post2 L0: read ualt, r, dinv; write z (4)
    49.0 + 3 * kE,  // mlp apply: read L, K, G1, G2, P, Vc, phi; write P, Vc, phi
    9.0 + kE,       // vessel: read L, w, V (writes only where a vessel changes)
    16.0,           // mg sweep L0: read u (4), r (4), dinv (4); write u' (4)
    12.5,           // mg prefused L0: read r (4), dinv (4); write u3 (4), r1 (1/8 of 4)
    16.5 + kE,      // mg postfused L0: read u3 (4), e (1/8), r (4), dinv (4), r (stored); write z (4)
    3 * kE,         // cg_finish: read x, p; write x (once per solve)
    11 * kE};       // guess fit, per voxel of one fitted field: read x1, x2, x3, c, b (the products);
                    // read x1, x2, x3; write x0, x1, x2 (the shifted history; x0 and x1 alone
                    // when the history buffers rotate)
constexpr double kBytesSetupVegf = 8.0 + 3 * kE;   // setup_step with vegf: + read V, Vc; write c, b
constexpr double kBytesSetupDrug3 = 3 * kE;        // setup_step with drug3: + read G3; write c, b
constexpr double kBytesStatsField = kE;            // stats: per extra field scanned (V, G3)
// cg_update, multigrid: the compulsory r, q read and r written (the CG's own
// traffic; x += alpha p moved to the next apply); the kernel also reads the
// FP32 z and writes the FP32 copy of r for the multigrid (8 B more per voxel,
// not counted here)
constexpr double kBytesUpdateMg = 3 * kE;
constexpr double kBytesApplyJacobi = 7 * kE;       // cg_apply, Jacobi: z is a stored field value
constexpr double kBytesApplyX = 2 * kE;            // cg_apply's x read and write (not on a solve's first)

constexpr int kTagState = -2;   // launches over every voxel of every replicate
constexpr int kTagAll = -1;     // solver launches over every system

struct RepHost {
  int nx, ny, nz;
  long long off, n;
  uint64_t seed;
  int tx, tz;   // stencil tile: tx x (256/tx) columns, tz planes deep
};

struct ProfEntry {
  int kc;
  hipEvent_t a, b;
  int tag;       // CG iteration index of the launch, kTagAll or kTagState
  double bpv;    // bytes per active voxel
};

}  // namespace

struct Ctx : ::hca_ctx {
  Ctx() { precision = kPrecision; }
  hca_params prm;
  DevParams dp;
  int nreps = 0;
  std::vector<RepHost> reps;
  long long ntot = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t cap_stream = nullptr;              // capture only (never executes work)
  hipGraphExec_t iter_graph[2] = {nullptr, nullptr};   // two CG iterations, per solve kind
  bool graph_failed = false;
  int device = 0;

  // state
  uint8_t *L = nullptr, *code = nullptr, *win = nullptr;
  CaList ca_list{};                             // committed cells of the CA pass
  double *w = nullptr, *P = nullptr, *Vc = nullptr, *phi = nullptr;
  Real* F = nullptr;                            // [K | G1 | G2 (| G3) (| V)]
  Real *K = nullptr, *G1 = nullptr, *G2 = nullptr, *G3 = nullptr, *V = nullptr;
  // solver, nf x ntot (nf = dp.nf fields)
  Real *c = nullptr, *b = nullptr;
  SolverBufs sb{};
  bool use_mg = false;
  MgBufs mg_all{}, mg1{};                       // all systems / oxygen systems only
  std::vector<void*> mg_mem;
  double *dose_t = nullptr, *dose_a = nullptr, *g0 = nullptr;
  Real* b_o2lin = nullptr;                       // o2_newton: the linearised O2 right-hand side
  Real* Fprev = nullptr;                         // x0_extrapolate: fields of the previous solve
  Real* Fprev2 = nullptr;                        // x0_extrapolate = 3: and of the solve before
  double* d_gpart = nullptr;                     // x0_extrapolate = 3: products per solver tile
  double* d_galpha = nullptr;                    // and the choice and fit coefficients per system (4)
  CgFinish<Real>* d_fin = nullptr;               // the solve end that the ODE phase can make
  long long* d_step = nullptr;
  // replicate tables (state kernels)
  RepDev* d_reps = nullptr;
  FlatBlk* d_flat = nullptr;
  Tile* d_tiles = nullptr;
  Work work{};
  // system tables (solver kernels); sys1 is the oxygen prefix of sys_all
  RepDev* d_sys = nullptr;
  FlatBlk* d_sflat = nullptr;
  Tile* d_stiles = nullptr;
  Tile* d_ftiles = nullptr;        // level 0's fused-smoothing tiles (systems)
  int nftiles_all = 0, nftiles1 = 0;
  int fchunk = 16;                 // fused tiles per XCD run
  Work sys_all{}, sys1{};
  std::vector<long long> sys_n;
  Counters* d_cnt = nullptr;
  unsigned long long* d_cpart = nullptr;   // per flat item x kCounterSlots
  unsigned long long* d_bad = nullptr;
  // ODE surrogate (hca_set_surrogate) and training-pair harvest buffers
  bool sur_on = false;
  MlpDev net{};
  float* d_theta = nullptr;
  bf16x8* d_pack = nullptr;
  float2* d_gelu = nullptr;
  double* before = nullptr;       // 3 x ntot
  int* item_cnt = nullptr;        // per flat work item
  long long* item_off = nullptr;  // nflat + 1

  SolveScal* h_ss = nullptr;     // pinned, nf x nreps
  Counters* h_cnt = nullptr;     // pinned
  long long step = 0;
  int last_it[2] = {0, 0};       // iterations of the last step solve / init solve
  bool fin_pending = false;      // the last solve's x += alpha p left to the ODE phase
  // The fields but oxygen have a c (and so multigrid data) that follows the
  // vessel map and the constants only: true while the stored ones are current
  // (cleared by anything that writes a state field; never set with the
  // vessel update, which changes the map between steps).
  bool fixed_ops = false;
  std::vector<SolveScal> last_ss;
  int picard_iters = 0;

  bool failed = false;
  std::string err;

  // profiling
  std::vector<ProfEntry> pending;
  std::vector<hipEvent_t> free_events;
  double prof_ms[KC_COUNT] = {0};
  long long prof_n[KC_COUNT] = {0};
  double prof_bytes[KC_COUNT] = {0};
};

namespace {

hca_status fail(Ctx* c, hca_status st, const std::string& msg) {
  if (c) {
    c->err = msg;
    if (st != HCA_E_RANGE) c->failed = true;
  }
  return st;
}

#define HIPCHK(ctx, expr)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, HCA_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
}

// ---- kernel timing (params.profile) ----------------------------------------

hipEvent_t take_event(Ctx* c) {
  if (!c->free_events.empty()) {
    hipEvent_t e = c->free_events.back();
    c->free_events.pop_back();
    return e;
  }
  // timing-only events: no system-scope fence (no cache writeback and
  // invalidation between the kernels being timed)
  hipEvent_t e;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

double bpv_of(const Ctx* c, int kc) {
  if (kc == KC_CG_UPDATE && c->use_mg) return kBytesUpdateMg;
  if (kc == KC_CG_APPLY && !c->use_mg) return kBytesApplyJacobi;
  if (kc == KC_SETUP)
    return kBytesPerVoxel[kc] + (c->dp.vegf ? kBytesSetupVegf : 0.0) + (c->dp.drug3 ? kBytesSetupDrug3 : 0.0);
  if (kc == KC_STATS) return kBytesPerVoxel[kc] + (c->dp.nf - 3) * kBytesStatsField;
  return kBytesPerVoxel[kc];
}

// params.profile: 0 off, 1 every kernel class, k + 2 class k only.
inline bool prof_on(const Ctx* c, int kc) {
  return c->prm.profile == 1 || c->prm.profile == kc + 2;
}

// Times the launches issued while it is alive.  single: the first kernel
// launched (through hca_launch) carries the start/stop events itself, so the
// time is that kernel's execution; otherwise events are recorded on the
// stream before and after (a segment of several kernels, gaps included).
struct ProfScope {
  Ctx* c;
  int kc;
  int tag;
  bool single;
  double dbpv;   // added to the class's bytes per voxel for this launch
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(Ctx* c_, int kc_, int tag_, bool single_ = true, double dbpv_ = 0.0)
      : c(c_), kc(kc_), tag(tag_), single(single_), dbpv(dbpv_) {
    if (!prof_on(c, kc)) return;
    a = take_event(c);
    b = take_event(c);
    if (!a || !b) {
      if (a) c->free_events.push_back(a);
      if (b) c->free_events.push_back(b);
      a = b = nullptr;
      return;
    }
    if (single)
      g_kernel_events = KernelEvents{a, b};
    else
      (void)hipEventRecord(a, c->stream);
  }
  ~ProfScope() {
    if (!a) return;
    if (single) {
      if (g_kernel_events.start == a) {   // nothing was launched
        g_kernel_events = KernelEvents{};
        c->free_events.push_back(a);
        c->free_events.push_back(b);
        return;
      }
    } else {
      (void)hipEventRecord(b, c->stream);
    }
    c->pending.push_back(ProfEntry{kc, a, b, tag, bpv_of(c, kc) + dbpv});
  }
};

// Accumulate the pending timings.  A solver launch with tag t does work for
// the systems still iterating (iterations > t); launches that found every
// system finished are dropped, the others are priced on the active voxels.
void prof_flush(Ctx* c, const SolveScal* ss, int nsys) {
  if (c->pending.empty()) return;
  (void)hipEventSynchronize(c->pending.back().b);
  for (const ProfEntry& e : c->pending) {
    double vox = (double)c->ntot;
    if (e.tag >= kTagAll && ss) {
      vox = 0.0;
      for (int s = 0; s < nsys; ++s)
        if (e.tag == kTagAll || ss[s].it > e.tag) vox += (double)c->sys_n[s];
    }
    if (vox > 0.0) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
        c->prof_ms[e.kc] += ms;
        c->prof_n[e.kc] += 1;
        c->prof_bytes[e.kc] += e.bpv * vox;
      }
    }
    c->free_events.push_back(e.a);
    c->free_events.push_back(e.b);
  }
  c->pending.clear();
}

// Event pairs around the V-cycle's launch segments.
struct MgProf {
  Ctx* c;
  hipEvent_t start[10];   // per MgSegment
  int tag;
};

int mg_segment_class(int seg) {
  switch (seg) {
    case MG_PRE0: return KC_MG_PRE0;
    case MG_RESTRICT0: return KC_MG_RESTRICT0;
    case MG_COARSE: return KC_MG_COARSE;
    case MG_POST1_0: return KC_MG_POST1_0;
    case MG_POST2_0: return KC_MG_POST2_0;
    case MG_SWEEP0: return KC_MG_SWEEP0;
    case MG_PRE3_0: return KC_MG_PRE3_0;
    case MG_POST3_0: return KC_MG_POST3_0;
    default: return KC_MG_LEVELS;
  }
}

void mg_hook(void* p, int seg, int begin) {
  MgProf* m = (MgProf*)p;
  Ctx* c = m->c;
  if (!prof_on(c, mg_segment_class(seg))) return;
  if (begin) {
    m->start[seg] = take_event(c);
    if (m->start[seg]) (void)hipEventRecord(m->start[seg], c->stream);
    return;
  }
  if (!m->start[seg]) return;
  hipEvent_t b = take_event(c);
  if (!b) return;
  (void)hipEventRecord(b, c->stream);
  const int kc = mg_segment_class(seg);
  c->pending.push_back(ProfEntry{kc, m->start[seg], b, m->tag, bpv_of(c, kc)});
  m->start[seg] = nullptr;
}

void run_vcycle(Ctx* c, const Work& W, const MgBufs& mg, int tag) {
  MgProf mp{};
  mp.c = c;
  mp.tag = tag;
  launch_mg_vcycle(c->stream, W, mg, c->sb, mg_hook, &mp);
}

// The third drug's propagator exp(M t) = S diag(e^{lam t}) S^-1.  M (state
// G0, G1, G2) is similar to the symmetric Ms = D^{1/2} M D^{-1/2} with
// D = diag(1, w1/w2, w1/w3): Ms_00 = -(k10 + k12 + k13), Ms_11 = -k21,
// Ms_22 = -k31, Ms_01 = q2/sqrt(w1 w2), Ms_02 = q3/sqrt(w1 w3), Ms_12 = 0.
// Cyclic Jacobi rotations give Ms = Q diag(lam) Q^T; then S = D^{-1/2} Q and
// S^-1 = Q^T D^{1/2}.
void epi_propagator(const hca_params& p, DevParams& d) {
  const double k10 = p.epi_cl / p.epi_w1, k12 = p.epi_q2 / p.epi_w1, k13 = p.epi_q3 / p.epi_w1;
  const double k21 = p.epi_q2 / p.epi_w2, k31 = p.epi_q3 / p.epi_w3;
  double A[3][3] = {{-(k10 + k12 + k13), p.epi_q2 / std::sqrt(p.epi_w1 * p.epi_w2),
                     p.epi_q3 / std::sqrt(p.epi_w1 * p.epi_w3)},
                    {0.0, -k21, 0.0},
                    {0.0, 0.0, -k31}};
  A[1][0] = A[0][1];
  A[2][0] = A[0][2];
  double Q[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  for (int sweep = 0; sweep < 50; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-34 * dia) break;
    for (int a = 0; a < 2; ++a)
      for (int b = a + 1; b < 3; ++b) {
        if (A[a][b] == 0.0) continue;
        // rotation in the (a, b) plane that zeroes A[a][b]
        const double th = (A[b][b] - A[a][a]) / (2.0 * A[a][b]);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        double J[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
        J[a][a] = cs;
        J[b][b] = cs;
        J[a][b] = sn;
        J[b][a] = -sn;
        double T[3][3], N[3][3], Qn[3][3];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            T[i][j] = 0.0;
            for (int k = 0; k < 3; ++k) T[i][j] += A[i][k] * J[k][j];
          }
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            N[i][j] = 0.0;
            Qn[i][j] = 0.0;
            for (int k = 0; k < 3; ++k) {
              N[i][j] += J[k][i] * T[k][j];
              Qn[i][j] += Q[i][k] * J[k][j];
            }
          }
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            A[i][j] = N[i][j];
            Q[i][j] = Qn[i][j];
          }
        A[a][b] = A[b][a] = 0.0;
      }
  }
  const double dd[3] = {1.0, p.epi_w1 / p.epi_w2, p.epi_w1 / p.epi_w3};
  for (int i = 0; i < 3; ++i) {
    d.epi_lam[i] = A[i][i];
    for (int j = 0; j < 3; ++j) {
      d.epi_S[3 * i + j] = Q[i][j] / std::sqrt(dd[i]);
      d.epi_Si[3 * i + j] = Q[j][i] * std::sqrt(dd[j]);
    }
  }
}

DevParams make_dev_params(const hca_params& p) {
  DevParams d{};
  d.dt = p.dt_min;
  d.inv_dt = 1.0 / p.dt_min;
  d.nsub_pde = p.pde_substeps;
  d.tau = p.dt_min / p.pde_substeps;
  d.inv_tau = 1.0 / d.tau;
  d.theta = p.pde_theta;
  d.pk_mm = p.pk_mm;
  d.mm_vmax = p.mm_vmax;
  d.mm_km = p.mm_km;
  d.vegf = p.vegf;
  d.drug3 = p.drug3;
  d.nf = 3 + p.drug3 + p.vegf;
  d.fV = 3 + p.drug3;
  d.G_ref3 = p.G_ref3;
  d.b3 = p.b_int3;
  if (p.drug3) epi_propagator(p, d);
  d.aV = p.D_V / (p.h_um * p.h_um);
  d.psi_V = p.psi_V;
  d.sec_V = p.sec_V;
  d.dv_steps = std::llround(p.dv_min / p.dt_min);
  d.V_low = p.V_low;
  d.V_high = p.V_high;
  d.p_death = p.p_death;
  d.birth_per_V = p.birth_per_V;
  d.w_new = p.w_new;
  d.aK = p.D_K / (p.h_um * p.h_um);
  d.aG = p.D_G / (p.h_um * p.h_um);
  d.r_k = p.r_k;
  d.K0 = p.K0;
  d.phi_K = p.phi_K;
  d.K1 = p.K1;
  d.psi_G = p.psi_G;
  d.kappa_G = p.kappa_G;
  for (int i = 0; i < 2; ++i) {
    d.k_pk[i] = p.k_pk[i];
    d.G_ref[i] = p.G_ref[i];
    d.b_int[i] = p.b_int[i];
  }
  d.k1 = p.k1;
  d.k1p = p.k1p;
  d.K_p53 = p.K_p53;
  d.k2 = p.k2;
  d.k2p = p.k2p;
  d.k2pp = p.k2pp;
  d.J5 = p.J5;
  d.K_V = p.K_V;
  d.K_phi = p.K_phi;
  d.T_cycle = p.T_cycle;
  d.nsub = p.ode_substeps;
  return d;
}

// Tile width (tiles are tx x 256/tx columns): 32 x 8 unless the lattice is
// at most 16 wide.  The restriction kernel relies on tx in {16, 32} (a cell's
// y-neighbour in the same wavefront) and on even tile origins.
int pick_tx(int nx) {
  if (nx > 16) return 32;
  return 16;
}

// ---- the solver driver -------------------------------------------------------

// Captures two CG iterations (parities 0 and 1, with their V-cycles) of the
// systems of W into a HIP graph on the capture-only stream.  On failure the
// context falls back to direct launches for good.
bool capture_iterations(Ctx* c, const Work& W, const MgBufs& mg, double rtol, int maxit,
                        int kind) {
  hipStream_t cs = c->cap_stream;
  if (!cs) return false;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    c->graph_failed = true;
    return false;
  }
  for (int par = 0; par < 2; ++par) {
    launch_cg_apply(cs, W, c->c, c->F, c->sb, par);
    launch_cg_update(cs, W, rtol, maxit, c->sb);
    if (c->use_mg) launch_mg_vcycle(cs, W, mg, c->sb, nullptr, nullptr);
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(cs, &g);
  hipGraphExec_t ex = nullptr;
  if (e == hipSuccess && g) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
  if (e != hipSuccess || !ex) {
    c->graph_failed = true;
    return false;
  }
  c->iter_graph[kind] = ex;
  return true;
}

// Iterations of a solve's first batch before the first convergence poll: the
// previous solve's count plus this (HCA_SOLVE_LEAD; then polls every two):
// measured on the 128^3 workload, leads -1, 0, 1, 2, 3 give 2.364, 2.321,
// 2.357, 2.394, 2.425 ms per step (a poll costs about as much as one extra
// no-op iteration pair of launches).
int g_solve_lead = 0;

// Flexible CG on the systems of W (all systems: sys_all, oxygen only: sys1) for
// (diag(c) - a Lap) x = b, x = the field array F.  Systems of fields outside
// `fmask` are marked finished at the start.  Iterations are launched in
// batches sized from the previous solve of the same kind, with a poll of the
// per-system scalars between batches.  In a solve of all fields, once every
// system but the oxygen ones has converged (the drugs often need only a few
// iterations), the remaining iterations run on the oxygen prefix's tables
// (sys1, mg1: the same arrays, fewer workgroups) and its captured graph.
// defer_finish (a solve of every field that the ODE phase follows): when every
// system converged, the last iteration's x += alpha p is left to the ODE
// kernel (c->fin_pending), which reads every voxel of the fields anyway.
// prep_o2_only: the other fields' multigrid data are current (c->fixed_ops);
// only the oxygen systems' are rebuilt from this step's c.
hca_status solve(Ctx* c, const Work& W_all, const MgBufs& mg_all, unsigned fmask, double rtol,
                 int maxit, int kind, bool defer_finish = false, bool prep_o2_only = false) {
  const int nsys = W_all.nreps;
  const Work* Wp = &W_all;
  const MgBufs* mgp = &mg_all;
  int gk = kind;   // graph of the active tables
  const Work& W = W_all;
  const MgBufs& mg = mg_all;
  if (c->use_mg) {
    const double nf = c->dp.nf;   // oxygen alone: 1/nf of the priced voxels
    ProfScope ps(c, KC_MG_PREP, kTagAll, false, prep_o2_only ? -bpv_of(c, KC_MG_PREP) * (nf - 1.0) / nf : 0.0);
    launch_mg_prepare(c->stream, prep_o2_only ? c->sys1 : W, prep_o2_only ? c->mg1 : mg, c->c);
  }
  {
    ProfScope ps(c, KC_CG_START, kTagAll);
    launch_cg_start(c->stream, W, rtol, maxit, c->c, c->b, c->F, c->sb, fmask, c->nreps);
  }
  if (c->use_mg) run_vcycle(c, W, mg, 0);   // z of the start residual
  int launched = 0;
  int batch = std::max(1, c->last_it[kind] + g_solve_lead);
  int real = 0;
  auto iteration = [&](int it) {
    {
      // a solve's first apply has no earlier x += alpha p to make
      ProfScope ps(c, KC_CG_APPLY, it, true, it == 0 ? -kBytesApplyX : 0.0);
      launch_cg_apply(c->stream, *Wp, c->c, c->F, c->sb, it & 1);
    }
    {
      ProfScope ps(c, KC_CG_UPDATE, it);
      launch_cg_update(c->stream, *Wp, rtol, maxit, c->sb);
    }
    // z = M r for the next direction (work only where this iteration did not converge)
    if (c->use_mg) run_vcycle(c, *Wp, *mgp, it + 1);
  };
  // Replays of a captured pair of iterations (even, odd) when no kernel is
  // being timed; finished systems make the extra launches no-ops.
  bool graphs = c->prm.graphs && c->prm.profile == 0 && !c->graph_failed &&
                (c->iter_graph[kind] || capture_iterations(c, W, mg, rtol, maxit, kind));
  for (;;) {
    batch = std::min(batch, maxit - launched);
    int k = 0;
    if (graphs) {
      if ((launched & 1) && k < batch) {
        iteration(launched);
        ++k;
        ++launched;
      }
      for (; k + 2 <= batch; k += 2, launched += 2)
        HIPCHK(c, hipGraphLaunch(c->iter_graph[gk], c->stream));
    }
    for (; k < batch; ++k, ++launched) iteration(launched);
    HIPCHK(c, hipMemcpyAsync(c->h_ss, c->sb.ss, sizeof(SolveScal) * nsys, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    bool all = true;
    real = 0;
    for (int s = 0; s < nsys; ++s) {
      all = all && c->h_ss[s].done;
      real = std::max(real, c->h_ss[s].it);
    }
    if (all || launched >= maxit) break;
    batch = 2;
    if (kind == 0 && Wp != &c->sys1 && nsys > c->nreps) {
      bool rest = true;
      for (int s = c->nreps; s < nsys; ++s) rest = rest && c->h_ss[s].done;
      if (rest) {
        Wp = &c->sys1;
        mgp = &c->mg1;
        gk = 1;
        graphs = graphs && (c->iter_graph[1] || capture_iterations(c, c->sys1, c->mg1, rtol, maxit, 1));
      }
    }
  }
  bool allconv = true;
  for (int s = 0; s < nsys; ++s) allconv = allconv && c->h_ss[s].conv;
  if (defer_finish && allconv) {
    c->fin_pending = true;
  } else {   // the last iteration's x += alpha p (systems that iterated)
    ProfScope ps(c, KC_CG_FINISH, 0);
    launch_cg_finish(c->stream, W_all, c->F, c->sb);
  }
  prof_flush(c, c->h_ss, nsys);
  c->last_it[kind] = real;
  if (kind == 0) c->last_ss.assign(c->h_ss, c->h_ss + nsys);
  for (int s = 0; s < nsys; ++s)
    if (!c->h_ss[s].conv) {
      char buf[160];
      snprintf(buf, sizeof buf, "field %d replicate %d: CG stopped at %d iterations, rel. res %.3e",
               s / c->nreps, s % c->nreps, c->h_ss[s].it,
               c->h_ss[s].bb > 0 ? std::sqrt(c->h_ss[s].rr / c->h_ss[s].bb) : 0.0);
      return fail(c, HCA_E_NOCONV, buf);
    }
  return HCA_OK;
}

// The deferred solve end for the ODE phase (null: none) and its bytes per
// voxel (x, p read and x written for each system that iterated).
const CgFinish<Real>* take_finish(Ctx* c, double& bpv) {
  bpv = 0.0;
  if (!c->fin_pending) return nullptr;
  c->fin_pending = false;
  double vox = 0.0;
  for (int s = 0; s < c->dp.nf * c->nreps; ++s)
    if (c->h_ss[s].it > 0) vox += (double)c->sys_n[s];
  bpv = kBytesPerVoxel[KC_CG_FINISH] * vox / (double)c->ntot;
  return c->d_fin;
}

// The solves' stopping tolerance: cg_rtol, and no less than FP32 storage can
// attain in precision 32.
inline double solve_rtol(const Ctx* c) { return std::max(c->prm.cg_rtol, kRtolFloor); }

hca_status run_phases(Ctx* c, unsigned mask) {
  const Work& wk = c->work;
  hipStream_t s = c->stream;
  const unsigned drugs = c->dp.drug3 ? 14u : 6u;   // fields 1, 2 (and 3)
  const unsigned fmask = ((mask & HCA_PH_O2) ? 1u : 0u) | ((mask & HCA_PH_DRUGS) ? drugs : 0u) |
                         (((mask & HCA_PH_VEGF) && c->dp.vegf) ? (1u << c->dp.fV) : 0u);
  // the field solves: pde_substeps theta-scheme substeps (one by default)
  for (int j = 0; fmask && j < c->dp.nsub_pde; ++j) {
    {
      ProfScope ps(c, KC_PLASMA, kTagState);
      launch_plasma(s, wk, c->dp, c->d_step, j, c->dose_t, c->dose_a, c->g0);
    }
    // the initial guess in the setup pass where nothing reads F after it
    // (extrapolations), or fitted to this solve's system after the setup
    // (x0_extrapolate 3: the fields but oxygen fitted after the setup, from
    // this solve's system; oxygen, whose operator follows the cells, keeps the
    // geometric extrapolation)
    const unsigned fitmask = (c->Fprev && c->prm.x0_extrapolate == 3) ? (fmask & ~1u) : 0u;
    const unsigned xmask = fmask & ~fitmask;
    const bool guess_in_setup = c->Fprev && c->dp.theta >= 1.0;
    // the fields but oxygen keep their c and multigrid data while the vessel
    // map is unchanged (2 or 3 stored values per voxel fewer in the setup)
    const bool keep = c->fixed_ops && !c->dp.vegf;
    // with every field solved and every guess formed here, the history
    // rotates: this solve's starting values go to Fprev2's buffer (whose
    // values are read for the last time), then Fprev and Fprev2 swap roles
    const bool rotate = fitmask && guess_in_setup && fmask == (1u << c->dp.nf) - 1u;
    {
      ProfScope ps(c, KC_SETUP, kTagState, true, keep ? -(2.0 + c->dp.drug3) * kE : 0.0);
      launch_setup_step(s, wk, c->dp, c->ntot, c->L, c->w, c->F, c->Vc, c->g0, c->c, c->b,
                        guess_in_setup ? c->Fprev : nullptr, rotate ? c->Fprev2 : c->Fprev, xmask,
                        c->prm.x0_extrapolate, keep ? 1 : 0);
      if (c->dp.theta < 1.0) launch_rhs_lap(s, wk, c->dp, c->ntot, c->F, c->b);
    }
    if (c->Fprev && !guess_in_setup && xmask) {
      ProfScope ps(c, KC_SETUP, kTagState);
      launch_extrapolate(s, wk, c->ntot, c->dp.nf, xmask, c->prm.x0_extrapolate, c->F, c->Fprev);
    }
    if (fitmask) {   // priced per voxel of each fitted field (three launches; one stored value less rotating)
      const double per_field = kBytesPerVoxel[KC_GUESS] - (rotate ? kE : 0.0);
      ProfScope ps(c, KC_GUESS, kTagState, false,
                   __builtin_popcount(fitmask) * per_field - kBytesPerVoxel[KC_GUESS]);
      launch_guess_projection(s, c->sys_all, c->c, c->b, c->F, c->Fprev, c->Fprev2, c->d_gpart, c->d_galpha,
                              fitmask, c->nreps, rotate ? 1 : 0);
    }
    if (rotate) std::swap(c->Fprev, c->Fprev2);
    const bool newton = c->prm.o2_newton > 0 && (fmask & 1u);
    if (newton)
      HIPCHK(c, hipMemcpyAsync(c->b_o2lin, c->b, sizeof(Real) * (size_t)c->ntot, hipMemcpyDeviceToDevice, s));
    // the last substep's solve ends in the ODE phase when one follows
    const bool defer = (mask & HCA_PH_ODE) && j + 1 == c->dp.nsub_pde && !newton;
    hca_status st = solve(c, c->sys_all, c->mg_all, fmask, solve_rtol(c), c->prm.cg_maxit, 0, defer,
                          keep);
    if (st != HCA_OK) return st;
    c->fixed_ops = !c->dp.vegf;
    // Newton steps on the oxygen uptake at the new value, from the linearised solution
    for (int k = 0; newton && k < c->prm.o2_newton; ++k) {
      {
        ProfScope ps(c, KC_SETUP, kTagState);
        launch_setup_o2_newton(s, wk, c->dp, c->L, c->w, c->K, c->b_o2lin, c->c, c->b);
      }
      st = solve(c, c->sys1, c->mg1, 1u, solve_rtol(c), c->prm.cg_maxit, 1);
      if (st != HCA_OK) return st;
    }
  }
  if (mask & HCA_PH_ODE) {
    double fin_bpv;
    const CgFinish<Real>* fin = take_finish(c, fin_bpv);
    if (c->sur_on) {
      ProfScope ps(c, KC_MLP_APPLY, kTagState, true, fin_bpv);
      launch_mlp_apply(s, wk, c->dp, c->net, c->L, c->K, c->G1, c->G2, c->P, c->Vc, c->phi,
                       c->d_cpart, c->d_cnt, c->ca_list, fin);
    } else {
      ProfScope ps(c, KC_ODE, kTagState, true, fin_bpv);
      launch_ode(s, wk, c->dp, c->L, c->K, c->P, c->Vc, c->phi, fin);
    }
  }
  if (mask & HCA_PH_CA) {
    {
      ProfScope ps(c, KC_CA_PROPOSE, kTagState, false);
      launch_ca_propose(s, wk, c->dp, c->d_step, c->L, c->w, c->K, c->G1, c->G2, c->G3, c->phi,
                        c->code, c->win, c->ca_list);
    }
    {
      ProfScope ps(c, KC_CA_RESOLVE, kTagState);
      launch_ca_resolve(s, wk, c->phi, c->code, c->win, c->ca_list);
    }
    {
      ProfScope ps(c, KC_CA_FINALIZE, kTagState);
      launch_ca_finalize(s, wk, c->L, c->phi, c->P, c->Vc, c->code, c->win, c->d_cpart, c->d_cnt);
    }
    if (c->dp.vegf) {
      ProfScope ps(c, KC_VESSEL, kTagState);
      launch_vessel(s, wk, c->dp, c->d_step, c->L, c->V, c->w, c->d_cpart, c->d_cnt);
    }
  }
  if (mask & HCA_PH_STATS) {
    ProfScope ps(c, KC_STATS, kTagState);
    launch_stats(s, wk, c->L, c->w, c->F, c->dp.nf, c->ntot, c->P, c->Vc, c->phi, c->d_cpart, c->d_cnt);
  }
  if (mask & HCA_PH_ADVANCE) {
    launch_advance(s, c->d_step);
    c->step += 1;
  }
  HIPCHK(c, hipGetLastError());
  return HCA_OK;
}

hca_status check_after(Ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->h_cnt, c->d_cnt, sizeof(Counters) * c->nreps, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_flush(c, nullptr, 0);
  for (int r = 0; r < c->nreps; ++r)
    if (c->h_cnt[r].nonfinite) {
      char buf[96];
      snprintf(buf, sizeof buf, "replicate %d: %llu non-finite field values", r,
               (unsigned long long)c->h_cnt[r].nonfinite);
      return fail(c, HCA_E_NONFINITE, buf);
    }
  return HCA_OK;
}

// ---- validation ----------------------------------------------------------------

hca_status validate_reps(const hca_replicate* reps, int n, std::string& msg, int& singular) {
  singular = -1;
  for (int r = 0; r < n; ++r) {
    const hca_replicate& R = reps[r];
    char buf[160];
    if (R.nx < 1 || R.ny < 1 || R.nz < 1 || R.nx > 32767 || R.ny > 32767 || R.nz > 32767) {
      snprintf(buf, sizeof buf, "replicate %d: lattice %dx%dx%d out of range", r, R.nx, R.ny, R.nz);
      msg = buf;
      return HCA_E_INVALID;
    }
    if (!R.cell || !R.vessel_w) {
      snprintf(buf, sizeof buf, "replicate %d: null cell or vessel map", r);
      msg = buf;
      return HCA_E_INVALID;
    }
    const long long nv = (long long)R.nx * R.ny * R.nz;
    long long nves = 0;
    for (long long i = 0; i < nv; ++i) {
      const double wv = R.vessel_w[i];
      const uint8_t l = R.cell[i];
      if (!(std::isfinite(wv) && wv >= 0.0) || l > 2 || (l != 0 && wv != 0.0)) {
        snprintf(buf, sizeof buf,
                 "replicate %d voxel %lld: cell %d, w %g (codes 0..2, finite w >= 0, no cell "
                 "on a vessel)",
                 r, i, (int)l, wv);
        msg = buf;
        return HCA_E_INVALID;
      }
      nves += wv > 0.0;
    }
    if (nves == 0 && singular < 0) singular = r;
    for (int d = 0; d < 3; ++d) {
      const int nd = d < 2 ? R.n_doses[d] : R.n_doses3;
      const double* ts = d < 2 ? R.dose_t_min[d] : R.dose_t_min3;
      const double* as = d < 2 ? R.dose_amt[d] : R.dose_amt3;
      if (nd < 0 || nd > HCA_MAX_DOSES || (nd > 0 && (!ts || !as))) {
        snprintf(buf, sizeof buf, "replicate %d drug %d: bad dose list", r, d);
        msg = buf;
        return HCA_E_INVALID;
      }
      for (int k = 0; k < nd; ++k) {
        if (!std::isfinite(ts[k]) || !std::isfinite(as[k]) || ts[k] < 0.0 || as[k] < 0.0 ||
            (k > 0 && ts[k] < ts[k - 1])) {
          snprintf(buf, sizeof buf, "replicate %d drug %d: dose %d not finite, negative or unsorted",
                   r, d, k);
          msg = buf;
          return HCA_E_INVALID;
        }
      }
    }
  }
  return HCA_OK;
}

hca_status validate_params(const hca_params* p, std::string& msg) {
  if (p->precision != kPrecision) {
    msg = "precision must be 64 or 32";
    return HCA_E_INVALID;
  }
  const double pos[] = {p->h_um, p->dt_min, p->D_K, p->D_G, p->K1, p->G_ref[0], p->G_ref[1],
                        p->K_p53, p->J5, p->K_V, p->K_phi, p->T_cycle, p->cg_rtol, p->init_rtol};
  for (double v : pos)
    if (!(std::isfinite(v) && v > 0.0)) {
      msg = "parameter must be finite and > 0";
      return HCA_E_INVALID;
    }
  const double nonneg[] = {p->r_k, p->K0, p->phi_K, p->psi_G, p->kappa_G, p->k_pk[0], p->k_pk[1],
                           p->k1, p->k1p, p->k2, p->k2p};
  for (double v : nonneg)
    if (!(std::isfinite(v) && v >= 0.0)) {
      msg = "parameter must be finite and >= 0";
      return HCA_E_INVALID;
    }
  if (!std::isfinite(p->k2pp) || p->b_int[0] < 1 || p->b_int[1] < 1 || p->b_int[0] > 64 ||
      p->b_int[1] > 64 || p->ode_substeps < 1 || p->cg_maxit < 1 || p->init_maxit < 1 ||
      (p->precond != 0 && p->precond != 1) || p->mg_coarse_max < 1 || p->profile < 0 ||
      p->profile > KC_COUNT + 1 || (p->graphs != 0 && p->graphs != 1) ||
      (p->autotune != 0 && p->autotune != 1) || (p->mg_fuse != 0 && p->mg_fuse != 1)) {
    msg = "integer parameter out of range";
    return HCA_E_INVALID;
  }
  if (p->pde_substeps < 1 || p->pde_substeps > 1000 || !(p->pde_theta >= 0.5 && p->pde_theta <= 1.0) ||
      p->o2_newton < 0 || p->o2_newton > 20) {
    msg = "pde_substeps in [1, 1000], pde_theta in [0.5, 1] and o2_newton in [0, 20] required";
    return HCA_E_INVALID;
  }
  if ((p->pk_mm != 0 && p->pk_mm != 1) || !(std::isfinite(p->mm_vmax) && p->mm_vmax >= 0.0) ||
      !(std::isfinite(p->mm_km) && p->mm_km > 0.0)) {
    msg = "pk_mm in {0, 1}, finite mm_vmax >= 0 and mm_km > 0 required";
    return HCA_E_INVALID;
  }
  {
    const double ratio = p->dv_min / p->dt_min;
    const bool whole = std::isfinite(ratio) && ratio >= 1.0 && ratio <= 1e9 &&
                       std::fabs(ratio - std::round(ratio)) <= 1e-9 * ratio;
    const bool fin = std::isfinite(p->D_V) && std::isfinite(p->psi_V) && std::isfinite(p->sec_V) &&
                     std::isfinite(p->V_low) && std::isfinite(p->V_high) &&
                     std::isfinite(p->birth_per_V) && std::isfinite(p->w_new);
    if ((p->vegf != 0 && p->vegf != 1) || !fin || !(p->D_V > 0.0) || !(p->psi_V >= 0.0) ||
        !(p->sec_V >= 0.0) || !whole || !(p->V_low >= 0.0) || !(p->V_high >= p->V_low) ||
        !(p->p_death >= 0.0 && p->p_death <= 1.0) || !(p->birth_per_V >= 0.0) ||
        !(p->birth_per_V * p->V_high <= 1.0) || !(p->w_new > 0.0)) {
      msg = "vegf in {0, 1}; D_V > 0, psi_V >= 0, sec_V >= 0; dv_min a whole multiple of dt_min; "
            "0 <= V_low <= V_high; p_death in [0, 1]; 0 <= birth_per_V <= 1 / V_high; w_new > 0";
      return HCA_E_INVALID;
    }
  }
  {
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    auto nonneg = [](double v) { return std::isfinite(v) && v >= 0.0; };
    if ((p->drug3 != 0 && p->drug3 != 1) || !pos(p->epi_w1) || !pos(p->epi_w2) || !pos(p->epi_w3) ||
        !nonneg(p->epi_q2) || !nonneg(p->epi_q3) || !nonneg(p->epi_cl) || !pos(p->G_ref3) ||
        p->b_int3 < 1 || p->b_int3 > 64) {
      msg = "drug3 in {0, 1}; epi_w* > 0; epi_q2, epi_q3, epi_cl >= 0; G_ref3 > 0; b_int3 in 1..64";
      return HCA_E_INVALID;
    }
  }
  if (p->x0_extrapolate < 0 || p->x0_extrapolate > 3) {
    msg = "x0_extrapolate in {0, 1, 2, 3}";
    return HCA_E_INVALID;
  }
  if (p->mg_smooth != 2) {
    msg = "mg_smooth: the multigrid smoothers implement two sweeps before and after";
    return HCA_E_INVALID;
  }
  return HCA_OK;
}

// ---- work tables -------------------------------------------------------------

// z-extent of a column tile: about `target` tiles per lattice (enough to fill
// the chip for a lone lattice), at most 16 planes per tile.
// Tile depth tz made even (at least 2) unless one chunk covers the lattice.
int even_depth(int tz, int nz) {
  if (tz >= nz) return nz;
  return std::max(2, tz & ~1);
}

// Depth of level 0's fused-smoothing tiles: each tile recomputes three planes
// below and above its own, so deeper tiles (up to 64 planes) while a system
// still has about g_fused_target of them (HCA_FUSED_TARGET), and at least
// g_fused_min planes (HCA_FUSED_MIN).  Measured (same GPU, two passes): the
// 128^3 workload 2.319 ms per step at depth 8, 2.34 at 12, 2.26 at 16, 2.36
// at 20; the 64-replicate ensemble within 0.2 % for depths 8 to 64; the
// 4 x 384^3 lattices take 64.
double g_fused_target = 256.0;
int g_fused_min = 16;
// Coarser levels smooth in fused passes from this many cells over all systems
// (HCA_FUSE_MIN_CELLS).  Measured per V-cycle segment: one 384^3 lattice's
// levels >= 1 take 214 us unfused, 184 us with level 1 (21 M cells) fused,
// 178 us with level 2 (2.7 M) too; the 128^3 lattice's level 1 (0.8 M) runs
// at 25 us unfused and 33 us fused.
long long g_fuse_min_cells = 2LL << 20;
int fused_depth(int nx, int ny, int nz, int tx) {
  const int ty = kF3Block / tx;
  const double nxy = (double)((nx + tx - 1) / tx) * (double)((ny + ty - 1) / ty);
  const int tz = (int)std::floor(nz * nxy / g_fused_target);
  return even_depth(std::max(g_fused_min, std::min(64, tz)), nz);
}

int pick_tz(int nx, int ny, int nz, int tx, double target) {
  const int ty = kBlock / tx;
  const double nxy = (double)((nx + tx - 1) / tx) * (double)((ny + ty - 1) / ty);
  const int tz = (int)std::floor(nz * nxy / std::max(1.0, target));
  return std::max(1, std::min(16, tz));
}

void add_tiles(std::vector<Tile>& v, int rep, int nx, int ny, int nz, int tx, int tz, int ty = 0) {
  if (ty == 0) ty = kBlock / tx;
  for (int z0 = 0; z0 < nz; z0 += tz)
    for (int y0 = 0; y0 < ny; y0 += ty)
      for (int x0 = 0; x0 < nx; x0 += tx) {
        Tile t{};
        t.rep = rep;
        t.x0 = (short)x0;
        t.y0 = (short)y0;
        t.z0 = (short)z0;
        t.z1 = (short)std::min(nz, z0 + tz);
        v.push_back(t);
      }
}

// Stencil tiles are g_tile_depth planes deep (at most nz; tuning knob
// HCA_TILE_DEPTH, 0 = instead aim at HCA_TILE_TARGET tiles per lattice).
// Deep tiles keep the z-halo re-reads of the plane-marching stencils small;
// batches and large lattices supply the parallelism.
double g_tile_target = 1024.0;
int g_tile_depth = 16;
// Tiles per system the coarser multigrid levels aim at (HCA_MG_TILE_TARGET).
double g_mg_tile_target = 512.0;

template <typename T>
hca_status upload(Ctx* c, T** p, const std::vector<T>& v) {
  HIPCHK(c, dalloc(p, v.size()));
  if (!v.empty()) HIPCHK(c, hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return HCA_OK;
}

// Table entry of one lattice (a replicate, or one field's system of it).
// Tile shape and flat blocking come from the lattice's own size only, so a
// lattice's arithmetic and rounding are the same alone or in a batch.
RepDev lattice_entry(const RepHost& R, long long off, int idx, std::vector<FlatBlk>& flat,
                     std::vector<Tile>& tiles) {
  RepDev d;
  memset(&d, 0, sizeof d);
  d.nx = R.nx;
  d.ny = R.ny;
  d.nz = R.nz;
  d.off = off;
  d.n = R.n;
  d.seed = R.seed;
  const long long chunks = (R.n + kFlatChunk - 1) / kFlatChunk;
  d.flat_nb = (int)std::min<long long>(chunks, kMaxFlatBlocksPerRep);
  d.flat_b0 = (int)flat.size();
  for (int k = 0; k < d.flat_nb; ++k) {
    FlatBlk fb{};
    fb.rep = idx;
    fb.begin = R.n * k / d.flat_nb;
    fb.end = R.n * (k + 1) / d.flat_nb;
    flat.push_back(fb);
  }
  d.tx = R.tx;
  d.tile_b0 = (int)tiles.size();
  add_tiles(tiles, idx, R.nx, R.ny, R.nz, R.tx, R.tz);
  d.tile_nb = (int)tiles.size() - d.tile_b0;
  return d;
}

// ---- tile autotuner ---------------------------------------------------------------

// Stencil tile shape of every lattice: tx from nx (pick_tx), g_tile_depth
// planes deep; with params.autotune, the depth (2 ... 32 planes) and the width
// policy (pick_tx, or 16 x 16) are instead the fastest of 10 candidates, timed on the CG apply kernel (the dominant
// stencil) over the whole batch at once on scratch arrays of the batch's
// shape (one warm-up launch, then the best of three), so the choice accounts
// for the parallelism the batch already has.  Tiles fix the order of the
// dot-product partial sums, so a tuned context agrees with an untuned one to
// rounding, not bit for bit.
hca_status plan_tiles(Ctx* c) {
  // width policy 0: pick_tx; 1: 16 x 16 everywhere.  Depths are even (or the
  // whole lattice), as the restriction needs even tile origins.
  auto apply_plan = [&](int depth, int policy) {
    for (RepHost& R : c->reps) {
      R.tx = policy == 1 ? 16 : pick_tx(R.nx);
      R.tz = even_depth(depth > 0 ? depth : pick_tz(R.nx, R.ny, R.nz, R.tx, g_tile_target), R.nz);
    }
  };
  apply_plan(g_tile_depth, 0);
  if (!c->prm.autotune) return HCA_OK;
  const long long n = c->ntot;
  std::vector<void*> mem;
  auto scratch = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 8)) != hipSuccess) return nullptr;
    mem.push_back(p);
    return p;
  };
  auto release = [&]() {
    for (void* p : mem) (void)hipFree(p);
    mem.clear();
  };
  const int R = c->nreps;
  size_t maxtiles = 1;   // most tiles any candidate can make (tz >= 1)
  for (int tx : {16, 32, 64}) {
    size_t t = 0;
    for (const RepHost& H : c->reps)
      t += (size_t)((H.nx + tx - 1) / tx) * (size_t)((H.ny + kBlock / tx - 1) / (kBlock / tx)) * H.nz;
    maxtiles = std::max(maxtiles, t);
  }
  Real* cb = (Real*)scratch(sizeof(Real) * n);
  Real* tx = (Real*)scratch(sizeof(Real) * n);   // the apply's x (a zero alpha leaves it as it is)
  SolverBufs tsb{};
  tsb.z32 = (float*)scratch(4 * n);   // multigrid layout (jacobi = 0)
  tsb.p0 = (Real*)scratch(sizeof(Real) * n);
  tsb.p1 = (Real*)scratch(sizeof(Real) * n);
  tsb.q = (Real*)scratch(sizeof(Real) * n);
  tsb.partial = (double*)scratch(3 * 8 * maxtiles);
  tsb.ss = (SolveScal*)scratch(sizeof(SolveScal) * R);
  RepDev* drep = (RepDev*)scratch(sizeof(RepDev) * R);
  Tile* dtiles = (Tile*)scratch(sizeof(Tile) * maxtiles);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!cb || !tx || !tsb.z32 || !tsb.p0 || !tsb.p1 || !tsb.q || !tsb.partial || !tsb.ss || !drep || !dtiles ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    release();
    if (e0) (void)hipEventDestroy(e0);
    return fail(c, HCA_E_NOMEM, "autotune: scratch allocation failed");
  }
  hca_status st = HCA_OK;
  auto check = [&](hipError_t e) {
    if (e != hipSuccess && st == HCA_OK)
      st = fail(c, HCA_E_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
  };
  for (void* p : {(void*)cb, (void*)tx, (void*)tsb.p0, (void*)tsb.p1})
    check(hipMemsetAsync(p, 0, sizeof(Real) * n, c->stream));
  check(hipMemsetAsync(tsb.z32, 0, 4 * n, c->stream));
  check(hipMemsetAsync(tsb.ss, 0, sizeof(SolveScal) * R, c->stream));
  float tbest = 1e30f;
  int best_depth = g_tile_depth;
  int best_policy = 0;
  for (int policy = 0; policy < 2 && st == HCA_OK; ++policy)
    for (int depth : {2, 4, 8, 16, 32}) {
      apply_plan(depth, policy);
      std::vector<RepDev> rd;
      std::vector<Tile> tiles;
      for (int r = 0; r < R; ++r) {
        const RepHost& H = c->reps[r];
        RepDev d;
        memset(&d, 0, sizeof d);
        d.nx = H.nx;
        d.ny = H.ny;
        d.nz = H.nz;
        d.off = H.off;
        d.n = H.n;
        d.tx = H.tx;
        d.tile_b0 = (int)tiles.size();
        add_tiles(tiles, r, H.nx, H.ny, H.nz, H.tx, H.tz);
        d.tile_nb = (int)tiles.size() - d.tile_b0;
        d.a = c->dp.aG;
        rd.push_back(d);
      }
      check(hipMemcpyAsync(drep, rd.data(), sizeof(RepDev) * R, hipMemcpyHostToDevice, c->stream));
      check(hipMemcpyAsync(dtiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice,
                           c->stream));
      Work w{};
      w.nreps = R;
      w.reps = drep;
      w.tiles = dtiles;
      w.ntiles = (int)tiles.size();
      w.max_blocks = c->work.max_blocks;
      launch_cg_apply_kernel(c->stream, w, cb, tx, tsb, 0);
      float tmin = 1e30f;
      for (int k = 0; k < 3; ++k) {
        check(hipEventRecord(e0, c->stream));
        launch_cg_apply_kernel(c->stream, w, cb, tx, tsb, 0);
        check(hipEventRecord(e1, c->stream));
        check(hipEventSynchronize(e1));
        float ms = 0.f;
        check(hipEventElapsedTime(&ms, e0, e1));
        tmin = std::min(tmin, ms);
      }
      check(hipGetLastError());
      if (tmin < tbest) {
        tbest = tmin;
        best_depth = depth;
        best_policy = policy;
      }
    }
  check(hipStreamSynchronize(c->stream));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  release();
  if (st != HCA_OK) return st;
  apply_plan(best_depth, best_policy);
  return HCA_OK;
}

hca_status build_tables(Ctx* c, const hca_replicate* in) {
  const int R = c->nreps;
  // work-item kernels: one item per workgroup unless HCA_MAX_BLOCKS caps the
  // grid (then each workgroup loops over a contiguous run of items)
  int max_blocks = 1 << 30;
  if (const char* e = getenv("HCA_MAX_BLOCKS")) {
    const int v = atoi(e);
    if (v > 0) max_blocks = v;
  }
  if (const char* e = getenv("HCA_XCD_REMAP")) g_xcd_remap = atoi(e) != 0;
  if (const char* e = getenv("HCA_TILE_REMAP")) g_tile_remap = atoi(e) != 0;
  if (const char* e = getenv("HCA_TILE_DEPTH")) g_tile_depth = std::max(0, atoi(e));
  if (const char* e = getenv("HCA_SOLVE_LEAD")) g_solve_lead = std::max(-8, std::min(8, atoi(e)));
  if (const char* e = getenv("HCA_FUSED_TARGET")) {
    const double v = atof(e);
    if (v >= 1.0) g_fused_target = v;
  }
  if (const char* e = getenv("HCA_FUSED_MIN")) g_fused_min = std::max(2, std::min(64, atoi(e)));
  {
    const char* e = getenv("HCA_FUSE_MIN_CELLS");
    g_fuse_min_cells = e ? std::max(1LL, atoll(e)) : (2LL << 20);
  }
  if (const char* e = getenv("HCA_MG_TILE_TARGET")) {
    const double v = atof(e);
    if (v >= 1.0) g_mg_tile_target = v;
  }
  if (const char* e = getenv("HCA_TILE_TARGET")) {
    const double v = atof(e);
    if (v >= 1.0) g_tile_target = v;
  }
  c->work.max_blocks = max_blocks;
  {
    hca_status st = plan_tiles(c);
    if (st != HCA_OK) return st;
  }
  {
    std::vector<RepDev> rd;
    std::vector<FlatBlk> flat;
    std::vector<Tile> tiles;
    for (int r = 0; r < R; ++r) {
      RepDev d = lattice_entry(c->reps[r], c->reps[r].off, r, flat, tiles);
      d.dose_off = r * 3 * HCA_MAX_DOSES;
      d.ndose[0] = in[r].n_doses[0];
      d.ndose[1] = in[r].n_doses[1];
      d.ndose[2] = in[r].n_doses3;
      rd.push_back(d);
    }
    hca_status st;
    if ((st = upload(c, &c->d_reps, rd)) != HCA_OK || (st = upload(c, &c->d_flat, flat)) != HCA_OK ||
        (st = upload(c, &c->d_tiles, tiles)) != HCA_OK)
      return st;
    c->work.nreps = R;
    c->work.reps = c->d_reps;
    c->work.flat = c->d_flat;
    c->work.nflat = (int)flat.size();
    c->work.tiles = c->d_tiles;
    c->work.ntiles = (int)tiles.size();
    c->work.max_blocks = max_blocks;
  }
  {
    std::vector<RepDev> sd;
    std::vector<FlatBlk> flat;
    std::vector<Tile> tiles, ftiles;
    int nflat1 = 0, ntiles1 = 0, nftiles1 = 0;
    c->sys_n.clear();
    for (int f = 0; f < c->dp.nf; ++f) {
      for (int r = 0; r < R; ++r) {
        RepDev d = lattice_entry(c->reps[r], (long long)f * c->ntot + c->reps[r].off, f * R + r,
                                 flat, tiles);
        const RepHost& H = c->reps[r];
        d.ftile_b0 = (int)ftiles.size();
        add_tiles(ftiles, f * R + r, H.nx, H.ny, H.nz, H.tx, fused_depth(H.nx, H.ny, H.nz, H.tx),
                  kF3Block / H.tx);
        d.ftile_nb = (int)ftiles.size() - d.ftile_b0;
        const int ftx = (H.nx + H.tx - 1) / H.tx;   // tiles per row
        c->fchunk = std::max(c->fchunk, std::min(8 * ftx, 256));
        // the theta scheme's implicit coupling
        d.a = (f == 0 ? c->dp.aK : (c->dp.vegf && f == c->dp.fV) ? c->dp.aV : c->dp.aG) * c->dp.theta;
        sd.push_back(d);
        c->sys_n.push_back(c->reps[r].n);
      }
      if (f == 0) {
        nflat1 = (int)flat.size();
        ntiles1 = (int)tiles.size();
        nftiles1 = (int)ftiles.size();
      }
    }
    hca_status st;
    if ((st = upload(c, &c->d_sys, sd)) != HCA_OK || (st = upload(c, &c->d_sflat, flat)) != HCA_OK ||
        (st = upload(c, &c->d_stiles, tiles)) != HCA_OK || (st = upload(c, &c->d_ftiles, ftiles)) != HCA_OK)
      return st;
    c->nftiles_all = (int)ftiles.size();
    c->nftiles1 = nftiles1;
    c->sys_all.nreps = c->dp.nf * R;
    c->sys_all.reps = c->d_sys;
    c->sys_all.flat = c->d_sflat;
    c->sys_all.nflat = (int)flat.size();
    c->sys_all.tiles = c->d_stiles;
    c->sys_all.ntiles = (int)tiles.size();
    c->sys_all.max_blocks = max_blocks;
    c->sys1 = c->sys_all;
    c->sys1.nreps = R;
    c->sys1.nflat = nflat1;
    c->sys1.ntiles = ntiles1;
  }
  return HCA_OK;
}

hca_status alloc_all(Ctx* c) {
  const size_t n = (size_t)c->ntot;
  const size_t n3 = (size_t)c->dp.nf * n;   // solver arrays: nf fields
  const int nsys = c->dp.nf * c->nreps;
  auto big = [&](auto** p, size_t count) -> hca_status {
    hipError_t e = dalloc(p, count);
    if (e == hipErrorOutOfMemory) return fail(c, HCA_E_NOMEM, "device memory exhausted");
    HIPCHK(c, e);
    return HCA_OK;
  };
  HIPCHK(c, dalloc(&c->L, n));
  HIPCHK(c, dalloc(&c->code, n));
  HIPCHK(c, dalloc(&c->win, n));
  HIPCHK(c, dalloc(&c->ca_list.cells, n));
  HIPCHK(c, dalloc(&c->ca_list.item_n, (size_t)c->work.nflat));
  hca_status st;
  double** f1[] = {&c->w, &c->P, &c->Vc, &c->phi};
  for (double** p : f1)
    if ((st = big(p, n)) != HCA_OK) return st;
  Real** f3[] = {&c->F, &c->c, &c->b, &c->sb.r, &c->sb.p0, &c->sb.p1, &c->sb.q};
  for (Real** p : f3)
    if ((st = big(p, n3)) != HCA_OK) return st;
  if (c->use_mg) {
    for (float** p : {&c->sb.z32, &c->sb.r32}) {
      hipError_t e = dalloc(p, n3);
      if (e == hipErrorOutOfMemory) return fail(c, HCA_E_NOMEM, "device memory exhausted");
      HIPCHK(c, e);
    }
  } else if ((st = big(&c->sb.z, n3)) != HCA_OK) {
    return st;
  }
  // every state and solver array starts at 0 (a state is imported replicate
  // by replicate; the solver reads the whole nf x ntot arrays)
  for (void* p : {(void*)c->w, (void*)c->P, (void*)c->Vc, (void*)c->phi})
    HIPCHK(c, hipMemset(p, 0, sizeof(double) * n));
  for (void* p : {(void*)c->F, (void*)c->c, (void*)c->b, (void*)c->sb.r, (void*)c->sb.p0, (void*)c->sb.p1,
                  (void*)c->sb.q})
    HIPCHK(c, hipMemset(p, 0, sizeof(Real) * n3));
  HIPCHK(c, hipMemset(c->L, 0, n));
  c->K = c->F;
  c->G1 = c->F + n;
  c->G2 = c->F + 2 * n;
  c->G3 = c->dp.drug3 ? c->F + 3 * n : nullptr;
  c->V = c->dp.vegf ? c->F + (size_t)c->dp.fV * n : nullptr;
  c->sb.jacobi = c->use_mg ? 0 : 1;
  if (!c->use_mg && (st = big(&c->sb.dinv, n3)) != HCA_OK) return st;
  const size_t nwork = (size_t)std::max({c->sys_all.ntiles, c->sys_all.nflat, c->nftiles_all});
  HIPCHK(c, dalloc(&c->sb.partial, 3 * nwork));
  HIPCHK(c, dalloc(&c->sb.counter, nsys));
  HIPCHK(c, hipMemset(c->sb.counter, 0, sizeof(unsigned) * nsys));
  HIPCHK(c, dalloc(&c->sb.ss, nsys));
  HIPCHK(c, hipMemset(c->sb.ss, 0, sizeof(SolveScal) * nsys));
  HIPCHK(c, dalloc(&c->sb.ndone, 1));
  HIPCHK(c, dalloc(&c->dose_t, (size_t)c->nreps * 3 * HCA_MAX_DOSES));
  HIPCHK(c, dalloc(&c->dose_a, (size_t)c->nreps * 3 * HCA_MAX_DOSES));
  HIPCHK(c, dalloc(&c->g0, (size_t)c->nreps * 6));   // levels at both ends of a field substep
  if (c->prm.o2_newton > 0 && (st = big(&c->b_o2lin, (size_t)c->ntot)) != HCA_OK) return st;
  if (c->prm.x0_extrapolate && (st = big(&c->Fprev, n3)) != HCA_OK) return st;
  if (c->prm.x0_extrapolate == 3) {
    if ((st = big(&c->Fprev2, n3)) != HCA_OK) return st;
    HIPCHK(c, dalloc(&c->d_gpart, (size_t)kGuessPartsPerTile * std::max(1, c->sys_all.ntiles)));
    HIPCHK(c, dalloc(&c->d_galpha, 4 * (size_t)nsys));
  }
  {
    const CgFinish<Real> fin{c->F, c->sb.p0, c->sb.p1, c->sb.ss, c->ntot, c->dp.nf, c->nreps};
    HIPCHK(c, dalloc(&c->d_fin, 1));
    HIPCHK(c, hipMemcpy(c->d_fin, &fin, sizeof fin, hipMemcpyHostToDevice));
  }
  HIPCHK(c, dalloc(&c->d_step, 1));
  HIPCHK(c, dalloc(&c->d_cnt, c->nreps));
  HIPCHK(c, dalloc(&c->d_cpart, (size_t)c->work.nflat * kCounterSlots));
  HIPCHK(c, hipMemset(c->d_cnt, 0, sizeof(Counters) * c->nreps));
  HIPCHK(c, dalloc(&c->d_bad, 1));
  HIPCHK(c, hipHostMalloc((void**)&c->h_ss, sizeof(SolveScal) * nsys, hipHostMallocDefault));
  HIPCHK(c, hipHostMalloc((void**)&c->h_cnt, sizeof(Counters) * c->nreps, hipHostMallocDefault));
  return HCA_OK;
}

// ---- multigrid hierarchy -------------------------------------------------------

template <typename T>
hca_status mg_alloc(Ctx* c, T** p, size_t count) {
  hipError_t e = dalloc(p, count);
  if (e == hipErrorOutOfMemory) return fail(c, HCA_E_NOMEM, "device memory exhausted (multigrid)");
  HIPCHK(c, e);
  c->mg_mem.push_back((void*)*p);
  return HCA_OK;
}

template <typename T>
hca_status mg_upload(Ctx* c, T** p, const std::vector<T>& v) {
  hca_status st = mg_alloc(c, p, v.size());
  if (st != HCA_OK) return st;
  if (!v.empty()) HIPCHK(c, hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return HCA_OK;
}

// Hierarchy of every system (field-major, like the solver tables): level
// dims by ceil halving down to one cell (at least two levels); kc, the first
// level handed to the one-workgroup coarse solve (<= mg_coarse_max cells and
// its LDS block within the device's per-workgroup LDS); level arrays, per-level tiles, coarse-solve
// descriptors.  mg1 is the oxygen prefix (the first nreps systems) of mg_all.
hca_status build_mg(Ctx* c) {
  const int R = c->nreps;
  const int S = c->dp.nf * R;
  // LDS of one workgroup: the coarse solve's levels must fit (160 KiB on gfx950)
  int lds_dev = 65536;
  if (hipDeviceGetAttribute(&lds_dev, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess)
    lds_dev = 65536;
  // (less 1 KiB for the coarse kernel's static LDS)
  const size_t kLdsCap = (size_t)std::max(lds_dev, 65536) - 1024;
  auto cells = [](const std::array<int, 3>& a) { return (long long)a[0] * a[1] * a[2]; };
  std::vector<std::vector<std::array<int, 3>>> dims(R);
  std::vector<int> kcr(R, 1);
  for (int r = 0; r < R; ++r) {
    auto& d = dims[r];
    d.push_back({c->reps[r].nx, c->reps[r].ny, c->reps[r].nz});
    while (cells(d.back()) > 1 || d.size() < 2) {
      const auto b = d.back();
      d.push_back({(b[0] + 1) / 2, (b[1] + 1) / 2, (b[2] + 1) / 2});
      if ((int)d.size() > kMaxLevels) return fail(c, HCA_E_INVALID, "lattice too large for multigrid");
    }
    for (int k = 1; k < (int)d.size(); ++k) {
      size_t lds = 0;
      for (int j = k; j < (int)d.size(); ++j) lds += kCoarseLdsPerCell * sizeof(float) * (size_t)cells(d[j]);
      const long long n = cells(d[k]);
      if (n <= c->prm.mg_coarse_max && n <= (long long)kCoarseThreads * kCoarseMaxCellsPerThread &&
          lds <= kLdsCap) {
        kcr[r] = k;
        break;
      }
    }
  }
  int nglob = 1;
  for (int r = 0; r < R; ++r) nglob = std::max(nglob, kcr[r]);
  std::vector<RepDev> sd(S);
  HIPCHK(c, hipMemcpy(sd.data(), c->d_sys, sizeof(RepDev) * S, hipMemcpyDeviceToHost));
  MgBufs& mg = c->mg_all;
  mg.nlev_glob = nglob;
  // Smoothing: each pair of weighted-Jacobi sweeps is the two-step Chebyshev
  // polynomial (1 - w_a t)(1 - w_b t) of least maximum over t in [1/3, 2], the
  // spectrum of D^-1 A on the oscillatory modes of the 7-point operator in
  // 3-D (2 bounds D^-1 A by diagonal dominance; 1/3 is its smallest symbol
  // value with some frequency at pi/2): 1/w are the Chebyshev points
  // 7/6 -+ (5/6) cos(pi/4).  Its maximum there, 1/T_2(7/5) ~ 0.34, beats two
  // equal sweeps at the best single weight 6/7, (5/7)^2 ~ 0.51.
  {
    const double mid = 7.0 / 6.0, half = 5.0 / 6.0, c4 = std::sqrt(0.5);
    mg.w_a = (float)(1.0 / (mid + half * c4));
    mg.w_b = (float)(1.0 / (mid - half * c4));
  }
  // Level 0 smooths with the three-step Chebyshev polynomial of least
  // maximum over t in [0.2, 2] (1/w = 1.1 + 0.9 cos((2k - 1) pi / 6)): the
  // finest level's smoothing is what limits the oxygen operator's
  // convergence (its vessel voxels' reaction terms are orders of magnitude
  // above the couplings); a third sweep there takes the oxygen solve from 8 to
  // 6 iterations at 128^3, one on the coarser levels changes nothing.
  for (int k = 0; k < 3; ++k)
    mg.w0[k] = (float)(1.0 / (1.1 + 0.9 * std::cos((2 * k + 1) * M_PI / 6.0)));
  mg.fused = c->prm.mg_fuse;
  c->mg1 = mg;
  std::vector<float*> pc(kMaxLevels, nullptr), pr(kMaxLevels, nullptr), pu(kMaxLevels, nullptr);
  std::vector<std::vector<MgRep>> mreps(nglob + 1);
  for (int k = 0; k <= nglob; ++k) {
    std::vector<MgRep>& mr = mreps[k];
    mr.resize(S);
    std::vector<Tile> tiles, rtiles, ftiles;
    int ntiles1 = 0, nrtiles1 = 0, nftiles1 = 0, fchunk = 16;
    long long off = 0;
    // a coarser level smooths in fused passes when every system iterates on
    // it, all its cells are full 2^k-cubes (uniform couplings a 2^k) and the
    // level holds at least g_fuse_min_cells cells over all systems (smaller
    // levels run faster as one kernel per sweep)
    bool fuse_k = k >= 1 && c->prm.mg_fuse;
    long long cells_k = 0;
    for (int r = 0; fuse_k && r < R; ++r) {
      for (int i = 0; i < 3; ++i)
        fuse_k = fuse_k && k < kcr[r] && dims[r][0][i] % (1 << k) == 0;
      if (fuse_k) cells_k += (long long)dims[r][k][0] * dims[r][k][1] * dims[r][k][2];
    }
    fuse_k = fuse_k && cells_k * (S / R) >= g_fuse_min_cells;
    for (int s = 0; s < S; ++s) {
      const int r = s % R;
      MgRep& m = mr[s];
      memset(&m, 0, sizeof m);
      m.k = k;
      m.n0x = dims[r][0][0];
      m.n0y = dims[r][0][1];
      m.n0z = dims[r][0][2];
      m.a = (float)sd[s].a;
      if (k < (int)dims[r].size() && k <= kcr[r]) {
        m.nx = dims[r][k][0];
        m.ny = dims[r][k][1];
        m.nz = dims[r][k][2];
        m.active = k < kcr[r];
        if (k == 0) {
          m.tx = sd[s].tx;
          m.off = sd[s].off;
          m.tile_b0 = sd[s].tile_b0;
          m.tile_nb = sd[s].tile_nb;
        } else {
          m.tx = pick_tx(m.nx);
          m.off = off;
          off += (long long)m.nx * m.ny * m.nz;
          const int tz = even_depth(pick_tz(m.nx, m.ny, m.nz, m.tx, g_mg_tile_target), m.nz);
          if (m.active) {
            m.tile_b0 = (int)tiles.size();
            add_tiles(tiles, s, m.nx, m.ny, m.nz, m.tx, tz);
            m.tile_nb = (int)tiles.size() - m.tile_b0;
          }
          m.rtile_b0 = (int)rtiles.size();
          add_tiles(rtiles, s, m.nx, m.ny, m.nz, m.tx, tz);
          m.rtile_nb = (int)rtiles.size() - m.rtile_b0;
          if (fuse_k) {
            add_tiles(ftiles, s, m.nx, m.ny, m.nz, m.tx, fused_depth(m.nx, m.ny, m.nz, m.tx), kF3Block / m.tx);
            fchunk = std::max(fchunk, std::min(8 * ((m.nx + m.tx - 1) / m.tx), 256));
          }
        }
      }
      if (s == R - 1) {
        ntiles1 = (int)tiles.size();
        nrtiles1 = (int)rtiles.size();
        nftiles1 = (int)ftiles.size();
      }
    }
    MgLevel& L = mg.lev[k];
    MgRep* d_mr = nullptr;
    hca_status st = mg_upload(c, &d_mr, mr);
    if (st != HCA_OK) return st;
    L.reps = d_mr;
    if (k == 0) {
      L.tiles = c->d_stiles;
      L.ntiles = c->sys_all.ntiles;
      ntiles1 = c->sys1.ntiles;
      L.ftiles = c->d_ftiles;
      L.nftiles = c->nftiles_all;
      L.fchunk = c->fchunk;
      const size_t n = (size_t)c->dp.nf * c->ntot;
      if ((st = mg_alloc(c, &L.dinv, n)) != HCA_OK || (st = mg_alloc(c, &L.u, n)) != HCA_OK ||
          (st = mg_alloc(c, &L.ualt, n)) != HCA_OK)
        return st;
    } else {
      Tile* dt = nullptr;
      Tile* drt = nullptr;
      Tile* dft = nullptr;
      if ((st = mg_upload(c, &dt, tiles)) != HCA_OK || (st = mg_upload(c, &drt, rtiles)) != HCA_OK ||
          (!ftiles.empty() && (st = mg_upload(c, &dft, ftiles)) != HCA_OK))
        return st;
      L.tiles = dt;
      L.ntiles = (int)tiles.size();
      L.rtiles = drt;
      L.nrtiles = (int)rtiles.size();
      L.ftiles = dft;
      L.nftiles = (int)ftiles.size();
      L.fchunk = fchunk;
      const size_t n = (size_t)std::max<long long>(off, 1);
      if ((st = mg_alloc(c, &L.c, n)) != HCA_OK || (st = mg_alloc(c, &L.dinv, n)) != HCA_OK ||
          (st = mg_alloc(c, &L.r, n)) != HCA_OK || (st = mg_alloc(c, &L.u, n)) != HCA_OK ||
          (st = mg_alloc(c, &L.ualt, n)) != HCA_OK)
        return st;
      pc[k] = L.c;
      pr[k] = L.r;
      pu[k] = L.u;
    }
    c->mg1.lev[k] = L;
    c->mg1.lev[k].ntiles = ntiles1;
    c->mg1.lev[k].nftiles = k == 0 ? c->nftiles1 : nftiles1;
    c->mg1.lev[k].nrtiles = k == 0 ? 0 : nrtiles1;
  }
  int nglob1 = 1;
  for (int r = 0; r < R; ++r) nglob1 = std::max(nglob1, kcr[r]);
  c->mg1.nlev_glob = nglob1;
  // coarse-solve descriptors
  std::vector<MgCoarseRep> cr(S);
  size_t lds_max = 0;
  long long pre_total = 0;
  for (int s = 0; s < S; ++s) {
    const int r = s % R;
    MgCoarseRep& d = cr[s];
    memset(&d, 0, sizeof d);
    d.kc = kcr[r];
    d.nlev = (int)dims[r].size() - kcr[r];
    d.a = (float)sd[s].a;
    for (int i = 0; i < 3; ++i) d.n0[i] = dims[r][0][i];
    int o = 0, g = 0;
    for (int j = 0; j < d.nlev; ++j) {
      for (int i = 0; i < 3; ++i) d.dims[j][i] = dims[r][kcr[r] + j][i];
      d.lds_off[j] = o;
      d.pre_lev[j] = g;
      o += (kCoarseLdsPerCell - 4) * d.dims[j][0] * d.dims[j][1] * d.dims[j][2];
      g += 4 * d.dims[j][0] * d.dims[j][1] * d.dims[j][2];
    }
    d.pre_len = g;
    lds_max = std::max(lds_max, (size_t)(o + g) * sizeof(float));
    d.off_kc = mreps[kcr[r]][s].off;
    d.r_kc = pr[kcr[r]] + d.off_kc;
    d.u_kc = pu[kcr[r]] + d.off_kc;
    d.pre_off = pre_total;
    pre_total += g;
  }
  MgCoarseRep* dcr = nullptr;
  hca_status st = mg_upload(c, &dcr, cr);
  if (st != HCA_OK) return st;
  mg.coarse = dcr;
  mg.coarse_lds_bytes = (int)lds_max;
  if (lds_max > 65536) HIPCHK(c, mg_set_coarse_lds((int)lds_max));
  if ((st = mg_alloc(c, &mg.coarse_pre, (size_t)pre_total)) != HCA_OK) return st;
  if ((st = mg_upload(c, &mg.lev_c, pc)) != HCA_OK || (st = mg_upload(c, &mg.lev_r, pr)) != HCA_OK ||
      (st = mg_upload(c, &mg.lev_u, pu)) != HCA_OK)
    return st;
  c->mg1.coarse = mg.coarse;
  c->mg1.coarse_pre = mg.coarse_pre;
  c->mg1.coarse_lds_bytes = mg.coarse_lds_bytes;
  c->mg1.lev_c = mg.lev_c;
  c->mg1.lev_r = mg.lev_r;
  c->mg1.lev_u = mg.lev_u;
  return HCA_OK;
}

// Algorithm 1, steady oxygen: Picard on the uptake coefficient, each iterate
// one CG solve of the oxygen systems; stops when the nonlinear residual of the
// current iterate (the solve's initial residual) is below init_rtol ||b||.
hca_status steady_oxygen(Ctx* c) {
  const Work& wk = c->work;
  std::vector<Real> k0((size_t)c->ntot, (Real)c->prm.K0);
  HIPCHK(c, hipMemcpyAsync(c->K, k0.data(), k0.size() * sizeof(Real), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int m = 0; m < c->prm.init_maxit; ++m) {
    launch_setup_o2(c->stream, wk, c->dp, c->L, c->w, c->K, c->c, c->b, 1);
    launch_cg_start(c->stream, c->sys1, std::max(c->prm.init_rtol, kRtolFloor), c->prm.cg_maxit, c->c, c->b, c->F,
                    c->sb, 1u, c->nreps);
    HIPCHK(c, hipMemcpyAsync(c->h_ss, c->sb.ss, sizeof(SolveScal) * c->nreps,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    bool all = true;
    for (int r = 0; r < c->nreps; ++r) all = all && c->h_ss[r].conv;
    if (all) {
      c->picard_iters = m;
      return HCA_OK;
    }
    hca_status st = solve(c, c->sys1, c->mg1, 1u, solve_rtol(c), c->prm.cg_maxit, 1);
    if (st != HCA_OK) return st;
  }
  return fail(c, HCA_E_NOCONV, "steady oxygen Picard iteration did not converge");
}

void free_all(Ctx* c) {
  void* bufs[] = {c->L, c->code, c->win, (void*)c->ca_list.cells, (void*)c->ca_list.item_n, c->w, c->P, c->Vc, c->phi, c->F, c->c, c->b,
                  c->sb.r, c->sb.z, (void*)c->sb.z32, (void*)c->sb.r32, c->sb.p0, c->sb.p1, c->sb.q, c->sb.dinv, c->sb.partial,
                  c->sb.counter, c->sb.ss, c->sb.ndone, c->dose_t, c->dose_a, c->g0, c->b_o2lin, c->Fprev, c->Fprev2, c->d_gpart, c->d_galpha, (void*)c->d_fin, c->d_step,
                  c->d_reps, c->d_flat, c->d_tiles, c->d_sys, c->d_sflat, c->d_stiles, c->d_ftiles, c->d_cnt, (void*)c->d_cpart,
                  c->d_bad, c->d_theta, (void*)c->d_pack, (void*)c->d_gelu, c->before,
                  c->item_cnt, c->item_off};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  for (void* p : c->mg_mem)
    if (p) (void)hipFree(p);
  c->mg_mem.clear();
  if (c->h_ss) (void)hipHostFree(c->h_ss);
  if (c->h_cnt) (void)hipHostFree(c->h_cnt);
  for (auto& e : c->pending) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (auto e : c->free_events) (void)hipEventDestroy(e);
  for (auto& g : c->iter_graph)
    if (g) (void)hipGraphExecDestroy(g);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

// n stored field values (device, Real) out as FP64 into dst (host or device).
template <typename R>
hca_status field_out(Ctx* c, const R* src, size_t n, void* dst, int dst_is_device) {
  if constexpr (sizeof(R) == sizeof(double)) {
    HIPCHK(c, hipMemcpyAsync(dst, src, sizeof(double) * n,
                             dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  } else if (dst_is_device) {
    launch_convert(c->stream, src, static_cast<double*>(dst), (long long)n);
    HIPCHK(c, hipGetLastError());
  } else {
    std::vector<R> tmp(n);
    HIPCHK(c, hipMemcpyAsync(tmp.data(), src, sizeof(R) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<double> d(tmp.begin(), tmp.end());
    memcpy(dst, d.data(), sizeof(double) * n);
  }
  return HCA_OK;
}

// n FP64 values (host or device) into stored field values (device, Real),
// rounded to Real.  Returns after the copy has completed.
template <typename R>
hca_status field_in(Ctx* c, const void* src, size_t n, int src_is_device, R* dst) {
  if constexpr (sizeof(R) == sizeof(double)) {
    HIPCHK(c, hipMemcpyAsync(dst, src, sizeof(double) * n,
                             src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  } else if (src_is_device) {
    launch_convert(c->stream, static_cast<const double*>(src), dst, (long long)n);
    HIPCHK(c, hipGetLastError());
  } else {
    std::vector<double> d(n);
    memcpy(d.data(), src, sizeof(double) * n);
    std::vector<R> tmp(d.begin(), d.end());
    HIPCHK(c, hipMemcpyAsync(dst, tmp.data(), sizeof(R) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return HCA_OK;
}

// A solved field (stored as Real) or nullptr.
Real* real_field(Ctx* c, hca_field f) {
  switch (f) {
    case HCA_F_O2: return c->K;
    case HCA_F_DRUG1: return c->G1;
    case HCA_F_DRUG2: return c->G2;
    case HCA_F_VEGF: return c->V;
    case HCA_F_DRUG3: return c->G3;
    default: return nullptr;
  }
}

void* field_ptr(Ctx* c, hca_field f, size_t& elem) {
  elem = 8;
  switch (f) {
    case HCA_F_O2: return c->K;
    case HCA_F_DRUG1: return c->G1;
    case HCA_F_DRUG2: return c->G2;
    case HCA_F_CELL: elem = 1; return c->L;
    case HCA_F_P53: return c->P;
    case HCA_F_VEGF_IC: return c->Vc;
    case HCA_F_PHI: return c->phi;
    case HCA_F_VESSEL_W: return c->w;
    case HCA_F_VEGF: return c->V;
    case HCA_F_DRUG3: return c->G3;
  }
  return nullptr;
}

// ---- checkpoint / resume ---------------------------------------------------------
//
// State blob of one replicate (host or device memory, little-endian):
//   header (StateHeader, 96 bytes)
//   L     uint8 cell map, n bytes, padded to a multiple of 8
//   w     FP64 vessel map, n
//   F     FP64 solved fields in solver order K, G1, G2 (G3 with drug3, V with
//         vegf), nf x n
//   cells FP64 P, Vc, phi, 3 x n
//   Fprev FP64 each solved field at its previous solve (the initial-guess
//         history), nf x n, present with flag bit 2
//   Fprev2 FP64 each solved field at the solve before that, nf x n, present
//         with flag bit 3
// n = nx ny nz, arrays x-fastest as everywhere.

constexpr uint64_t kStateMagic = 0x4554415453414348ull;   // "HCASTATE"
constexpr uint32_t kStateVersion = 1;
constexpr uint32_t kStateVegf = 1u, kStateDrug3 = 2u, kStatePrev = 4u, kStatePrev2 = 8u;

struct StateHeader {
  uint64_t magic;
  uint32_t version, flags;
  int32_t nx, ny, nz, nf;
  int64_t step;
  uint64_t seed;
  int64_t total_divisions, total_kills, total_births, total_deaths;
  uint64_t reserved[2];
};
static_assert(sizeof(StateHeader) == 96, "state header layout");

struct StateLayout {
  StateHeader hdr;
  size_t n, off_L, off_w, off_F, off_cell, off_prev, off_prev2, bytes;
};

StateLayout state_layout(const StateHeader& h) {
  StateLayout l;
  l.hdr = h;
  l.n = (size_t)h.nx * h.ny * h.nz;
  l.off_L = sizeof(StateHeader);
  l.off_w = l.off_L + (l.n + 7) / 8 * 8;
  l.off_F = l.off_w + 8 * l.n;
  l.off_cell = l.off_F + 8 * (size_t)h.nf * l.n;
  l.off_prev = l.off_cell + 24 * l.n;
  l.off_prev2 = l.off_prev + ((h.flags & kStatePrev) ? 8 * (size_t)h.nf * l.n : 0);
  l.bytes = l.off_prev2 + ((h.flags & kStatePrev2) ? 8 * (size_t)h.nf * l.n : 0);
  return l;
}

StateHeader context_header(const Ctx* c, int rep) {
  StateHeader h{};
  const RepHost& R = c->reps[rep];
  h.magic = kStateMagic;
  h.version = kStateVersion;
  h.flags = (c->dp.vegf ? kStateVegf : 0u) | (c->dp.drug3 ? kStateDrug3 : 0u) |
            (c->Fprev ? kStatePrev : 0u) | (c->Fprev2 ? kStatePrev2 : 0u);
  h.nx = R.nx;
  h.ny = R.ny;
  h.nz = R.nz;
  h.nf = c->dp.nf;
  h.step = c->step;
  h.seed = R.seed;
  return h;
}

// Header checks against a replicate's lattice and seed; msg names the problem.
hca_status check_header(const StateHeader& h, size_t bytes, int nx, int ny, int nz, uint64_t seed,
                        StateLayout& lay, std::string& msg) {
  if (bytes < sizeof(StateHeader)) {
    msg = "state buffer shorter than its header";
    return HCA_E_RANGE;
  }
  if (h.magic != kStateMagic || h.version != kStateVersion) {
    msg = "not a state blob of this library version";
    return HCA_E_INVALID;
  }
  if (h.nx != nx || h.ny != ny || h.nz != nz || h.nf < 3 || h.nf > 5) {
    msg = "state lattice differs from the replicate's";
    return HCA_E_INVALID;
  }
  if (h.seed != seed) {
    msg = "state seed differs from the replicate's";
    return HCA_E_INVALID;
  }
  if (h.step < 0) {
    msg = "negative step index";
    return HCA_E_INVALID;
  }
  lay = state_layout(h);
  if (bytes < lay.bytes) {
    msg = "state buffer shorter than its arrays";
    return HCA_E_RANGE;
  }
  return HCA_OK;
}

hca_status parse_state_host(const void* src, size_t bytes, const hca_replicate& R, StateLayout& lay,
                            std::string& msg) {
  if (!src) {
    msg = "null state";
    return HCA_E_INVALID;
  }
  StateHeader h{};
  if (bytes >= sizeof h) memcpy(&h, src, sizeof h);
  return check_header(h, bytes, R.nx, R.ny, R.nz, R.seed, lay, msg);
}

hca_status export_state(Ctx* c, int rep, void* dst, size_t dst_bytes, int dst_is_device) {
  const RepHost& R = c->reps[rep];
  const StateLayout lay = state_layout(context_header(c, rep));
  if (dst_bytes < lay.bytes) return fail(c, HCA_E_RANGE, "state buffer too small");
  StateHeader h = lay.hdr;
  HIPCHK(c, hipMemcpyAsync(c->h_cnt, c->d_cnt, sizeof(Counters) * c->nreps, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  h.total_divisions = (int64_t)c->h_cnt[rep].total_divisions;
  h.total_kills = (int64_t)c->h_cnt[rep].total_kills;
  h.total_births = (int64_t)c->h_cnt[rep].total_births;
  h.total_deaths = (int64_t)c->h_cnt[rep].total_deaths;
  char* d = static_cast<char*>(dst);
  const hipMemcpyKind out = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const size_t n = lay.n;
  HIPCHK(c, hipMemcpyAsync(d, &h, sizeof h, dst_is_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(d + lay.off_L, c->L + R.off, n, out, c->stream));
  HIPCHK(c, hipMemcpyAsync(d + lay.off_w, c->w + R.off, 8 * n, out, c->stream));
  hca_status st;
  for (int f = 0; f < c->dp.nf; ++f)
    if ((st = field_out(c, c->F + (size_t)f * c->ntot + R.off, n, d + lay.off_F + 8 * n * f,
                        dst_is_device)) != HCA_OK)
      return st;
  const double* cell[3] = {c->P, c->Vc, c->phi};
  for (int k = 0; k < 3; ++k)
    HIPCHK(c, hipMemcpyAsync(d + lay.off_cell + 8 * n * k, cell[k] + R.off, 8 * n, out, c->stream));
  if (c->Fprev)
    for (int f = 0; f < c->dp.nf; ++f)
      if ((st = field_out(c, c->Fprev + (size_t)f * c->ntot + R.off, n, d + lay.off_prev + 8 * n * f,
                          dst_is_device)) != HCA_OK)
        return st;
  if (c->Fprev2)
    for (int f = 0; f < c->dp.nf; ++f)
      if ((st = field_out(c, c->Fprev2 + (size_t)f * c->ntot + R.off, n, d + lay.off_prev2 + 8 * n * f,
                          dst_is_device)) != HCA_OK)
        return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HCA_OK;
}

// check = false: leave the census and the non-finite check to the caller
// (a resume imports every replicate first: until then the others hold no state)
hca_status import_state(Ctx* c, int rep, const void* src, size_t src_bytes, int src_is_device,
                        bool check = true) {
  const RepHost& R = c->reps[rep];
  StateHeader h{};
  if (src_bytes >= sizeof h) {
    HIPCHK(c, hipMemcpyAsync(&h, src, sizeof h, src_is_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  StateLayout lay;
  std::string msg;
  hca_status st = check_header(h, src_bytes, R.nx, R.ny, R.nz, R.seed, lay, msg);
  if (st == HCA_OK && (h.nf != c->dp.nf || ((h.flags & kStateVegf) != 0) != (c->dp.vegf != 0) ||
                       ((h.flags & kStateDrug3) != 0) != (c->dp.drug3 != 0))) {
    msg = "state fields (third drug, VEGF) differ from the context's options";
    st = HCA_E_INVALID;
  }
  if (st == HCA_OK && c->nreps > 1 && h.step != c->step) {
    msg = "state step differs from the context's (a context advances its replicates together)";
    st = HCA_E_INVALID;
  }
  if (st != HCA_OK) {
    c->err = msg;
    return st;
  }
  const char* s = static_cast<const char*>(src);
  const hipMemcpyKind in = src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const size_t n = lay.n;
  c->fixed_ops = false;   // the vessel map may change: rebuild every field's c and multigrid data
  // the maps staged in the proposal buffer and the right-hand side (both
  // rewritten before their next use) and validated together
  double* wstage = reinterpret_cast<double*>(c->b);   // nf x ntot Real values: room for ntot doubles
  HIPCHK(c, hipMemcpyAsync(c->code + R.off, s + lay.off_L, n, in, c->stream));
  HIPCHK(c, hipMemcpyAsync(wstage + R.off, s + lay.off_w, 8 * n, in, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_bad, 0, sizeof(unsigned long long), c->stream));
  launch_validate_cells(c->stream, c->work, c->code, wstage, rep, c->d_bad);
  unsigned long long bad = 0;
  HIPCHK(c, hipMemcpyAsync(&bad, c->d_bad, sizeof bad, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (bad) {
    c->err = "state cell map has codes outside {0,1,2}, cells on vessel voxels or bad weights";
    return HCA_E_INVALID;
  }
  HIPCHK(c, hipMemcpyAsync(c->L + R.off, c->code + R.off, n, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->w + R.off, wstage + R.off, 8 * n, hipMemcpyDeviceToDevice, c->stream));
  for (int f = 0; f < c->dp.nf; ++f)
    if ((st = field_in(c, s + lay.off_F + 8 * n * f, n, src_is_device, c->F + (size_t)f * c->ntot + R.off)) !=
        HCA_OK)
      return st;
  double* cell[3] = {c->P, c->Vc, c->phi};
  for (int k = 0; k < 3; ++k)
    HIPCHK(c, hipMemcpyAsync(cell[k] + R.off, s + lay.off_cell + 8 * n * k, 8 * n, in, c->stream));
  if (c->Fprev)
    for (int f = 0; f < c->dp.nf; ++f) {
      Real* dstp = c->Fprev + (size_t)f * c->ntot + R.off;
      if (h.flags & kStatePrev) {
        if ((st = field_in(c, s + lay.off_prev + 8 * n * f, n, src_is_device, dstp)) != HCA_OK) return st;
      } else {   // no history saved: the extrapolation restarts from the state
        HIPCHK(c, hipMemcpyAsync(dstp, c->F + (size_t)f * c->ntot + R.off, sizeof(Real) * n,
                                 hipMemcpyDeviceToDevice, c->stream));
      }
    }
  if (c->Fprev2)   // after Fprev: without its own section the history restarts from Fprev
    for (int f = 0; f < c->dp.nf; ++f) {
      Real* dstp = c->Fprev2 + (size_t)f * c->ntot + R.off;
      if (h.flags & kStatePrev2) {
        if ((st = field_in(c, s + lay.off_prev2 + 8 * n * f, n, src_is_device, dstp)) != HCA_OK) return st;
      } else {
        HIPCHK(c, hipMemcpyAsync(dstp, c->Fprev + (size_t)f * c->ntot + R.off, sizeof(Real) * n,
                                 hipMemcpyDeviceToDevice, c->stream));
      }
    }
  // cumulative counts of the replicate; the last step's events restart at 0
  HIPCHK(c, hipMemcpyAsync(c->h_cnt, c->d_cnt, sizeof(Counters) * c->nreps, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  Counters k = c->h_cnt[rep];
  k.committed = k.kills = k.divisions = k.nospace = k.lost = 0;
  k.births = k.deaths = 0;
  k.total_divisions = (unsigned long long)h.total_divisions;
  k.total_kills = (unsigned long long)h.total_kills;
  k.total_births = (unsigned long long)h.total_births;
  k.total_deaths = (unsigned long long)h.total_deaths;
  HIPCHK(c, hipMemcpyAsync(c->d_cnt + rep, &k, sizeof k, hipMemcpyHostToDevice, c->stream));
  if (h.step != c->step) {
    long long st64 = h.step;
    HIPCHK(c, hipMemcpyAsync(c->d_step, &st64, sizeof st64, hipMemcpyHostToDevice, c->stream));
    c->step = h.step;
  }
  if (!check) return HCA_OK;
  launch_stats(c->stream, c->work, c->L, c->w, c->F, c->dp.nf, c->ntot, c->P, c->Vc, c->phi,
               c->d_cpart, c->d_cnt);
  HIPCHK(c, hipGetLastError());
  return check_after(c);
}

hca_status init_impl(::hca_ctx** out, const hca_params* p, const hca_replicate* reps, int n_reps,
                     void* stream, const void* const* states, const size_t* state_bytes,
                     int states_on_device);

}  // namespace


#if HCA_RT_PRIMARY
extern "C" hca_status hca_default_params(hca_params* out) {
  if (!out) return HCA_E_INVALID;
  memset(out, 0, sizeof *out);
  out->h_um = 20.0;
  out->dt_min = 30.0;
  out->D_K = 1.05e5;
  out->r_k = 1.88e4;
  out->K0 = 20.0;
  out->phi_K = 900.0;
  out->K1 = 2.5;
  out->D_G = 9.6e3;
  out->psi_G = 1.0e-2;
  out->kappa_G = 0.1;
  out->k_pk[0] = 3.93e3 / 2430e3;   // cyclophosphamide cl_3 / u
  out->k_pk[1] = 1.75 / 27.0;       // fluorouracil v_max / k_m (linear regime)
  out->G_ref[0] = 1.0;
  out->G_ref[1] = 1.0;
  out->b_int[0] = 1;
  out->b_int[1] = 1;
  out->k1 = 4.0e-4;
  out->k1p = 1.0e-2;
  out->K_p53 = 1.0e-2;
  out->k2 = 2.0e-3;
  out->k2p = 1.0e-2;
  out->k2pp = -2.0e-4;
  out->J5 = 4.0e-2;
  out->K_V = 1.0e-2;
  out->K_phi = 1.4;
  out->T_cycle = 3.74 * 1440.0;
  out->ode_substeps = 30;
  out->precond = 1;
  out->cg_rtol = 1.0e-10;
  out->cg_maxit = 2000;
  out->mg_smooth = 2;
  out->mg_coarse_max = 4096;
  out->init_rtol = 1.0e-10;
  out->init_maxit = 200;
  out->profile = 0;
  out->graphs = 1;
  out->autotune = 0;
  out->pde_substeps = 1;
  out->pde_theta = 1.0;
  out->o2_newton = 0;
  out->pk_mm = 0;
  out->mm_vmax = 1.75;
  out->mm_km = 27.0;
  out->vegf = 0;
  out->D_V = 3.52e3;
  out->psi_V = 1.0e-2;
  out->sec_V = 6.66e-6;
  out->dv_min = 720.0;
  out->V_low = 1.0e-6;
  out->V_high = 1.0e-4;
  out->p_death = 0.05;
  out->birth_per_V = 100.0;
  out->w_new = 1.0;
  out->drug3 = 0;
  out->epi_w1 = 18.0e3;
  out->epi_w2 = 957.0e3;
  out->epi_w3 = 25.0e3;
  out->epi_q2 = 0.918e3;
  out->epi_q3 = 0.25e3;
  out->epi_cl = 0.983e3;
  out->G_ref3 = 1.0;
  out->b_int3 = 1;
  out->x0_extrapolate = 3;
  out->precision = 64;
  out->mg_fuse = 1;
  return HCA_OK;
}
#endif

hca_status api_init(::hca_ctx** out, const hca_params* p, const hca_replicate* reps, int n_reps,
                    void* stream) {
  if constexpr (sizeof(Real) == sizeof(double)) {
    return init_impl(out, p, reps, n_reps, stream, nullptr, nullptr, 0);
  } else {
    // precision 32: Algorithm 1's initialisation (the steady oxygen, whose
    // operator amplifies residuals ~1e4-fold) in FP64, then the state rounded
    // to FP32 through device-resident state blobs
    if (!out || !p || !reps || n_reps < 1) return HCA_E_INVALID;
    *out = nullptr;
    hca_params p64 = *p;
    p64.precision = 64;
    ::hca_ctx* c64 = nullptr;
    hca_status st = hca::rt64::api_init(&c64, &p64, reps, n_reps, stream);
    if (st != HCA_OK) return st;
    std::vector<void*> blobs((size_t)n_reps, nullptr);
    std::vector<size_t> bytes((size_t)n_reps, 0);
    for (int r = 0; r < n_reps && st == HCA_OK; ++r) {
      st = hca::rt64::api_state_bytes(c64, r, &bytes[r]);
      if (st == HCA_OK && hipMalloc(&blobs[r], bytes[r]) != hipSuccess) st = HCA_E_NOMEM;
      if (st == HCA_OK) st = hca::rt64::api_export_state(c64, r, blobs[r], bytes[r], 1);
    }
    hca::rt64::api_destroy(c64);
    if (st == HCA_OK) st = init_impl(out, p, reps, n_reps, stream, blobs.data(), bytes.data(), 1);
    for (void* b : blobs)
      if (b) (void)hipFree(b);
    return st;
  }
}

hca_status api_init_from_state(::hca_ctx** out, const hca_params* p, const hca_replicate* reps,
                               const void* const* states, const size_t* state_bytes, int n_reps,
                               void* stream) {
  if (!out || !p || !reps || !states || !state_bytes || n_reps < 1) return HCA_E_INVALID;
  *out = nullptr;
  // the cell and vessel maps come from the states (validated with the
  // replicates' dose lists before anything is allocated)
  std::vector<hca_replicate> rr(reps, reps + n_reps);
  int64_t step0 = -1;
  for (int r = 0; r < n_reps; ++r) {
    StateLayout lay;
    std::string msg;
    const hca_status st = parse_state_host(states[r], state_bytes[r], reps[r], lay, msg);
    if (st != HCA_OK) {
      fprintf(stderr, "hca_init_from_state: replicate %d: %s\n", r, msg.c_str());
      return st;
    }
    if (step0 >= 0 && lay.hdr.step != step0) {
      fprintf(stderr, "hca_init_from_state: replicate %d is at step %lld, replicate 0 at %lld "
                      "(a context advances its replicates together)\n",
              r, (long long)lay.hdr.step, (long long)step0);
      return HCA_E_INVALID;
    }
    step0 = lay.hdr.step;
    const char* base = static_cast<const char*>(states[r]);
    rr[r].cell = reinterpret_cast<const uint8_t*>(base + lay.off_L);
    rr[r].vessel_w = reinterpret_cast<const double*>(base + lay.off_w);
  }
  return init_impl(out, p, rr.data(), n_reps, stream, states, state_bytes, 0);
}


namespace {

hca_status init_impl(::hca_ctx** out, const hca_params* p, const hca_replicate* reps, int n_reps,
                     void* stream, const void* const* states, const size_t* state_bytes,
                     int states_on_device) {
  if (!out || !p || !reps || n_reps < 1) return HCA_E_INVALID;
  *out = nullptr;
  std::string msg;
  hca_status st = validate_params(p, msg);
  if (st != HCA_OK) return st;
  int singular = -1;
  st = validate_reps(reps, n_reps, msg, singular);
  if (st != HCA_OK) {
    fprintf(stderr, "hca_init: %s\n", msg.c_str());
    return st;
  }
  if (singular >= 0 && !states) {
    fprintf(stderr, "hca_init: replicate %d has no vessel: steady oxygen is zero\n", singular);
    return HCA_E_SINGULAR;
  }
  Ctx* c = new (std::nothrow) Ctx();
  if (!c) return HCA_E_NOMEM;
  c->prm = *p;
  c->dp = make_dev_params(*p);
  c->nreps = n_reps;
  c->use_mg = p->precond == 1;
  long long off = 0;
  for (int r = 0; r < n_reps; ++r) {
    RepHost R{};
    R.nx = reps[r].nx;
    R.ny = reps[r].ny;
    R.nz = reps[r].nz;
    R.n = (long long)R.nx * R.ny * R.nz;
    R.off = off;
    R.seed = reps[r].seed;
    off += R.n;
    c->reps.push_back(R);
  }
  c->ntot = off;
  auto bail = [&](hca_status s) {
    if (!c->err.empty()) fprintf(stderr, "hca_init: %s\n", c->err.c_str());
    free_all(c);
    delete c;
    return s;
  };
  if (hipGetDevice(&c->device) != hipSuccess) return bail(HCA_E_DEVICE);
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(HCA_E_DEVICE);
    c->own_stream = true;
  }
  if (p->graphs && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(HCA_E_DEVICE);
  if ((st = build_tables(c, reps)) != HCA_OK) return bail(st);
  if ((st = alloc_all(c)) != HCA_OK) return bail(st);
  if (c->use_mg && (st = build_mg(c)) != HCA_OK) return bail(st);
  // upload inputs and dose tables
  std::vector<double> dt((size_t)n_reps * 3 * HCA_MAX_DOSES, 0.0), da(dt.size(), 0.0);
  for (int r = 0; r < n_reps; ++r) {
    const RepHost& R = c->reps[r];
    if (hipMemcpy(c->L + R.off, reps[r].cell, (size_t)R.n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->w + R.off, reps[r].vessel_w, (size_t)R.n * 8, hipMemcpyHostToDevice) !=
            hipSuccess)
      return bail(HCA_E_DEVICE);
    for (int d = 0; d < 3; ++d) {
      const int nd = d < 2 ? reps[r].n_doses[d] : reps[r].n_doses3;
      const double* ts = d < 2 ? reps[r].dose_t_min[d] : reps[r].dose_t_min3;
      const double* as = d < 2 ? reps[r].dose_amt[d] : reps[r].dose_amt3;
      for (int k = 0; k < nd; ++k) {
        dt[(size_t)r * 3 * HCA_MAX_DOSES + d * HCA_MAX_DOSES + k] = ts[k];
        da[(size_t)r * 3 * HCA_MAX_DOSES + d * HCA_MAX_DOSES + k] = as[k];
      }
    }
  }
  if (hipMemcpy(c->dose_t, dt.data(), dt.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dose_a, da.data(), da.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
    return bail(HCA_E_DEVICE);
  long long zero = 0;
  if (hipMemcpy(c->d_step, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess)
    return bail(HCA_E_DEVICE);
  if (states) {   // resume: every replicate's state from its blob (all at one step)
    StateHeader h0{};
    if (states_on_device) {
      if (hipMemcpy(&h0, states[0], sizeof h0, hipMemcpyDeviceToHost) != hipSuccess) return bail(HCA_E_DEVICE);
    } else {
      memcpy(&h0, states[0], sizeof h0);
    }
    long long s0 = h0.step;
    if (hipMemcpy(c->d_step, &s0, sizeof s0, hipMemcpyHostToDevice) != hipSuccess)
      return bail(HCA_E_DEVICE);
    c->step = h0.step;
    launch_zero_counters(c->stream, c->d_cnt, n_reps, 1);
    launch_zero_counters(c->stream, c->d_cnt, n_reps, 0);
    for (int r = 0; r < n_reps; ++r)
      if ((st = import_state(c, r, states[r], state_bytes[r], states_on_device, false)) != HCA_OK)
        return bail(st);
    launch_stats(c->stream, c->work, c->L, c->w, c->F, c->dp.nf, c->ntot, c->P, c->Vc, c->phi,
                 c->d_cpart, c->d_cnt);
    if (hipGetLastError() != hipSuccess) return bail(HCA_E_DEVICE);
    if ((st = check_after(c)) != HCA_OK) return bail(st);
    c->last_it[0] = 0;
    for (int k = 0; k < KC_COUNT; ++k) c->prof_ms[k] = c->prof_n[k] = c->prof_bytes[k] = 0;
    *out = c;
    return HCA_OK;
  }
  if ((st = steady_oxygen(c)) != HCA_OK) return bail(st);
  launch_init_cells(c->stream, c->work, c->dp, c->L, c->K, c->P, c->Vc, c->phi);
  if (hipMemsetAsync(c->G1, 0, (size_t)c->ntot * 2 * sizeof(Real), c->stream) != hipSuccess)   // G1 and G2
    return bail(HCA_E_DEVICE);
  if (c->V && hipMemsetAsync(c->V, 0, (size_t)c->ntot * sizeof(Real), c->stream) != hipSuccess)
    return bail(HCA_E_DEVICE);
  if (c->G3 && hipMemsetAsync(c->G3, 0, (size_t)c->ntot * sizeof(Real), c->stream) != hipSuccess)
    return bail(HCA_E_DEVICE);
  if (c->Fprev && hipMemcpyAsync(c->Fprev, c->F, (size_t)c->dp.nf * c->ntot * sizeof(Real), hipMemcpyDeviceToDevice,
                                 c->stream) != hipSuccess)
    return bail(HCA_E_DEVICE);
  if (c->Fprev2 && hipMemcpyAsync(c->Fprev2, c->F, (size_t)c->dp.nf * c->ntot * sizeof(Real),
                                  hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return bail(HCA_E_DEVICE);
  launch_zero_counters(c->stream, c->d_cnt, n_reps, 1);
  launch_zero_counters(c->stream, c->d_cnt, n_reps, 0);
  launch_stats(c->stream, c->work, c->L, c->w, c->F, c->dp.nf, c->ntot, c->P, c->Vc, c->phi,
               c->d_cpart, c->d_cnt);
  if (hipGetLastError() != hipSuccess) return bail(HCA_E_DEVICE);
  if ((st = check_after(c)) != HCA_OK) return bail(st);
  c->last_it[0] = 0;
  for (int k = 0; k < KC_COUNT; ++k) c->prof_ms[k] = c->prof_n[k] = c->prof_bytes[k] = 0;
  *out = c;
  return HCA_OK;
}

}  // namespace


hca_status api_run_phases(::hca_ctx* c_, unsigned mask) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c) return HCA_E_INVALID;
  if (c->failed) return HCA_E_INVALID;
  hca_status st = run_phases(c, mask);
  if (st != HCA_OK) return st;
  return check_after(c);
}

hca_status api_step(::hca_ctx* c_, int n_steps) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c || n_steps < 0) return HCA_E_INVALID;
  if (c->failed) return HCA_E_INVALID;
  for (int k = 0; k < n_steps; ++k) {
    hca_status st = run_phases(c, HCA_PH_ALL);
    if (st != HCA_OK) return st;
  }
  return check_after(c);
}

hca_status api_fields(::hca_ctx* c_, int rep, hca_field f, void* dst, size_t dst_bytes,
                      int dst_is_device) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c || !dst) return HCA_E_INVALID;
  if (rep < 0 || rep >= c->nreps) return fail(c, HCA_E_RANGE, "replicate index out of range");
  size_t elem = 0;
  char* src = (char*)field_ptr(c, f, elem);
  if (!src) return HCA_E_INVALID;
  const RepHost& R = c->reps[rep];
  const size_t bytes = (size_t)R.n * elem;
  if (dst_bytes < bytes) return fail(c, HCA_E_RANGE, "destination buffer too small");
  if (Real* rf = real_field(c, f)) {   // stored as Real, delivered as FP64
    hca_status st = field_out(c, rf + R.off, (size_t)R.n, dst, dst_is_device);
    if (st != HCA_OK) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HCA_OK;
  }
  HIPCHK(c, hipMemcpyAsync(dst, src + (size_t)R.off * elem, bytes,
                           dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HCA_OK;
}

hca_status api_set_field(::hca_ctx* c_, int rep, hca_field f, const void* src, size_t src_bytes,
                         int src_is_device) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c || !src) return HCA_E_INVALID;
  if (rep < 0 || rep >= c->nreps) return fail(c, HCA_E_RANGE, "replicate index out of range");
  size_t elem = 0;
  char* dst = (char*)field_ptr(c, f, elem);
  if (!dst) return HCA_E_INVALID;
  const RepHost& R = c->reps[rep];
  const size_t bytes = (size_t)R.n * elem;
  if (src_bytes < bytes) return fail(c, HCA_E_RANGE, "source buffer too small");
  c->fixed_ops = false;   // the next solve rebuilds every field's c and multigrid data
  const hipMemcpyKind kind = src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (f == HCA_F_CELL) {
    // stage in the proposal buffer (rewritten by every CA pass) and validate
    HIPCHK(c, hipMemcpyAsync(c->code + R.off, src, bytes, kind, c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_bad, 0, sizeof(unsigned long long), c->stream));
    launch_validate_cells(c->stream, c->work, c->code, c->w, rep, c->d_bad);
    unsigned long long bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->d_bad, sizeof bad, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (bad) {
      c->err = "cell map has codes outside {0,1,2} or cells on vessel voxels";
      return HCA_E_INVALID;
    }
    HIPCHK(c, hipMemcpyAsync(dst + R.off, c->code + R.off, bytes, hipMemcpyDeviceToDevice,
                             c->stream));
  } else if (f == HCA_F_VESSEL_W) {
    // stage in the solver's right-hand side (rewritten by every setup) and
    // validate against the current cell map
    double* stage = reinterpret_cast<double*>(c->b);   // nf x ntot Real values: room for ntot doubles
    HIPCHK(c, hipMemcpyAsync(stage + R.off, src, bytes, kind, c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_bad, 0, sizeof(unsigned long long), c->stream));
    launch_validate_cells(c->stream, c->work, c->L, stage, rep, c->d_bad);
    unsigned long long bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->d_bad, sizeof bad, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (bad) {
      c->err = "vessel map has non-finite or negative weights or vessels on cells";
      return HCA_E_INVALID;
    }
    HIPCHK(c, hipMemcpyAsync(dst + (size_t)R.off * elem, stage + R.off, bytes, hipMemcpyDeviceToDevice,
                             c->stream));
  } else if (Real* rf = real_field(c, f)) {   // FP64 in, stored as Real
    hca_status st = field_in(c, src, (size_t)R.n, src_is_device, rf + R.off);
    if (st != HCA_OK) return st;
    // a solved field restarts its extrapolation from the new value
    if (c->Fprev) {
      const size_t off = (size_t)(rf - c->F) + (size_t)R.off;
      HIPCHK(c, hipMemcpyAsync(c->Fprev + off, c->F + off, sizeof(Real) * (size_t)R.n,
                               hipMemcpyDeviceToDevice, c->stream));
      if (c->Fprev2)
        HIPCHK(c, hipMemcpyAsync(c->Fprev2 + off, c->F + off, sizeof(Real) * (size_t)R.n,
                                 hipMemcpyDeviceToDevice, c->stream));
    }
  } else {
    HIPCHK(c, hipMemcpyAsync(dst + (size_t)R.off * elem, src, bytes, kind, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HCA_OK;
}

hca_status api_set_step(::hca_ctx* c_, int64_t step) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c || step < 0) return HCA_E_INVALID;
  long long s = step;
  HIPCHK(c, hipMemcpyAsync(c->d_step, &s, sizeof s, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->step = step;
  return HCA_OK;
}

hca_status api_state_bytes(::hca_ctx* c_, int rep, size_t* bytes) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c || !bytes) return HCA_E_INVALID;
  if (rep < 0 || rep >= c->nreps) return fail(c, HCA_E_RANGE, "replicate index out of range");
  *bytes = state_layout(context_header(c, rep)).bytes;
  return HCA_OK;
}

hca_status api_export_state(::hca_ctx* c_, int rep, void* dst, size_t dst_bytes, int dst_is_device) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c || !dst) return HCA_E_INVALID;
  if (rep < 0 || rep >= c->nreps) return fail(c, HCA_E_RANGE, "replicate index out of range");
  return export_state(c, rep, dst, dst_bytes, dst_is_device);
}

hca_status api_import_state(::hca_ctx* c_, int rep, const void* src, size_t src_bytes, int src_is_device) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c || !src) return HCA_E_INVALID;
  if (rep < 0 || rep >= c->nreps) return fail(c, HCA_E_RANGE, "replicate index out of range");
  return import_state(c, rep, src, src_bytes, src_is_device);
}

hca_status api_stats(::hca_ctx* c_, int rep, hca_stats_t* out) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c || !out) return HCA_E_INVALID;
  if (rep < 0 || rep >= c->nreps) return fail(c, HCA_E_RANGE, "replicate index out of range");
  HIPCHK(c, hipMemcpyAsync(c->h_cnt, c->d_cnt, sizeof(Counters) * c->nreps, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const Counters& k = c->h_cnt[rep];
  memset(out, 0, sizeof *out);
  out->step = c->step;
  out->n_cancer = (int64_t)k.n_cancer;
  out->n_stroma = (int64_t)k.n_stroma;
  out->n_empty = (int64_t)k.n_empty;
  out->n_vessel = (int64_t)k.n_vessel;
  out->committed = (int64_t)k.committed;
  out->divisions = (int64_t)k.divisions;
  out->kills = (int64_t)k.kills;
  out->nospace = (int64_t)k.nospace;
  out->lost = (int64_t)k.lost;
  out->total_divisions = (int64_t)k.total_divisions;
  out->total_kills = (int64_t)k.total_kills;
  if ((int)c->last_ss.size() == c->dp.nf * c->nreps) {
    for (int f = 0; f < c->dp.nf; ++f) {
      const SolveScal& s = c->last_ss[f * c->nreps + rep];
      const double rel = s.bb > 0 ? std::sqrt(s.rr / s.bb) : 0.0;
      if (f < 3) {
        out->cg_iters[f] = s.it;
        out->cg_relres[f] = rel;
      } else if (c->dp.vegf && f == c->dp.fV) {
        out->cg_iters_vegf = s.it;
        out->cg_relres_vegf = rel;
      } else {
        out->cg_iters_drug3 = s.it;
        out->cg_relres_drug3 = rel;
      }
    }
  }
  out->nonfinite = k.nonfinite ? 1 : 0;
  out->init_picard_iters = c->picard_iters;
  out->sur_voxels = (int64_t)k.sur_voxels;
  out->sur_fallbacks = (int64_t)k.sur_fallbacks;
  out->vessel_births = (int64_t)k.births;
  out->vessel_deaths = (int64_t)k.deaths;
  out->total_births = (int64_t)k.total_births;
  out->total_deaths = (int64_t)k.total_deaths;
  return HCA_OK;
}

#if HCA_RT_PRIMARY
extern "C" int hca_num_kernels(void) { return KC_COUNT; }

extern "C" const char* hca_kernel_name(int kernel) {
  if (kernel < 0 || kernel >= KC_COUNT) return "";
  return kKernelNames[kernel];
}
#endif

hca_status api_kernel_time(::hca_ctx* c_, int kernel, double* ms, int64_t* launches,
                           double* bytes_per_launch) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c || kernel < 0 || kernel >= KC_COUNT) return HCA_E_INVALID;
  prof_flush(c, nullptr, 0);
  if (ms) *ms = c->prof_ms[kernel];
  if (launches) *launches = c->prof_n[kernel];
  if (bytes_per_launch)
    *bytes_per_launch = c->prof_n[kernel] ? c->prof_bytes[kernel] / (double)c->prof_n[kernel] : 0.0;
  return HCA_OK;
}

hca_status api_set_profile(::hca_ctx* c_, int profile) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c || profile < 0 || profile >= KC_COUNT + 2) return HCA_E_INVALID;
  c->prm.profile = profile;
  return HCA_OK;
}

hca_status api_reset_kernel_time(::hca_ctx* c_) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c) return HCA_E_INVALID;
  prof_flush(c, nullptr, 0);
  for (int k = 0; k < KC_COUNT; ++k) c->prof_ms[k] = c->prof_n[k] = c->prof_bytes[k] = 0;
  return HCA_OK;
}

hca_status api_tile_shape(::hca_ctx* c_, int rep, int32_t* tx, int32_t* ty, int32_t* tz) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c || !tx || !ty || !tz) return HCA_E_INVALID;
  if (rep < 0 || rep >= c->nreps) return fail(c, HCA_E_RANGE, "replicate index out of range");
  *tx = c->reps[rep].tx;
  *ty = kBlock / c->reps[rep].tx;
  *tz = c->reps[rep].tz;
  return HCA_OK;
}

hca_status api_set_surrogate(::hca_ctx* c_, const hca_mlp* net, double margin) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c) return HCA_E_INVALID;
  if (!net) {
    c->sur_on = false;
    return HCA_OK;
  }
  auto reject = [&](const char* msg) {
    c->err = msg;
    return HCA_E_INVALID;
  };
  if (!net->theta || !std::isfinite(margin) || margin < 0.0)
    return reject("surrogate: null parameters or bad margin");
  for (int f = 0; f < HCA_MLP_NIN; ++f)
    if (!std::isfinite(net->in_mean[f]) || !std::isfinite(net->in_scale[f]) ||
        net->in_scale[f] == 0.f || std::isnan(net->in_lo[f]) || std::isnan(net->in_hi[f]))
      return reject("surrogate: bad input statistics");
  for (int o = 0; o < HCA_MLP_NOUT; ++o)
    if (!std::isfinite(net->out_mean[o]) || !std::isfinite(net->out_scale[o]) ||
        net->out_scale[o] == 0.f)
      return reject("surrogate: bad output statistics");
  if (!c->d_theta) {
    HIPCHK(c, dalloc(&c->d_theta, kMlpNparam));
    HIPCHK(c, dalloc(&c->d_pack, kPackAll));
    HIPCHK(c, dalloc(&c->d_gelu, kGeluN + 1));
    launch_mlp_gelu_table(c->stream, c->d_gelu);
  }
  HIPCHK(c, hipMemcpyAsync(c->d_theta, net->theta, sizeof(float) * kMlpNparam,
                           net->theta_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           c->stream));
  launch_mlp_pack(c->stream, c->d_theta, c->d_pack);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  MlpDev& d = c->net;
  d.packed = c->d_pack;
  d.theta = c->d_theta;
  d.gelu_tab = c->d_gelu;
  for (int f = 0; f < HCA_MLP_NIN; ++f) {
    d.in_mean[f] = net->in_mean[f];
    d.in_scale[f] = net->in_scale[f];
    d.in_lo[f] = net->in_lo[f];
    d.in_hi[f] = net->in_hi[f];
  }
  for (int o = 0; o < HCA_MLP_NOUT; ++o) {
    d.out_mean[o] = net->out_mean[o];
    d.out_scale[o] = net->out_scale[o];
  }
  d.box = net->box_check ? 1 : 0;
  d.margin = margin;
  c->sur_on = true;
  return HCA_OK;
}

hca_status api_harvest_step(::hca_ctx* c_, float* X, float* Y, int64_t cap_rows, int64_t* n_rows) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c || !X || !Y || !n_rows || cap_rows < 0) return HCA_E_INVALID;
  if (c->failed) return HCA_E_INVALID;
  *n_rows = 0;
  const Work& wk = c->work;
  hipStream_t s = c->stream;
  if (!c->before) {
    HIPCHK(c, dalloc(&c->before, 3 * (size_t)c->ntot));
    HIPCHK(c, dalloc(&c->item_cnt, (size_t)wk.nflat));
    HIPCHK(c, dalloc(&c->item_off, (size_t)wk.nflat + 1));
  }
  // rows = occupied voxels of the current map (the map changes only in the CA phase)
  launch_mlp_count(s, wk, c->L, c->item_cnt);
  launch_mlp_scan(s, wk.nflat, c->item_cnt, c->item_off);
  long long total = 0;
  HIPCHK(c, hipMemcpyAsync(&total, c->item_off + wk.nflat, sizeof total, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (total > cap_rows) return fail(c, HCA_E_RANGE, "harvest: more occupied voxels than cap_rows");
  hca_status st = run_phases(c, HCA_PH_O2 | HCA_PH_DRUGS | HCA_PH_VEGF);
  if (st != HCA_OK) return st;
  launch_mlp_save_state(s, wk, c->P, c->Vc, c->phi, c->before);
  {
    double fin_bpv;   // none: the solves above ran without the ODE phase
    const CgFinish<Real>* fin = take_finish(c, fin_bpv);
    ProfScope ps(c, KC_ODE, kTagState, true, fin_bpv);
    launch_ode(s, wk, c->dp, c->L, c->K, c->P, c->Vc, c->phi, fin);
  }
  launch_mlp_harvest(s, wk, c->dp, c->L, c->K, c->G1, c->G2, c->P, c->Vc, c->before, c->item_off,
                     X, Y);
  st = run_phases(c, HCA_PH_CA | HCA_PH_STATS | HCA_PH_ADVANCE);
  if (st != HCA_OK) return st;
  st = check_after(c);
  if (st != HCA_OK) return st;
  *n_rows = total;
  return HCA_OK;
}

hca_status api_synchronize(::hca_ctx* c_) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c) return HCA_E_INVALID;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HCA_OK;
}

const char* api_last_error(const ::hca_ctx* c_) {
  const Ctx* c = static_cast<const Ctx*>(c_);
  return c ? c->err.c_str() : "";
}

void api_destroy(::hca_ctx* c_) {
  Ctx* c = static_cast<Ctx*>(c_);
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
}

}  // namespace HCA_RT_NS
}  // namespace hca
