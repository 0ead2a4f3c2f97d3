// Matrix-free preconditioned conjugate gradient for the implicit-Euler
// systems of Eqs. (oxygen) and (chemo) on the voxel lattice:
//
//     (A u)_i = c_i u_i - a (Lap u)_i = b_i,    a = D/h^2,
//
// Lap the 7-point Laplacian with zero-flux faces (a missing neighbour is
// dropped), A a symmetric M-matrix.  The paper solves the same SPD systems
// with CG (chemotherapy, linearised oxygen).  Here every replicate of the
// batch runs its own CG in the same launches: each workgroup stores its
// partial dot products, and a one-workgroup-per-replicate reduce kernel sums
// them in a fixed order and advances the replicate's scalars.  A finished
// replicate's workgroups return at once.
//
// Iteration (flexible CG, Polak-Ribiere beta, so a varying preconditioner is
// allowed):
//   start:  r = b - A x,  z = M r,  p = z
//   loop:   q = A p,  alpha = r.z / p.q,  x += alpha p,  r -= alpha q,
//           stop if ||r|| <= rtol ||b||,
//           z' = M r,  beta = (r.z' - r.z_old) / r.z,  p = z' + beta p
// The direction update p = z + beta p is fused into the next A p: each
// workgroup forms p at its voxels and their neighbours from z and the
// previous p (double-buffered p, so no workgroup overwrites a value another
// still reads).  Nothing in the iteration reads x, so x += alpha p is made
// one iteration late, by the next apply, which reads the previous p anyway
// (x moves once per iteration instead of x and p in the update); the last
// iteration's update is made by a finishing pass after the solve.
#include "dev_util.h"

namespace hca {

struct TileCoord {
  int rep;
  int x, y, z0, z1;
  bool valid;
  int nx, ny, nz;
  long long off;
  double a;
  int x0, y0, tx, ty, lx, ly;   // tile origin and shape, thread position in it
};

__device__ inline TileCoord tile_coord(const Work& w, int ti) {
  const Tile t = w.tiles[ti];
  const RepDev rp = w.reps[t.rep];
  TileCoord tc;
  tc.rep = t.rep;
  tc.tx = rp.tx;
  tc.ty = kBlock / rp.tx;
  tc.lx = (int)(threadIdx.x % rp.tx);
  tc.ly = (int)(threadIdx.x / rp.tx);
  tc.x0 = t.x0;
  tc.y0 = t.y0;
  tc.x = t.x0 + tc.lx;
  tc.y = t.y0 + tc.ly;
  tc.z0 = t.z0;
  tc.z1 = t.z1;
  tc.nx = rp.nx;
  tc.ny = rp.ny;
  tc.nz = rp.nz;
  tc.off = rp.off;
  tc.a = rp.a;
  tc.valid = tc.x < rp.nx && tc.y < rp.ny;
  return tc;
}

// LDS plane of one tile with a one-cell frame: (tx + 2) (256/tx + 2) values,
// at most 66 x 6 (tx = 64).
constexpr int kPlaneMax = 400;

// Planes whose global loads are issued ahead of the plane being stored to
// LDS (the ring depth of plane_stencil).  One, i.e. plane z+2's operand and c
// in flight while plane z is computed, measured fastest for the CG kernels:
// deeper rings hold more registers (fewer resident waves) and measured slower.
constexpr int kStencilPrefetch = 1;

// Marches the tile over [z0, z1) and calls f(i, deg, u_i, (A u)_i) for every
// voxel of the tile inside the lattice, where u = op.value(op.load(j)) is the
// operand (possibly formed on the fly from several arrays) and
// (A u)_i = (c_i + a deg) u_i - a sum_nb u_j.  Values the op needs at the
// voxel itself only (op.load_ctr, prefetched with the plane like c) are
// handed, with the voxel's raw operand, to op.at_center(i, raw_i, extra_i)
// when the voxel's plane enters LDS.  Each plane of u, with its x/y
// frame, is formed once into LDS (double buffered); outside the lattice the
// frame holds 0, which adds nothing to the neighbour sum.  Software
// pipelined: the global loads (operand and c) of planes z+2 .. z+1+PD are in
// flight while plane z is computed, in a ring of registers (the z loop is
// unrolled by PD so every ring slot is a fixed register), so their latency
// overlaps the compute and the barrier.  Called by the whole workgroup.
//
// T is the storage type of the fields (double, or float in precision 32):
// the operand is rounded to T once (into LDS, and for a neighbour read from
// global memory), so every tile sees the same value at a voxel; the stencil
// arithmetic is FP64 in both.
template <int PD, typename T, typename OP, typename F>
__device__ inline void plane_stencil(const TileCoord& tc, const T* __restrict__ c,
                                     T (*lds)[kPlaneMax], const OP& op, F f) {
  using Raw = typename OP::Raw;
  using Ctr = typename OP::Ctr;
  struct Slot {
    Raw ri, rf;   // operand of the thread's cell and of its frame cell
    double c;     // c of the thread's cell
    Ctr e;        // the op's extra values at the thread's cell
  };
  const double a = tc.a;
  const int W = tc.tx + 2;
  const int o = (tc.ly + 1) * W + tc.lx + 1;
  const int nframe = 2 * W + 2 * tc.ty;
  const long long plane = (long long)tc.nx * tc.ny;
  // this thread's frame cell (at most one: nframe <= 256)
  const int k = threadIdx.x;
  const bool has_frame = k < nframe;
  int hx = 0, hy = 0;
  if (k < W) {
    hx = k;
    hy = 0;
  } else if (k < 2 * W) {
    hx = k - W;
    hy = tc.ty + 1;
  } else if (k < 2 * W + tc.ty) {
    hx = 0;
    hy = 1 + k - 2 * W;
  } else {
    hx = W - 1;
    hy = 1 + k - 2 * W - tc.ty;
  }
  const int gx = tc.x0 + hx - 1, gy = tc.y0 + hy - 1;
  const bool fin = has_frame && gx >= 0 && gx < tc.nx && gy >= 0 && gy < tc.ny;
  const int fo = hy * W + hx;
  const long long fidx = fin ? gx + (long long)tc.nx * gy : 0;
  const long long iidx = tc.x + (long long)tc.nx * tc.y;
  const int z0 = tc.z0, z1 = tc.z1;
  // plane zp into a slot; planes beyond z1 are never needed, and the plane
  // z1 only as the +z neighbour (no c)
  auto load_slot = [&](Slot& sl, int zp) {
    const long long pz = tc.off + plane * zp;
    if (tc.valid) sl.ri = op.load(pz + iidx);
    if (tc.valid && zp < z1) {
      sl.c = c[pz + iidx];
      sl.e = op.load_ctr(pz + iidx);
    }
    if (fin) sl.rf = op.load(pz + fidx);
  };
  auto store_slot = [&](const Slot& sl, T* buf) {
    buf[o] = tc.valid ? (T)op.value(sl.ri) : (T)0;
    if (has_frame) buf[fo] = fin ? (T)op.value(sl.rf) : (T)0;
  };
  const bool xl = tc.x > 0, xr = tc.x + 1 < tc.nx, yl = tc.y > 0, yr = tc.y + 1 < tc.ny;
  const int deg_xy = (int)xl + (int)xr + (int)yl + (int)yr;
  long long i = tc.off + iidx + plane * z0;
  T* cur = lds[0];
  T* nxt = lds[1];
  // ring: plane zp (z0 < zp <= min(z1, nz - 1)) in slot (zp - z0 - 1) % PD
  Slot ring[PD];
#pragma unroll
  for (int d = 0; d < PD; ++d) ring[d] = Slot{op.zero(), op.zero(), 0.0, op.ctr_zero()};
  __syncthreads();   // the previous tile's readers are done with both buffers
  double um, cc;
  {
    Slot s0{op.zero(), op.zero(), 0.0, op.ctr_zero()};
    load_slot(s0, z0);
    if (tc.valid) op.at_center(i, s0.ri, s0.e);
    um = (tc.valid && z0 > 0) ? (double)(T)op.value(op.load(i - plane)) : 0.0;
#pragma unroll
    for (int d = 0; d < PD; ++d)
      if (z0 + 1 + d <= z1 && z0 + 1 + d < tc.nz) load_slot(ring[d], z0 + 1 + d);
    cc = s0.c;
    store_slot(s0, cur);
  }
  __syncthreads();
  double uc = cur[o];
  for (int zb = z0; zb < z1; zb += PD) {
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      const int z = zb + d;
      if (z < z1) {   // uniform over the workgroup
        const bool zl = z > 0, zr = z + 1 < tc.nz;
        double cn = 0.0;
        if (zr) {   // plane z+1 into LDS; its slot then takes plane z+1+PD
          store_slot(ring[d], nxt);
          cn = ring[d].c;
          if (tc.valid && z + 1 < z1) op.at_center(i + plane, ring[d].ri, ring[d].e);
          const int zq = z + 1 + PD;
          if (zq <= z1 && zq < tc.nz) load_slot(ring[d], zq);
        }
        double s = cur[o - 1];
        s += (double)cur[o + 1];
        s += (double)cur[o - W];
        s += (double)cur[o + W];
        __syncthreads();
        const double up = zr ? (double)nxt[o] : 0.0;
        s += um;
        s += up;
        if (tc.valid) {
          const int deg = deg_xy + (int)zl + (int)zr;
          const double Au = (cc + a * deg) * uc - a * s;
          f(i, deg, uc, Au);
        }
        um = uc;
        uc = up;
        cc = cn;
        T* t = cur;
        cur = nxt;
        nxt = t;
        i += plane;
      }
    }
  }
}

// Operands of the stencil: the iterate x (start), and p = z + beta p_old
// formed on the fly (apply; z FP64 for Jacobi, the multigrid's FP32 result
// otherwise).
template <typename T>
struct OpX {
  struct Raw {
    double x;
  };
  struct Ctr {};
  const T* __restrict__ x;
  __device__ inline Raw zero() const { return Raw{0.0}; }
  __device__ inline Raw load(long long j) const { return Raw{x[j]}; }
  __device__ inline double value(const Raw& r) const { return r.x; }
  __device__ inline Ctr ctr_zero() const { return Ctr{}; }
  __device__ inline Ctr load_ctr(long long) const { return Ctr{}; }
  __device__ inline void at_center(long long, const Raw&, const Ctr&) const {}
};

// The voxel's own x comes with it (extra) when the previous iteration's
// x += alpha p_old is due (every iteration but a solve's first; alpha the
// previous iteration's), made as the voxel's plane enters LDS.
template <bool JAC, typename T>
struct OpP {
  struct Raw {
    double z, p;
  };
  struct Ctr {
    double x;
  };
  const T* __restrict__ z;
  const float* __restrict__ z32;
  const T* __restrict__ pold;
  T* __restrict__ x;
  double beta;
  double isc;   // multigrid: z = z32 / sc
  double alpha;
  bool first;
  __device__ inline Raw zero() const { return Raw{0.0, 0.0}; }
  __device__ inline Ctr ctr_zero() const { return Ctr{0.0}; }
  __device__ inline Ctr load_ctr(long long j) const { return Ctr{first ? 0.0 : (double)x[j]}; }
  __device__ inline void at_center(long long i, const Raw& r, const Ctr& e) const {
    if (!first) x[i] = (T)(e.x + alpha * r.p);
  }
  __device__ inline Raw load(long long j) const {
    Raw r;
    if constexpr (JAC)
      r.z = z[j];
    else
      r.z = (double)z32[j] * isc;
    r.p = first ? 0.0 : pold[j];
    return r;
  }
  __device__ inline double value(const Raw& r) const { return first ? r.z : r.z + beta * r.p; }
};

// r = b - A x; Jacobi mode also Dinv = 1/diag(A), z = Dinv r.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_cg_start(Work w, const T* __restrict__ c,
                                                     const T* __restrict__ b,
                                                     const T* __restrict__ x,
                                                     SolverBufsT<T> sb) {
  __shared__ double lds4[4];
  __shared__ T lds[2][kPlaneMax];
  int t0, t1;
  tile_range(w.ntiles, t0, t1);
  for (int ti = t0; ti < t1; ++ti) {
    const TileCoord tc = tile_coord(w, ti);
    const double a = tc.a;
    double bb = 0.0, rr = 0.0, rz = 0.0;
    {
      plane_stencil<kStencilPrefetch>(tc, c, lds, OpX<T>{x},
                     [&](long long i, int deg, double, double Ax) {
                       const double bi = b[i];
                       const double r = (double)(T)(bi - Ax);
                       sb.r[i] = (T)r;
                       bb += bi * bi;
                       rr += r * r;
                       if (sb.jacobi) {
                         const double di = (double)(T)(1.0 / ((double)c[i] + a * deg));
                         const double zz = (double)(T)(r * di);
                         sb.dinv[i] = (T)di;
                         sb.z[i] = (T)zz;
                         rz += r * zz;
                       }
                     });
    }
    bb = block_sum(bb, lds4);
    rr = block_sum(rr, lds4);
    rz = block_sum(rz, lds4);
    store_partials(sb.partial + (size_t)ti * 3, bb, rr, rz);
  }
}

// p_new = z + beta p_old (p_new = z on the first iteration), q = A p_new;
// and the previous iteration's x += alpha p_old (not on the first).
template <bool JAC, typename T>
__global__ void __launch_bounds__(kBlock) k_cg_apply(Work w, const T* __restrict__ c,
                                                     const T* __restrict__ z,
                                                     const T* __restrict__ pold,
                                                     T* __restrict__ pnew,
                                                     T* __restrict__ q, T* __restrict__ x,
                                                     SolverBufsT<T> sb) {
  __shared__ double lds4[4];
  __shared__ T lds[2][kPlaneMax];
  int t0, t1;
  tile_range(w.ntiles, t0, t1);
  for (int ti = t0; ti < t1; ++ti) {
    const TileCoord tc = tile_coord(w, ti);
    const SolveScal* ssr = sb.ss + tc.rep;
    if (ssr->done) continue;
    const double beta = ssr->beta;
    const bool first = ssr->first != 0;
    double pq = 0.0;
    {
      // ss.alpha is still the previous iteration's (this apply's reduce sets the next)
      const OpP<JAC, T> op{z, sb.z32, pold, x, beta, ssr->isc, ssr->alpha, first};
      plane_stencil<kStencilPrefetch>(tc, c, lds, op, [&](long long i, int, double pc, double Ap) {
        const T qi = (T)Ap;
        pnew[i] = (T)pc;
        q[i] = qi;
        pq += pc * (double)qi;
      });
    }
    pq = block_sum(pq, lds4);
    store_partials(sb.partial + (size_t)ti * 3, pq, 0.0, 0.0);
  }
}

// r -= alpha q; partials of r.r, r.z_old and (Jacobi) r.z'.  (x += alpha p
// is made by the next apply, or by k_cg_finish after the last iteration.)
template <bool JAC, typename T>
__global__ void __launch_bounds__(kBlock) k_cg_update(Work w, const T* __restrict__ q, SolverBufsT<T> sb) {
  __shared__ double lds4[4];
  constexpr bool jac = JAC;
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    const SolveScal* ssr = sb.ss + fb.rep;
    if (ssr->done) continue;
    const long long off = w.reps[fb.rep].off;
    const double alpha = ssr->alpha;
    const double sc = ssr->sc, isc_prev = ssr->isc_prev;
    double rr = 0.0, rzo = 0.0, rzn = 0.0;
    // kUpd voxels per thread per trip, every load issued before any use, so
    // enough bytes are in flight per CU to stream at HBM rate on long items
    constexpr int kUpd = 4;
    const long long end = off + fb.end;
    for (long long i0 = off + fb.begin + threadIdx.x; i0 < end; i0 += kUpd * kBlock) {
      double rv[kUpd], qv[kUpd], zo[kUpd], dv[kUpd];
#pragma unroll
      for (int u = 0; u < kUpd; ++u) {
        const long long i = i0 + (long long)u * kBlock;
        if (i < end) {
          rv[u] = sb.r[i];
          qv[u] = q[i];
          zo[u] = jac ? (double)sb.z[i] : (double)sb.z32[i] * isc_prev;
          dv[u] = jac ? (double)sb.dinv[i] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < kUpd; ++u) {
        const long long i = i0 + (long long)u * kBlock;
        if (i >= end) continue;
        const double r = (double)(T)(rv[u] - alpha * qv[u]);
        sb.r[i] = (T)r;
        if (!jac) sb.r32[i] = (float)(r * sc);   // the multigrid's scaled copy
        rr += r * r;
        rzo += r * zo[u];
        if (jac) {
          const double znew = (double)(T)(r * dv[u]);
          sb.z[i] = (T)znew;
          rzn += r * znew;
        }
      }
    }
    rr = block_sum(rr, lds4);
    rzo = block_sum(rzo, lds4);
    rzn = block_sum(rzn, lds4);
    store_partials(sb.partial + (size_t)it * 3, rr, rzo, rzn);
  }
}

// The last iteration's x += alpha p of every system that iterated (the
// earlier iterations' were made by the applies that followed them).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_cg_finish(Work w, T* __restrict__ x, SolverBufsT<T> sb) {
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    const SolveScal* ssr = sb.ss + fb.rep;
    const int n = ssr->it;
    if (n == 0) continue;
    const T* __restrict__ p = ((n - 1) & 1) ? sb.p0 : sb.p1;   // the direction of iteration n - 1
    const double alpha = ssr->alpha;
    const long long off = w.reps[fb.rep].off;
    for (long long i = off + fb.begin + threadIdx.x; i < off + fb.end; i += kBlock)
      x[i] = (T)fma(alpha, (double)p[i], (double)x[i]);
  }
}

// ---- the solves' initial guess from their previous solutions ---------------
//
// x1 is the field's value (its last solve's solution), x2 and x3 the two
// solutions before.  Candidates: the least-squares fits
//     x_f3 = c1 x1 + c2 (x1 - x2) + c3 (x2 - x3),   x_f2 = c1 x1 + c2 (x1 - x2),
// the coefficients minimising ||b - A x|| for this solve's system (normal
// equations in u = A x1, w1 = A (x1 - x2), w2 = A (x2 - x3)), and the
// geometric extrapolation x_g (the per-voxel rule of k_extrapolate).  The
// candidate with the smallest residual norm, ||b||^2 - 2 b.y + y.y from the
// same products, is taken.  A drug field's operator is the same from step to
// step and its solutions follow a smooth course in time, so b lies close to
// the span of A x1 and the differences; once a field decays geometrically
// voxel by voxel, x_g can do better.  The differences are formed per voxel
// before the operator is applied, so nearly equal solutions do not cancel
// in A x1 - A x2.
__device__ inline double geo_guess(double u, double up) {
  return (up > 0.0 && u > 0.0 && u < up) ? u * (u / up) : u;
}

// plane_stencil for NC operands at once: f(i, Au) with Au[k] = (A v_k)_i,
// v the operand values op.values(op.load(j), v) (rounded to T once, as in
// plane_stencil); the same marching, frame and one-plane prefetch.
template <int NC, typename T, typename OP, typename F>
__device__ inline void plane_stencil_n(const TileCoord& tc, const T* __restrict__ c,
                                       T (*lds)[NC][kPlaneMax], const OP& op, F f) {
  using Raw = typename OP::Raw;
  struct Slot {
    Raw ri, rf;
    double c;
  };
  const double a = tc.a;
  const int W = tc.tx + 2;
  const int o = (tc.ly + 1) * W + tc.lx + 1;
  const int nframe = 2 * W + 2 * tc.ty;
  const long long plane = (long long)tc.nx * tc.ny;
  const int k = threadIdx.x;
  const bool has_frame = k < nframe;
  int hx = 0, hy = 0;
  if (k < W) {
    hx = k;
  } else if (k < 2 * W) {
    hx = k - W;
    hy = tc.ty + 1;
  } else if (k < 2 * W + tc.ty) {
    hy = 1 + k - 2 * W;
  } else {
    hx = W - 1;
    hy = 1 + k - 2 * W - tc.ty;
  }
  const int gx = tc.x0 + hx - 1, gy = tc.y0 + hy - 1;
  const bool fin = has_frame && gx >= 0 && gx < tc.nx && gy >= 0 && gy < tc.ny;
  const int fo = hy * W + hx;
  const long long fidx = fin ? gx + (long long)tc.nx * gy : 0;
  const long long iidx = tc.x + (long long)tc.nx * tc.y;
  const int z0 = tc.z0, z1 = tc.z1;
  auto load_slot = [&](Slot& sl, int zp) {
    const long long pz = tc.off + plane * zp;
    if (tc.valid) sl.ri = op.load(pz + iidx);
    if (tc.valid && zp < z1) sl.c = c[pz + iidx];
    if (fin) sl.rf = op.load(pz + fidx);
  };
  auto store_slot = [&](const Slot& sl, T (*buf)[kPlaneMax]) {
    double v[NC], vf[NC];
    op.values(sl.ri, v);
    op.values(sl.rf, vf);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      buf[q][o] = tc.valid ? (T)v[q] : (T)0;
      if (has_frame) buf[q][fo] = fin ? (T)vf[q] : (T)0;
    }
  };
  const bool xl = tc.x > 0, xr = tc.x + 1 < tc.nx, yl = tc.y > 0, yr = tc.y + 1 < tc.ny;
  const int deg_xy = (int)xl + (int)xr + (int)yl + (int)yr;
  long long i = tc.off + iidx + plane * z0;
  int cur = 0;
  Slot ring{op.zero(), op.zero(), 0.0};
  __syncthreads();   // the previous tile's readers are done with both buffers
  double um[NC], uc[NC], cc;
  {
    Slot s0{op.zero(), op.zero(), 0.0};
    load_slot(s0, z0);
    double v[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) v[q] = 0.0;
    if (tc.valid && z0 > 0) op.values(op.load(i - plane), v);
#pragma unroll
    for (int q = 0; q < NC; ++q) um[q] = (double)(T)v[q];
    if (z0 + 1 <= z1 && z0 + 1 < tc.nz) load_slot(ring, z0 + 1);
    cc = s0.c;
    store_slot(s0, lds[0]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NC; ++q) uc[q] = lds[0][q][o];
  for (int z = z0; z < z1; ++z) {
    const bool zl = z > 0, zr = z + 1 < tc.nz;
    const int nx = cur ^ 1;
    double cn = 0.0;
    if (zr) {   // plane z+1 into LDS; the slot then takes plane z+2
      store_slot(ring, lds[nx]);
      cn = ring.c;
      if (z + 2 <= z1 && z + 2 < tc.nz) load_slot(ring, z + 2);
    }
    double s[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q)
      s[q] = (((double)lds[cur][q][o - 1] + (double)lds[cur][q][o + 1]) + (double)lds[cur][q][o - W]) +
             (double)lds[cur][q][o + W];
    __syncthreads();
    double up[NC], Au[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) up[q] = zr ? (double)lds[nx][q][o] : 0.0;
    if (tc.valid) {
      const int deg = deg_xy + (int)zl + (int)zr;
#pragma unroll
      for (int q = 0; q < NC; ++q) Au[q] = (cc + a * deg) * uc[q] - a * ((s[q] + um[q]) + up[q]);
      f(i, Au);
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      um[q] = uc[q];
      uc[q] = up[q];
    }
    cc = cn;
    cur = nx;
    i += plane;
  }
}

template <typename T>
struct OpHist {   // x1, x1 - x2, x2 - x3, x_g per voxel
  struct Raw {
    double x1, x2, x3;
  };
  const T* __restrict__ p1;
  const T* __restrict__ p2;
  const T* __restrict__ p3;
  __device__ inline Raw zero() const { return Raw{0.0, 0.0, 0.0}; }
  __device__ inline Raw load(long long j) const { return Raw{p1[j], p2[j], p3[j]}; }
  __device__ inline void values(const Raw& r, double (&v)[4]) const {
    v[0] = r.x1;
    v[1] = r.x1 - r.x2;
    v[2] = r.x2 - r.x3;
    v[3] = geo_guess(r.x1, r.x2);
  }
};

// Products per tile, in the order of kGuessPartsPerTile: u.u, u.w1, u.w2,
// w1.w1, w1.w2, w2.w2, b.u, b.w1, b.w2, b.b, b.g, g.g.
template <typename T>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) k_guess_dots(Work w, const T* __restrict__ c, const T* __restrict__ b,
                                                       const T* __restrict__ x1, const T* __restrict__ x2,
                                                       const T* __restrict__ x3, double* __restrict__ part,
                                                       unsigned fmask, int nrep) {
  __shared__ double lds4[4];
  __shared__ T lds[2][4][kPlaneMax];
  int t0, t1;
  tile_range(w.ntiles, t0, t1);
  for (int ti = t0; ti < t1; ++ti) {
    const TileCoord tc = tile_coord(w, ti);
    if (!((fmask >> (tc.rep / nrep)) & 1u)) continue;
    double d[kGuessPartsPerTile] = {};
    plane_stencil_n<4>(tc, c, lds, OpHist<T>{x1, x2, x3}, [&](long long i, const double (&A)[4]) {
      const double u = A[0], w1 = A[1], w2 = A[2], g = A[3], bi = b[i];
      d[0] += u * u;
      d[1] += u * w1;
      d[2] += u * w2;
      d[3] += w1 * w1;
      d[4] += w1 * w2;
      d[5] += w2 * w2;
      d[6] += bi * u;
      d[7] += bi * w1;
      d[8] += bi * w2;
      d[9] += bi * bi;
      d[10] += bi * g;
      d[11] += g * g;
    });
#pragma unroll
    for (int q = 0; q < kGuessPartsPerTile; ++q) d[q] = block_sum(d[q], lds4);
    if (threadIdx.x == 0) {
      double* o = part + (size_t)ti * kGuessPartsPerTile;
#pragma unroll
      for (int q = 0; q < kGuessPartsPerTile; ++q) o[q] = d[q];
    }
  }
}

// Least squares in the first n of the basis images (n = 1, 2, 3): the normal
// equations G c = r scaled to a unit diagonal and solved by Cholesky; false
// if a pivot is not well above 0 (the vectors nearly dependent).
__device__ inline bool ls_fit(const double (&G)[3][3], const double (&r)[3], int n, double (&cf)[3]) {
  double D[3], S[3][3], y[3];
  for (int p = 0; p < n; ++p) {
    if (!(G[p][p] > 0.0)) return false;
    D[p] = 1.0 / sqrt(G[p][p]);
  }
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) S[p][q] = G[p][q] * D[p] * D[q];
  double Lm[3][3] = {};
  for (int p = 0; p < n; ++p) {   // S = L L^T
    double dd = S[p][p];
    for (int k = 0; k < p; ++k) dd -= Lm[p][k] * Lm[p][k];
    if (!(dd > 1e-12)) return false;
    Lm[p][p] = sqrt(dd);
    for (int q = p + 1; q < n; ++q) {
      double v = S[q][p];
      for (int k = 0; k < p; ++k) v -= Lm[q][k] * Lm[p][k];
      Lm[q][p] = v / Lm[p][p];
    }
  }
  for (int p = 0; p < n; ++p) {   // L y = D r
    double v = r[p] * D[p];
    for (int k = 0; k < p; ++k) v -= Lm[p][k] * y[k];
    y[p] = v / Lm[p][p];
  }
  for (int p = n - 1; p >= 0; --p) {   // L^T z = y, c = D z
    double v = y[p];
    for (int k = p + 1; k < n; ++k) v -= Lm[k][p] * cf[k];
    cf[p] = v / Lm[p][p];
  }
  for (int p = 0; p < n; ++p) cf[p] *= D[p];
  for (int p = n; p < 3; ++p) cf[p] = 0.0;
  for (int p = 0; p < n; ++p)
    if (!isfinite(cf[p])) return false;
  return true;
}

// One workgroup per system: the tiles' products summed in a fixed order, the
// candidates' coefficients and residual norms, and the choice:
// alpha[4 s] = 1 for x_g, else 0; alpha[4 s + 1 .. 3] = (c1, c2, c3).
__global__ void __launch_bounds__(kBlock) k_guess_reduce(Work w, const double* __restrict__ part,
                                                         double* __restrict__ alpha, unsigned fmask,
                                                         int nrep) {
  __shared__ double lds4[4];
  const int rep = blockIdx.x;
  if (!((fmask >> (rep / nrep)) & 1u)) return;
  const RepDev rp = w.reps[rep];
  double t[kGuessPartsPerTile];
#pragma unroll
  for (int k = 0; k < kGuessPartsPerTile; ++k) {
    double s = 0.0;
    for (int j = threadIdx.x; j < rp.tile_nb; j += kBlock)
      s += part[(size_t)(rp.tile_b0 + j) * kGuessPartsPerTile + k];
    t[k] = block_sum(s, lds4);
  }
  if (threadIdx.x != 0) return;
  const double G[3][3] = {{t[0], t[1], t[2]}, {t[1], t[3], t[4]}, {t[2], t[4], t[5]}};
  const double r[3] = {t[6], t[7], t[8]};
  const double bb = t[9], bg = t[10], gg = t[11];
  auto resid = [&](const double (&cf)[3]) {
    double q = bb;
    for (int p = 0; p < 3; ++p) {
      q -= 2.0 * cf[p] * r[p];
      for (int k = 0; k < 3; ++k) q += cf[p] * G[p][k] * cf[k];
    }
    return q;
  };
  double best[3] = {1.0, 0.0, 0.0};   // x1 alone (also when x1 = 0)
  double rbest = resid(best);
  for (int n = 1; n <= 3; ++n) {
    double cf[3];
    if (ls_fit(G, r, n, cf)) {
      const double q = resid(cf);
      if (isfinite(q) && q < rbest) {
        rbest = q;
        for (int p = 0; p < 3; ++p) best[p] = cf[p];
      }
    }
  }
  const double rg = bb - 2.0 * bg + gg;
  alpha[4 * rep] = (isfinite(rg) && rg < rbest) ? 1.0 : 0.0;
  alpha[4 * rep + 1] = best[0];
  alpha[4 * rep + 2] = best[1];
  alpha[4 * rep + 3] = best[2];
}

// F <- the chosen candidate, Fprev2 <- Fprev, Fprev <- F (the systems of the
// fields in fmask).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_guess_apply(Work w, T* __restrict__ F, T* __restrict__ Fprev,
                                                        T* __restrict__ Fprev2, const double* __restrict__ alpha,
                                                        unsigned fmask, int nrep, int rotate) {
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    if (!((fmask >> (fb.rep / nrep)) & 1u)) continue;
    const bool geo = alpha[4 * fb.rep] != 0.0;
    const double c1 = alpha[4 * fb.rep + 1], c2 = alpha[4 * fb.rep + 2], c3 = alpha[4 * fb.rep + 3];
    const long long off = w.reps[fb.rep].off;
    for (long long i = off + fb.begin + threadIdx.x; i < off + fb.end; i += kBlock) {
      const double u1 = F[i], u2 = Fprev[i], u3 = Fprev2[i];
      F[i] = (T)(geo ? geo_guess(u1, u2)
                     : c1 * u1 + c2 * (double)(T)(u1 - u2) + c3 * (double)(T)(u2 - u3));
      if (rotate) {   // u3 is not needed again: its buffer takes u1 and the roles swap
        Fprev2[i] = (T)u1;
      } else {
        Fprev2[i] = (T)u2;
        Fprev[i] = (T)u1;
      }
    }
  }
}

template <typename T>
void launch_guess_projection(hipStream_t s, const Work& w, const T* c, const T* b, T* F, T* Fprev, T* Fprev2,
                             double* part, double* alpha, unsigned fmask, int nrep, int rotate) {
  hca_launch(k_guess_dots<T>, dim3(grid_tiles(w.ntiles, w.max_blocks)), dim3(kBlock), 0, s, w, c, b,
             (const T*)F, (const T*)Fprev, (const T*)Fprev2, part, fmask, nrep);
  hca_launch(k_guess_reduce, dim3(w.nreps), dim3(kBlock), 0, s, w, (const double*)part, alpha, fmask, nrep);
  hca_launch(k_guess_apply<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, F, Fprev, Fprev2,
             (const double*)alpha, fmask, nrep, rotate);
}

// Power of two near 1/rms(r) for a system of n unknowns with ||r||^2 = rr
// (1 when rr is 0 or not finite).
__device__ inline double residual_scale(double rr, long long n) {
  if (!(rr > 0.0) || !isfinite(rr)) return 1.0;
  return exp2(-rint(0.5 * log2(rr / (double)n)));
}

// r32 = r sc of the systems still iterating (after the start reduce).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_cg_r32(Work w, SolverBufsT<T> sb) {
  int b0, b1;
  work_range(w.nflat, b0, b1);
  for (int it = b0; it < b1; ++it) {
    const FlatBlk fb = w.flat[it];
    const SolveScal* ssr = sb.ss + fb.rep;
    if (ssr->done) continue;
    const long long off = w.reps[fb.rep].off;
    const double sc = ssr->sc;
    for (long long i = off + fb.begin + threadIdx.x; i < off + fb.end; i += kBlock)
      sb.r32[i] = (float)((double)sb.r[i] * sc);
  }
}

// Fixed-order sum of component k of the partials [b0, b0 + nb).
__device__ inline double sum_partials(const double* partial, int b0, int nb, int k, double* lds4) {
  double s = 0.0;
  for (int j = threadIdx.x; j < nb; j += kBlock) s += partial[(size_t)(b0 + j) * 3 + k];
  return block_sum(s, lds4);
}

// One workgroup per replicate: finish the reduction of the preceding kernel
// and advance the replicate's CG scalars.
template <int KIND, typename T>
__global__ void __launch_bounds__(kBlock) k_cg_reduce(Work w, SolverBufsT<T> sb, double rtol, int maxit,
                                                      unsigned fmask, int nrep) {
  __shared__ double lds4[4];
  const int rep = blockIdx.x;
  SolveScal& s = sb.ss[rep];
  if (KIND != RED_START && s.done) return;
  if (KIND == RED_START && !((fmask >> (rep / nrep)) & 1u)) {   // field not requested
    if (threadIdx.x == 0) {
      s.it = 0;
      s.rr = s.bb = 0.0;
      s.conv = 1;
      s.done = 1;
      atomicAdd(sb.ndone, 1);
    }
    return;
  }
  const RepDev rp = w.reps[rep];
  const bool tiles = KIND != RED_UPDATE;
  const int b0 = KIND == RED_RZF ? rp.ftile_b0 : tiles ? rp.tile_b0 : rp.flat_b0;
  const int nb = KIND == RED_RZF ? rp.ftile_nb : tiles ? rp.tile_nb : rp.flat_nb;
  const double t0 = sum_partials(sb.partial, b0, nb, 0, lds4);
  const double t1 = (KIND == RED_START || KIND == RED_UPDATE) ? sum_partials(sb.partial, b0, nb, 1, lds4) : 0.0;
  const double t2 = (KIND == RED_START || KIND == RED_UPDATE) ? sum_partials(sb.partial, b0, nb, 2, lds4) : 0.0;
  if (threadIdx.x != 0) return;
  if (KIND == RED_START) {
    s.bb = t0;
    s.rr = t1;
    s.rr0 = t1;
    s.rz = t2;
    s.rzn = t2;
    s.rzo = 0.0;
    s.beta = 0.0;
    s.alpha = 0.0;
    s.pq = 0.0;
    s.it = 0;
    s.first = 1;
    s.sc = residual_scale(t1, rp.n);
    s.isc = 1.0 / s.sc;
    s.isc_prev = s.isc;
    // A right-hand side with ||b||^2 < 1e-280 (a drug field hundreds of steps
    // after its last dose) counts as solved by the initial guess: its squared
    // norms would leave FP64's normal range, and no result depends on a field
    // that small (a kill probability of it is exactly 0).
    const bool conv = t1 <= rtol * rtol * t0 || t0 < 1e-280;
    const bool bad = !isfinite(t1) || !isfinite(t0);   // give up at once
    s.conv = conv ? 1 : 0;
    s.done = (conv || bad) ? 1 : 0;
    if (s.done) atomicAdd(sb.ndone, 1);
  } else if (KIND == RED_APPLY) {
    s.pq = t0;
    s.alpha = s.rz / t0;
    // the scale of the r32 the next update writes (from the current ||r||)
    s.isc_prev = s.isc;
    s.sc = residual_scale(s.rr, rp.n);
    s.isc = 1.0 / s.sc;
  } else if (KIND == RED_UPDATE) {
    s.rr = t0;
    s.rzo = t1;
    s.it += 1;
    s.first = 0;
    if (sb.jacobi) {
      s.rzn = t2;
      s.beta = (t2 - t1) / s.rz;
      s.rz = t2;
    }
    const bool conv = t0 <= rtol * rtol * s.bb;
    s.conv = conv ? 1 : 0;
    if (conv || s.it >= maxit || !isfinite(t0)) {
      s.done = 1;
      atomicAdd(sb.ndone, 1);
    }
  } else {   // RED_RZ, RED_RZF: r.z' of the preconditioner, beta of the flexible CG
    s.rzn = t0;
    s.beta = s.first ? 0.0 : (t0 - s.rzo) / s.rz;
    s.rz = t0;
  }
}

__global__ void k_zero_int(int* p) { *p = 0; }

template <typename T>
void launch_cg_reduce(hipStream_t s, const Work& w, const SolverBufsT<T>& sb, int kind, double rtol,
                      int maxit, unsigned fm, int nrep) {
  const dim3 g(w.nreps), b(kBlock);
  switch (kind) {
    case RED_START:
      hca_launch(k_cg_reduce<RED_START, T>, g, b, 0, s, w, sb, rtol, maxit, fm, nrep);
      break;
    case RED_APPLY:
      hca_launch(k_cg_reduce<RED_APPLY, T>, g, b, 0, s, w, sb, rtol, maxit, fm, nrep);
      break;
    case RED_UPDATE:
      hca_launch(k_cg_reduce<RED_UPDATE, T>, g, b, 0, s, w, sb, rtol, maxit, fm, nrep);
      break;
    case RED_RZF:
      hca_launch(k_cg_reduce<RED_RZF, T>, g, b, 0, s, w, sb, rtol, maxit, fm, nrep);
      break;
    default:
      hca_launch(k_cg_reduce<RED_RZ, T>, g, b, 0, s, w, sb, rtol, maxit, fm, nrep);
      break;
  }
}

template <typename T>
void launch_cg_start(hipStream_t s, const Work& w, double rtol, int maxit, const T* c, const T* b,
                     const T* x, const SolverBufsT<T>& sb, unsigned field_mask, int nrep) {
  hca_launch(k_cg_start<T>, dim3(grid_tiles(w.ntiles, w.max_blocks)), dim3(kBlock), 0, s, w, c, b, x,
             sb);
  hca_launch(k_zero_int, dim3(1), dim3(1), 0, s, sb.ndone);   // before the start reduce counts
  launch_cg_reduce(s, w, sb, RED_START, rtol, maxit, field_mask, nrep);
  if (!sb.jacobi)
    hca_launch(k_cg_r32<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, sb);
}

template <typename T>
void launch_cg_apply_kernel(hipStream_t s, const Work& w, const T* c, T* x, const SolverBufsT<T>& sb,
                            int parity) {
  const T* pold = parity ? sb.p1 : sb.p0;
  T* pnew = parity ? sb.p0 : sb.p1;
  if (sb.jacobi)
    hca_launch(k_cg_apply<true, T>, dim3(grid_tiles(w.ntiles, w.max_blocks)), dim3(kBlock), 0, s, w, c,
               (const T*)sb.z, pold, pnew, sb.q, x, sb);
  else
    hca_launch(k_cg_apply<false, T>, dim3(grid_tiles(w.ntiles, w.max_blocks)), dim3(kBlock), 0, s, w, c,
               (const T*)sb.z, pold, pnew, sb.q, x, sb);
}

template <typename T>
void launch_cg_apply(hipStream_t s, const Work& w, const T* c, T* x, const SolverBufsT<T>& sb, int parity) {
  launch_cg_apply_kernel(s, w, c, x, sb, parity);
  launch_cg_reduce(s, w, sb, RED_APPLY, 0.0, 0);
}

template <typename T>
void launch_cg_update(hipStream_t s, const Work& w, double rtol, int maxit, const SolverBufsT<T>& sb) {
  if (sb.jacobi)
    hca_launch(k_cg_update<true, T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w,
               (const T*)sb.q, sb);
  else
    hca_launch(k_cg_update<false, T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w,
               (const T*)sb.q, sb);
  launch_cg_reduce(s, w, sb, RED_UPDATE, rtol, maxit);
}

template <typename T>
void launch_cg_finish(hipStream_t s, const Work& w, T* x, const SolverBufsT<T>& sb) {
  hca_launch(k_cg_finish<T>, dim3(grid_for(w.nflat, w.max_blocks)), dim3(kBlock), 0, s, w, x, sb);
}

#define HCA_SOLVER_INST(T)                                                                         \
  template void launch_cg_reduce<T>(hipStream_t, const Work&, const SolverBufsT<T>&, int, double,  \
                                    int, unsigned, int);                                           \
  template void launch_cg_start<T>(hipStream_t, const Work&, double, int, const T*, const T*,      \
                                   const T*, const SolverBufsT<T>&, unsigned, int);                \
  template void launch_cg_apply_kernel<T>(hipStream_t, const Work&, const T*, T*,                  \
                                          const SolverBufsT<T>&, int);                             \
  template void launch_cg_apply<T>(hipStream_t, const Work&, const T*, T*, const SolverBufsT<T>&,   \
                                   int);                                                           \
  template void launch_cg_update<T>(hipStream_t, const Work&, double, int, const SolverBufsT<T>&);  \
  template void launch_cg_finish<T>(hipStream_t, const Work&, T*, const SolverBufsT<T>&);        \
  template void launch_guess_projection<T>(hipStream_t, const Work&, const T*, const T*, T*, T*, T*, \
                                           double*, double*, unsigned, int, int);
HCA_SOLVER_INST(double)
HCA_SOLVER_INST(float)

}  // namespace hca
