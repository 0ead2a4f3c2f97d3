// Matrix-free preconditioned conjugate gradient for the implicit-Euler
// systems of Eqs. (oxygen) and (chemo) on the voxel lattice:
//
//     (A u)_i = c_i u_i - a (Lap u)_i = b_i,    a = D/h^2,
//
// Lap the 7-point Laplacian with zero-flux faces (a missing neighbour is
// dropped), A a symmetric M-matrix.  The paper solves the same SPD systems
// with CG (chemotherapy, linearised oxygen).  Here every replicate of the
// batch runs its own CG in the same launches: per-replicate dot products are
// reduced in a fixed order by the last workgroup of the replicate, and a
// finished replicate's workgroups return at once.
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
// still reads).
#include "dev_util.h"

namespace hca {

struct TileCoord {
  int rep;
  int x, y, z0, z1;
  bool valid;
  int nx, ny, nz;
  long long off;
};

__device__ inline TileCoord tile_coord(const Work& w) {
  const Tile t = w.tiles[blockIdx.x];
  const RepDev rp = w.reps[t.rep];
  TileCoord tc;
  tc.rep = t.rep;
  tc.x = t.x0 + (int)(threadIdx.x % rp.tx);
  tc.y = t.y0 + (int)(threadIdx.x / rp.tx);
  tc.z0 = t.z0;
  tc.z1 = t.z1;
  tc.nx = rp.nx;
  tc.ny = rp.ny;
  tc.nz = rp.nz;
  tc.off = rp.off;
  tc.valid = tc.x < rp.nx && tc.y < rp.ny;
  return tc;
}

// Marches one column (x, y) over [z0, z1) and calls f(i, z, u_c, Au, deg)
// where u = U(j) is the operand (possibly formed on the fly) and
// Au = (c_i + a deg) u_i - a sum_nb u_j.
template <typename UF, typename F>
__device__ inline void stencil_column(const TileCoord& tc, const double* __restrict__ c, double a,
                                      UF U, F f) {
  const long long plane = (long long)tc.nx * tc.ny;
  long long i = tc.off + tc.x + (long long)tc.nx * (tc.y + (long long)tc.ny * tc.z0);
  double um = tc.z0 > 0 ? U(i - plane) : 0.0;
  double uc = U(i);
  const bool xl = tc.x > 0, xr = tc.x + 1 < tc.nx, yl = tc.y > 0, yr = tc.y + 1 < tc.ny;
  const int deg_xy = (int)xl + (int)xr + (int)yl + (int)yr;
  for (int z = tc.z0; z < tc.z1; ++z) {
    const bool zl = z > 0, zr = z + 1 < tc.nz;
    const double up = zr ? U(i + plane) : 0.0;
    double s = 0.0;
    if (xl) s += U(i - 1);
    if (xr) s += U(i + 1);
    if (yl) s += U(i - tc.nx);
    if (yr) s += U(i + tc.nx);
    if (zl) s += um;
    if (zr) s += up;
    const int deg = deg_xy + (int)zl + (int)zr;
    const double Au = (c[i] + a * deg) * uc - a * s;
    f(i, deg, uc, Au);
    um = uc;
    uc = up;
    i += plane;
  }
}

// r = b - A x; Jacobi z = r / diag(A); p is set by the first iteration.
__global__ void __launch_bounds__(kBlock) k_cg_start(Work w, double a, double rtol,
                                                     const double* __restrict__ c,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ x,
                                                     SolverBufs sb) {
  __shared__ double lds4[4];
  const TileCoord tc = tile_coord(w);
  double bb = 0.0, rr = 0.0, rz = 0.0;
  if (tc.valid) {
    stencil_column(tc, c, a, [&](long long j) { return x[j]; },
                   [&](long long i, int deg, double, double Ax) {
                     const double bi = b[i];
                     const double r = bi - Ax;
                     sb.r[i] = r;
                     bb += bi * bi;
                     rr += r * r;
                     if (sb.jacobi) {
                       const double di = 1.0 / (c[i] + a * deg);
                       const double zz = r * di;
                       sb.dinv[i] = di;
                       sb.z[i] = zz;
                       rz += r * zz;
                     }
                   });
  }
  double v[3];
  v[0] = block_sum(bb, lds4);
  v[1] = block_sum(rr, lds4);
  v[2] = block_sum(rz, lds4);
  const RepDev rp = w.reps[tc.rep];
  if (publish_and_check_last(sb.partial + (size_t)blockIdx.x * 3, v, 3, sb.counter + tc.rep,
                             rp.tile_nb)) {
    const double* base = sb.partial + (size_t)rp.tile_b0 * 3;
    const double tbb = reduce_partials(base, rp.tile_nb, 3, 0, lds4);
    const double trr = reduce_partials(base, rp.tile_nb, 3, 1, lds4);
    const double trz = reduce_partials(base, rp.tile_nb, 3, 2, lds4);
    if (threadIdx.x == 0) {
      SolveScal& s = sb.ss[tc.rep];
      s.bb = tbb;
      s.rr = trr;
      s.rr0 = trr;
      s.rz = trz;
      s.rzn = trz;
      s.rzo = 0.0;
      s.beta = 0.0;
      s.alpha = 0.0;
      s.pq = 0.0;
      s.it = 0;
      s.first = 1;
      const bool conv = trr <= rtol * rtol * tbb;
      const bool bad = !isfinite(trr) || !isfinite(tbb);   // give up at once
      s.conv = conv ? 1 : 0;
      s.done = (conv || bad) ? 1 : 0;
      if (s.done) atomicAdd(sb.ndone, 1);
    }
  }
}

// p_new = z + beta p_old (p_new = z on the first iteration), q = A p_new,
// alpha = r.z / p.q.
__global__ void __launch_bounds__(kBlock) k_cg_apply(Work w, double a,
                                                     const double* __restrict__ c,
                                                     const double* __restrict__ z,
                                                     const double* __restrict__ pold,
                                                     double* __restrict__ pnew,
                                                     double* __restrict__ q, SolverBufs sb) {
  __shared__ double lds4[4];
  const TileCoord tc = tile_coord(w);
  const SolveScal* ssr = sb.ss + tc.rep;
  if (ssr->done) return;
  const double beta = ssr->beta;
  const bool first = ssr->first != 0;
  double pq = 0.0;
  if (tc.valid) {
    auto U = [&](long long j) { return first ? z[j] : z[j] + beta * pold[j]; };
    stencil_column(tc, c, a, U, [&](long long i, int, double pc, double Ap) {
      pnew[i] = pc;
      q[i] = Ap;
      pq += pc * Ap;
    });
  }
  double v = block_sum(pq, lds4);
  const RepDev rp = w.reps[tc.rep];
  if (publish_and_check_last(sb.partial + (size_t)blockIdx.x * 3, &v, 1, sb.counter + tc.rep,
                             rp.tile_nb)) {
    const double tpq = reduce_partials(sb.partial + (size_t)rp.tile_b0 * 3, rp.tile_nb, 3, 0, lds4);
    if (threadIdx.x == 0) {
      SolveScal& s = sb.ss[tc.rep];
      s.pq = tpq;
      s.alpha = s.rz / tpq;
    }
  }
}

// x += alpha p, r -= alpha q; convergence check.  Jacobi mode also forms
// z' = r / diag(A) and beta = (r.z' - r.z_old) / r.z; multigrid mode leaves z'
// and beta to the V-cycle and only records r.z_old.
__global__ void __launch_bounds__(kBlock) k_cg_update(Work w, double rtol, int maxit,
                                                      double* __restrict__ x,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ q,
                                                      SolverBufs sb) {
  __shared__ double lds4[4];
  const FlatBlk fb = w.flat[blockIdx.x];
  const SolveScal* ssr = sb.ss + fb.rep;
  if (ssr->done) return;
  const RepDev rp = w.reps[fb.rep];
  const double alpha = ssr->alpha;
  const bool jac = sb.jacobi != 0;
  double rr = 0.0, rzo = 0.0, rzn = 0.0;
  const long long nchunks = (rp.n + kFlatChunk - 1) / kFlatChunk;
  for (long long ch = fb.first; ch < nchunks; ch += rp.flat_nb) {
    const long long base = rp.off + ch * kFlatChunk;
    const long long lim = rp.off + rp.n;
#pragma unroll
    for (int k = 0; k < kFlatChunk / kBlock; ++k) {
      const long long i = base + k * kBlock + threadIdx.x;
      if (i < lim) {
        x[i] += alpha * p[i];
        const double r = sb.r[i] - alpha * q[i];
        sb.r[i] = r;
        const double zold = sb.z[i];
        rr += r * r;
        rzo += r * zold;
        if (jac) {
          const double znew = r * sb.dinv[i];
          sb.z[i] = znew;
          rzn += r * znew;
        }
      }
    }
  }
  double v[3];
  v[0] = block_sum(rr, lds4);
  v[1] = block_sum(rzo, lds4);
  v[2] = block_sum(rzn, lds4);
  if (publish_and_check_last(sb.partial + (size_t)blockIdx.x * 3, v, 3, sb.counter + fb.rep,
                             rp.flat_nb)) {
    const double* base = sb.partial + (size_t)rp.flat_b0 * 3;
    const double trr = reduce_partials(base, rp.flat_nb, 3, 0, lds4);
    const double trzo = reduce_partials(base, rp.flat_nb, 3, 1, lds4);
    const double trzn = reduce_partials(base, rp.flat_nb, 3, 2, lds4);
    if (threadIdx.x == 0) {
      SolveScal& s = sb.ss[fb.rep];
      s.rr = trr;
      s.rzo = trzo;
      s.it += 1;
      s.first = 0;
      if (jac) {
        s.rzn = trzn;
        s.beta = (trzn - trzo) / s.rz;
        s.rz = trzn;
      }
      const bool conv = trr <= rtol * rtol * s.bb;
      s.conv = conv ? 1 : 0;
      if (conv || s.it >= maxit || !isfinite(trr)) {
        s.done = 1;
        atomicAdd(sb.ndone, 1);
      }
    }
  }
}

__global__ void k_zero_int(int* p) { *p = 0; }

void launch_cg_start(hipStream_t s, const Work& w, double a, double rtol, int,
                     const double* c, const double* b, const double* x, const SolverBufs& sb) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, sb.ndone);
  hipLaunchKernelGGL(k_cg_start, dim3(w.ntiles), dim3(kBlock), 0, s, w, a, rtol, c, b, x, sb);
}

void launch_cg_apply(hipStream_t s, const Work& w, double a, const double* c,
                     const SolverBufs& sb, int parity) {
  const double* pold = parity ? sb.p1 : sb.p0;
  double* pnew = parity ? sb.p0 : sb.p1;
  hipLaunchKernelGGL(k_cg_apply, dim3(w.ntiles), dim3(kBlock), 0, s, w, a, c, sb.z, pold, pnew,
                     sb.q, sb);
}

void launch_cg_update(hipStream_t s, const Work& w, double, double rtol, int maxit,
                      const double*, double* x, const SolverBufs& sb, int parity) {
  const double* pnew = parity ? sb.p0 : sb.p1;
  hipLaunchKernelGGL(k_cg_update, dim3(w.nflat), dim3(kBlock), 0, s, w, rtol, maxit, x, pnew,
                     (const double*)sb.q, sb);
}

}  // namespace hca
