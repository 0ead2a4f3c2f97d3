// Geometric multigrid V-cycle, FP32, used as the preconditioner of the FP64
// flexible CG for the implicit-Euler systems of Eqs. (oxygen) and (chemo).
// (The paper preconditions the same SPD systems with algebraic multigrid.)
//
// Hierarchy: voxel-centred 2:1 coarsening per axis, n_{k+1} = ceil(n_k / 2); a
// level-k cell I covers the fine cells [I 2^k, min((I+1) 2^k, n0)) per axis
// (ragged at odd edges).  The level-k operator is
//     (A_k u)_I = c_I u_I + sum_faces g_IJ (u_I - u_J),
// c_I the sum of the fine reaction coefficients over the cell, and g_IJ the
// finite-volume coupling of the two aggregates: D/h^2 times the shared face
// area over the centre distance, both in fine-voxel units,
//     g = a * area / ((e_I + e_J) / 2),   e = extents along the face normal.
// Restriction sums fine residuals over the aggregate; prolongation is
// cell-centred linear interpolation (about a third fewer CG iterations than
// piecewise-constant for the diffusion-dominated drug operator); smoothing is
// weighted Jacobi (two sweeps before and two after the coarse-grid
// correction).  Levels above `mg_coarse_max` cells run as multi-workgroup
// kernels; the remaining levels of each system are one workgroup working in
// LDS down to a single cell (solved exactly), the same cycle.
//
// Fused kernels per global level k:
//   pre      u1 = w Dinv r (first sweep from zero, formed on the fly at the
//            neighbours), u2 = (1-w) u1 + w Dinv (r + sum g u1_J)
//   restrict r_{k+1}(I) = sum over children of (r - A u2)
//   post1    u3 = u2 + P e_{k+1} (formed on the fly; P the cell-centred
//            linear interpolation, restriction stays the aggregate sum), u4 =
//            Jacobi(u3)
//   post2    u5 = Jacobi(u4); at level 0 u5 is the CG's z, and the same kernel
//            reduces r.z and finishes beta of the flexible CG.
#include "dev_util.h"

namespace hca {

template <bool UNI>
struct Geo {
  int nx, ny, nz, k, n0x, n0y, n0z;
  float a;

  __device__ inline int ext(int I, int n0) const {
    if (UNI) return 1;
    const int lo = I << k;
    const int hi = min((I + 1) << k, n0);
    return hi - lo;
  }
  // couplings of the faces (x,y,z)-(x+1,y,z), (x,y,z)-(x,y+1,z), (x,y,z)-(x,y,z+1)
  __device__ inline float gx(int x, int y, int z) const {
    if (UNI) return a;
    return 2.f * a * (float)(ext(y, n0y) * ext(z, n0z)) / (float)(ext(x, n0x) + ext(x + 1, n0x));
  }
  __device__ inline float gy(int x, int y, int z) const {
    if (UNI) return a;
    return 2.f * a * (float)(ext(x, n0x) * ext(z, n0z)) / (float)(ext(y, n0y) + ext(y + 1, n0y));
  }
  __device__ inline float gz(int x, int y, int z) const {
    if (UNI) return a;
    return 2.f * a * (float)(ext(x, n0x) * ext(y, n0y)) / (float)(ext(z, n0z) + ext(z + 1, n0z));
  }
  // sum of the couplings of the existing faces of (x,y,z)
  __device__ inline float gsum(int x, int y, int z) const {
    float s = 0.f;
    if (x > 0) s += gx(x - 1, y, z);
    if (x + 1 < nx) s += gx(x, y, z);
    if (y > 0) s += gy(x, y - 1, z);
    if (y + 1 < ny) s += gy(x, y, z);
    if (z > 0) s += gz(x, y, z - 1);
    if (z + 1 < nz) s += gz(x, y, z);
    return s;
  }
};

template <bool UNI>
__device__ inline Geo<UNI> geo_of(const MgRep& m) {
  const float a = m.a;
  Geo<UNI> g;
  g.nx = m.nx;
  g.ny = m.ny;
  g.nz = m.nz;
  g.k = m.k;
  g.n0x = m.n0x;
  g.n0y = m.n0y;
  g.n0z = m.n0z;
  g.a = a;
  return g;
}

// LDS plane of one tile with a one-cell frame: (tx + 2) (256/tx + 2) values.
constexpr int kPlaneMaxF = 400;

// Marches a tile over [t.z0, t.z1) and calls f(z, i, v_i, sum_J g_IJ v_J, ctr)
// for the tile's cells inside the level, v = op.value(op.load(x, y, z, j))
// possibly formed on the fly and ctr = op.ctr(i) the cell's own further
// operands (D^-1, r).  Each plane of v with its x/y frame is formed once into
// LDS (double buffered), so v is evaluated about once per cell instead of at
// every neighbour; the neighbour terms are added in the order -x, +x, -y, +y,
// -z, +z.  Software pipelined: the loads of plane z+2 and the centre
// operands of plane z+1 are issued before plane z is computed.  Called by the
// whole workgroup (it synchronises).
template <bool UNI, typename OP, typename F, typename E>
__device__ inline void mg_plane(const Geo<UNI>& G, const Tile& t, int tx, long long base,
                                float (*lds)[kPlaneMaxF], const OP& op, F f, E epilogue) {
  using Raw = typename OP::Raw;
  using Ctr = typename OP::Ctr;
  const int ty = kBlock / tx;
  const int lx = (int)(threadIdx.x % tx), ly = (int)(threadIdx.x / tx);
  const int x = t.x0 + lx, y = t.y0 + ly;
  const bool valid = x < G.nx && y < G.ny;
  const int W = tx + 2;
  const int o = (ly + 1) * W + lx + 1;
  const int nframe = 2 * W + 2 * ty;
  const long long plane = (long long)G.nx * G.ny;
  // this thread's frame cell (at most one: nframe <= 256)
  const int k = threadIdx.x;
  const bool has_frame = k < nframe;
  int hx = 0, hy = 0;
  if (k < W) {
    hx = k;
    hy = 0;
  } else if (k < 2 * W) {
    hx = k - W;
    hy = ty + 1;
  } else if (k < 2 * W + ty) {
    hx = 0;
    hy = 1 + k - 2 * W;
  } else {
    hx = W - 1;
    hy = 1 + k - 2 * W - ty;
  }
  const int gx = t.x0 + hx - 1, gy = t.y0 + hy - 1;
  const bool fin = has_frame && gx >= 0 && gx < G.nx && gy >= 0 && gy < G.ny;
  const int fo = hy * W + hx;
  const long long fidx = fin ? gx + (long long)G.nx * gy : 0;
  const long long iidx = x + (long long)G.nx * y;
  Raw ri = op.zero(), rf = op.zero();
  auto load_plane = [&](int z) {
    const long long pz = base + plane * z;
    if (valid) ri = op.load(x, y, z, pz + iidx);
    if (fin) rf = op.load(gx, gy, z, pz + fidx);
  };
  auto store_plane = [&](float* buf) {
    buf[o] = valid ? op.value(ri) : 0.f;
    if (has_frame) buf[fo] = fin ? op.value(rf) : 0.f;
  };
  const int z0 = t.z0, z1 = t.z1;
  long long i = base + iidx + plane * z0;
  float* cur = lds[0];
  float* nxt = lds[1];
  __syncthreads();   // the previous tile's readers are done with both buffers
  load_plane(z0);
  float vm = (valid && z0 > 0) ? op.value(op.load(x, y, z0 - 1, i - plane)) : 0.f;
  Ctr cc = op.ctr_zero();
  if (valid) {
    if constexpr (OP::kCtrInRaw)
      cc = op.ctr_of(ri);
    else
      cc = op.ctr(i);
  }
  store_plane(cur);
  if (z0 + 1 < G.nz) load_plane(z0 + 1);
  __syncthreads();
  float vc = cur[o];
  for (int z = z0; z < z1; ++z) {
    const bool zr = z + 1 < G.nz;
    const bool more = z + 1 < z1;
    Ctr cn = op.ctr_zero();
    if constexpr (OP::kCtrInRaw) {   // plane z+1's raw operands are its centre operands
      if (more && valid) cn = op.ctr_of(ri);
    }
    if (zr) store_plane(nxt);
    if (more && z + 2 < G.nz) load_plane(z + 2);
    if constexpr (!OP::kCtrInRaw) cn = (more && valid) ? op.ctr(i + plane) : op.ctr_zero();
    float s = 0.f;
    if (valid) {
      if (x > 0) s += G.gx(x - 1, y, z) * cur[o - 1];
      if (x + 1 < G.nx) s += G.gx(x, y, z) * cur[o + 1];
      if (y > 0) s += G.gy(x, y - 1, z) * cur[o - W];
      if (y + 1 < G.ny) s += G.gy(x, y, z) * cur[o + W];
    }
    __syncthreads();
    const float vp = zr ? nxt[o] : 0.f;
    if (valid) {
      if (z > 0) s += G.gz(x, y, z - 1) * vm;
      if (zr) s += G.gz(x, y, z) * vp;
      f(z, i, vc, s, cc);
    }
    epilogue(z);   // every thread, every plane
    vm = vc;
    vc = vp;
    cc = cn;
    float* tmp = cur;
    cur = nxt;
    nxt = tmp;
    i += plane;
  }
}

template <bool UNI, typename OP, typename F>
__device__ inline void mg_plane(const Geo<UNI>& G, const Tile& t, int tx, long long base,
                                float (*lds)[kPlaneMaxF], const OP& op, F f) {
  mg_plane(G, t, tx, base, lds, op, f, [](int) {});
}

// Centre operands of the smoothers: D^-1 and r of the cell.
template <typename RT>
struct CtrDR {
  float dinv;
  RT r;
};

struct TileXY {
  int rep, x, y, z0, z1;
  bool valid;
};

__device__ inline TileXY tile_xy(const Tile* tiles, const MgRep* reps, int ti) {
  const Tile t = tiles[ti];
  const MgRep& m = reps[t.rep];
  TileXY c;
  c.rep = t.rep;
  c.x = t.x0 + (int)(threadIdx.x % m.tx);
  c.y = t.y0 + (int)(threadIdx.x / m.tx);
  c.z0 = t.z0;
  c.z1 = t.z1;
  c.valid = c.x < m.nx && c.y < m.ny;
  return c;
}

// Every kernel below loops over its workgroup's contiguous run of tiles.
#define FOR_MY_TILES(ntiles)   \
  int tile_b_, tile_e_;        \
  tile_range((ntiles), tile_b_, tile_e_); \
  for (int ti = tile_b_; ti < tile_e_; ++ti)

// ---- setup per solve -------------------------------------------------------

// Level 0: Dinv = 1 / (c + a deg).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_mg_prep0(MgLevel L0, const T* __restrict__ c) {
  FOR_MY_TILES(L0.ntiles) {
    const TileXY t = tile_xy(L0.tiles, L0.reps, ti);
    if (!t.valid) continue;
    const MgRep m = L0.reps[t.rep];
    const Geo<true> G = geo_of<true>(m);
    long long i = m.off + t.x + (long long)m.nx * (t.y + (long long)m.ny * t.z0);
    const long long plane = (long long)m.nx * m.ny;
    for (int z = t.z0; z < t.z1; ++z, i += plane)
      L0.dinv[i] = (float)(1.0 / ((double)c[i] + (double)G.gsum(t.x, t.y, z)));
  }
}

// Level k+1 from level k: c_{k+1} = sum of the children's c, Dinv_{k+1}.
// From level 0 (FROM0) the same pass also writes level 0's Dinv = 1 / (c +
// a deg) of every child (each level-0 cell is the child of exactly one
// level-1 cell), so level 0's c is read once.
template <bool FROM0, typename T>
__global__ void __launch_bounds__(kBlock) k_mg_coarsen(MgLevel Lf, MgLevel Lc,
                                                       const T* __restrict__ c0) {
  FOR_MY_TILES(Lc.nrtiles) {
    const TileXY t = tile_xy(Lc.rtiles, Lc.reps, ti);
    if (!t.valid) continue;
    const MgRep mc = Lc.reps[t.rep];
    const MgRep mf = Lf.reps[t.rep];
    const Geo<false> G = geo_of<false>(mc);
    const Geo<true> Gf = geo_of<true>(mf);
    for (int Z = t.z0; Z < t.z1; ++Z) {
      float s = 0.f;
      for (int dz = 0; dz < 2; ++dz) {
        const int z = 2 * Z + dz;
        if (z >= mf.nz) break;
        for (int dy = 0; dy < 2; ++dy) {
          const int y = 2 * t.y + dy;
          if (y >= mf.ny) break;
          for (int dx = 0; dx < 2; ++dx) {
            const int x = 2 * t.x + dx;
            if (x >= mf.nx) break;
            const long long j = mf.off + x + (long long)mf.nx * (y + (long long)mf.ny * z);
            if (FROM0) {
              const double cj = (double)c0[j];
              Lf.dinv[j] = (float)(1.0 / (cj + (double)Gf.gsum(x, y, z)));
              s += (float)cj;
            } else {
              s += Lf.c[j];
            }
          }
        }
      }
      const long long I = mc.off + t.x + (long long)mc.nx * (t.y + (long long)mc.ny * Z);
      Lc.c[I] = s;
      Lc.dinv[I] = 1.f / (s + G.gsum(t.x, t.y, Z));
    }
  }
}

// ---- V-cycle, global levels ------------------------------------------------

// First sweep from zero, formed on the fly at the neighbours: u1 = w D^-1 r.
template <typename RT>
struct OpPre {
  struct Raw {
    float dinv;
    RT r;
  };
  using Ctr = CtrDR<RT>;
  static constexpr bool kCtrInRaw = true;   // ctr_of(raw) instead of a second load
  const float* __restrict__ dinv;
  const RT* __restrict__ r;
  float omega;
  __device__ inline Raw zero() const { return Raw{0.f, (RT)0}; }
  __device__ inline Raw load(int, int, int, long long j) const { return Raw{dinv[j], r[j]}; }
  __device__ inline float value(const Raw& v) const { return omega * v.dinv * (float)v.r; }
  __device__ inline Ctr ctr_zero() const { return Ctr{0.f, (RT)0}; }
  __device__ inline Ctr ctr(long long i) const { return Ctr{dinv[i], r[i]}; }
  __device__ inline Ctr ctr_of(const Raw& v) const { return Ctr{v.dinv, v.r}; }
};

template <bool L0, typename RT>
__global__ void __launch_bounds__(kBlock) k_mg_pre(MgLevel Lk, float wa, float wb,
                                                   const RT* __restrict__ r, float* __restrict__ u,
                                                   const SolveScal* ss) {
  __shared__ float lds[2][kPlaneMaxF];
  FOR_MY_TILES(Lk.ntiles) {
    const Tile t = Lk.tiles[ti];
    if (ss[t.rep].done) continue;
    const MgRep m = Lk.reps[t.rep];
    const Geo<L0> G = geo_of<L0>(m);
    const OpPre<RT> op{Lk.dinv, r, wa};
    mg_plane(G, t, m.tx, m.off, lds, op,
             [&](int, long long i, float u1, float s, const CtrDR<RT>& c) {
               u[i] = (1.f - wb) * u1 + wb * c.dinv * ((float)c.r + s);
             });
  }
}
// Plain operand v = u with the cell's (D^-1, r) (second post-sweep, and the
// residual of the restriction).
template <typename RT>
struct OpU {
  struct Raw {
    float u;
  };
  using Ctr = CtrDR<RT>;
  static constexpr bool kCtrInRaw = false;
  const float* __restrict__ u;
  const float* __restrict__ dinv;
  const RT* __restrict__ r;
  __device__ inline Raw zero() const { return Raw{0.f}; }
  __device__ inline Raw load(int, int, int, long long j) const { return Raw{u[j]}; }
  __device__ inline float value(const Raw& v) const { return v.u; }
  __device__ inline Ctr ctr_zero() const { return Ctr{0.f, (RT)0}; }
  __device__ inline Ctr ctr(long long i) const { return Ctr{dinv[i], r[i]}; }
};

// Restriction r_{k+1}(I) = sum over the children of (r - A u), marched over
// the fine level's tiles: each cell's residual from the LDS plane of u, the
// 2 x 2 children of a coarse cell summed across lanes (tiles are 16 or 32
// columns wide, so a cell's x-neighbour is lane ^ 1 and its y-neighbour
// lane ^ tx, both in the same wavefront), the two child planes in a register.
// Tile origins are even in x, y and z.
template <bool L0, typename RT>
__global__ void __launch_bounds__(kBlock) k_mg_restrict(MgLevel Lf, MgLevel Lc,
                                                        const RT* __restrict__ r,
                                                        const SolveScal* ss) {
  __shared__ float lds[2][kPlaneMaxF];
  FOR_MY_TILES(Lf.ntiles) {
    const Tile t = Lf.tiles[ti];
    if (ss[t.rep].done) continue;
    const MgRep mf = Lf.reps[t.rep];
    const MgRep mc = Lc.reps[t.rep];
    const Geo<L0> G = geo_of<L0>(mf);
    const int tx = mf.tx;
    const int lx = (int)(threadIdx.x % tx), ly = (int)(threadIdx.x / tx);
    const int x = t.x0 + lx, y = t.y0 + ly;
    const bool lead = ((lx | ly) & 1) == 0 && x < mf.nx && y < mf.ny;
    float res = 0.f, acc = 0.f;
    const OpU<RT> op{Lf.u, Lf.dinv, r};
    mg_plane(G, t, tx, mf.off, lds, op,
             [&](int, long long, float uc, float s, const CtrDR<RT>& c) {
               res = (float)c.r - uc / c.dinv + s;
             },
             [&](int z) {
               float q = res + __shfl_xor(res, 1, 64);
               q = q + __shfl_xor(q, tx, 64);
               acc += q;
               res = 0.f;
               if ((z & 1) || z + 1 == mf.nz) {
                 if (lead)
                   Lc.r[mc.off + (x >> 1) + (long long)mc.nx * ((y >> 1) + (long long)mc.ny * (z >> 1))] = acc;
                 acc = 0.f;
               }
             });
  }
}

// Cell-centred linear prolongation, per axis: fine cell i of a level with nf
// cells takes 3/4 of its own aggregate I = i/2 and 1/4 of the neighbouring
// aggregate J on its side; at the lattice boundary, and inside or next to the
// single-cell aggregate of an odd edge, it takes its own aggregate alone.
__device__ inline void lin_axis(int i, int nf, int nc, int& I, int& J, float& wJ) {
  I = i >> 1;
  J = (i & 1) ? I + 1 : I - 1;
  wJ = 0.25f;
  const bool ragged = (nf & 1) != 0;
  if (J < 0 || J >= nc || (ragged && (I == nc - 1 || J == nc - 1))) {
    J = I;
    wJ = 0.f;
  }
}


// Post-smoothing after the coarse-grid correction: u3 = u2 + P e, then one
// weighted-Jacobi sweep of u3 into ualt.  P e is separable: a coarse plane Z
// interpolated in x and y to one of this thread's fine columns,
//     E_Z = (1 - wy) ((1 - wx) e[Z,Iy,Ix] + wx e[Z,Iy,Jx])
//           + wy ((1 - wx) e[Z,Jy,Ix] + wx e[Z,Jy,Jx]),
// serves every fine plane whose z interpolation takes Z (four of them), and a
// fine plane takes (1 - wz) E_Iz + wz E_Jz.  Each thread owns two columns (its
// interior cell and at most one frame cell of the tile) and keeps E of the
// coarse planes I - 1, I, I + 1 around the current fine plane's I = z / 2 in
// registers, the four coarse values of plane I + 2 in flight: four coarse
// loads per column per two fine planes instead of eight per cell.  The
// marching (one plane of u3 with its frame in LDS, double buffered, the
// loads of plane z + 2 issued before plane z is computed, neighbour terms in
// the order -x, +x, -y, +y, -z, +z) is that of mg_plane.
struct PCol {
  int o[4];    // offsets of (Iy,Ix), (Iy,Jx), (Jy,Ix), (Jy,Jx) within a coarse plane
  float wx, wy;
};

__device__ inline PCol pcol(int x, int y, int nfx, int nfy, const MgRep& mc) {
  int Ix, Jx, Iy, Jy;
  PCol c;
  lin_axis(x, nfx, mc.nx, Ix, Jx, c.wx);
  lin_axis(y, nfy, mc.ny, Iy, Jy, c.wy);
  c.o[0] = Iy * mc.nx + Ix;
  c.o[1] = Iy * mc.nx + Jx;
  c.o[2] = Jy * mc.nx + Ix;
  c.o[3] = Jy * mc.nx + Jx;
  return c;
}

// E of coarse plane Z (x first along each coarse row, then y)
__device__ inline float pcol_interp(const PCol& c, const float (&g)[4]) {
  const float r0 = (1.f - c.wx) * g[0] + c.wx * g[1];
  const float r1 = (1.f - c.wx) * g[2] + c.wx * g[3];
  return (1.f - c.wy) * r0 + c.wy * r1;
}

// The coarse-plane window of one column: E of planes I-1, I, I+1 and the raw
// values of plane I+2 (planes outside the level read as 0; they only ever
// enter with weight 0).
struct PWin {
  float em, e0, ep;
  float g[4];
};

template <bool L0, typename RT>
__global__ void __launch_bounds__(kBlock) k_mg_post1(MgLevel Lk, MgLevel Lc, const float* __restrict__ e,
                                                     float omega, const RT* __restrict__ r,
                                                     const SolveScal* ss) {
  __shared__ float lds[2][kPlaneMaxF];
  float* __restrict__ out = Lk.ualt;
  const float* __restrict__ u = Lk.u;
  const float* __restrict__ dinv = Lk.dinv;
  FOR_MY_TILES(Lk.ntiles) {
    const Tile t = Lk.tiles[ti];
    if (ss[t.rep].done) continue;
    const MgRep m = Lk.reps[t.rep];
    const MgRep mc = Lc.reps[t.rep];
    const Geo<L0> G = geo_of<L0>(m);
    const int tx = m.tx, ty = kBlock / tx;
    const int lx = (int)(threadIdx.x % tx), ly = (int)(threadIdx.x / tx);
    const int x = t.x0 + lx, y = t.y0 + ly;
    const bool valid = x < G.nx && y < G.ny;
    const int W = tx + 2;
    const int o = (ly + 1) * W + lx + 1;
    const int nframe = 2 * W + 2 * ty;
    const int k = threadIdx.x;
    const bool has_frame = k < nframe;
    int hx = 0, hy = 0;
    if (k < W) {
      hx = k;
      hy = 0;
    } else if (k < 2 * W) {
      hx = k - W;
      hy = ty + 1;
    } else if (k < 2 * W + ty) {
      hx = 0;
      hy = 1 + k - 2 * W;
    } else {
      hx = W - 1;
      hy = 1 + k - 2 * W - ty;
    }
    const int fx = t.x0 + hx - 1, fy = t.y0 + hy - 1;
    const bool fin = has_frame && fx >= 0 && fx < G.nx && fy >= 0 && fy < G.ny;
    const int fo = hy * W + hx;
    const long long plane = (long long)G.nx * G.ny;
    const long long fidx = fin ? fx + (long long)G.nx * fy : 0;
    const long long iidx = x + (long long)G.nx * y;
    const PCol ci = pcol(valid ? x : 0, valid ? y : 0, G.nx, G.ny, mc);
    const PCol cf = pcol(fin ? fx : 0, fin ? fy : 0, G.nx, G.ny, mc);
    const float* __restrict__ eb = e + mc.off;
    const long long csz = (long long)mc.nx * mc.ny;
    auto gather = [&](const PCol& c, bool on, int Z, float (&g)[4]) {
      if (on && Z >= 0 && Z < mc.nz) {
        const float* b = eb + csz * Z;
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = b[c.o[q]];
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = 0.f;
      }
    };
    PWin wi, wf;
    int Iw;
    // window centred on coarse plane I (prologue: E of I-1, I, I+1 directly)
    auto win_start = [&](int I) {
      Iw = I;
      float g[4];
      gather(ci, valid, I - 1, g);
      wi.em = pcol_interp(ci, g);
      gather(ci, valid, I, g);
      wi.e0 = pcol_interp(ci, g);
      gather(ci, valid, I + 1, g);
      wi.ep = pcol_interp(ci, g);
      gather(ci, valid, I + 2, wi.g);
      gather(cf, fin, I - 1, g);
      wf.em = pcol_interp(cf, g);
      gather(cf, fin, I, g);
      wf.e0 = pcol_interp(cf, g);
      gather(cf, fin, I + 1, g);
      wf.ep = pcol_interp(cf, g);
      gather(cf, fin, I + 2, wf.g);
    };
    auto win_step = [&](PWin& w, const PCol& c, bool on) {
      w.em = w.e0;
      w.e0 = w.ep;
      w.ep = pcol_interp(c, w.g);
      gather(c, on, Iw + 2, w.g);
    };
    // P e of fine plane z at a column (the window moved to z / 2 first)
    auto pe = [&](const PWin& w, int z) {
      int Iz, Jz;
      float wz;
      lin_axis(z, G.nz, mc.nz, Iz, Jz, wz);
      if (Jz == Iz) return w.e0;
      return (1.f - wz) * w.e0 + wz * (Jz < Iz ? w.em : w.ep);
    };
    auto win_to = [&](int z) {
      if ((z >> 1) != Iw) {   // planes are formed in increasing z: one step
        ++Iw;
        win_step(wi, ci, valid);
        win_step(wf, cf, fin);
      }
    };
    float ui = 0.f, uf = 0.f;   // raw u of the next plane to form
    auto load_plane = [&](int z) {
      const long long pz = m.off + plane * z;
      if (valid) ui = u[pz + iidx];
      if (fin) uf = u[pz + fidx];
    };
    auto store_plane = [&](float* buf, int z) {
      win_to(z);
      buf[o] = valid ? ui + pe(wi, z) : 0.f;
      if (has_frame) buf[fo] = fin ? uf + pe(wf, z) : 0.f;
    };
    const int z0 = t.z0, z1 = t.z1;
    long long i = m.off + iidx + plane * z0;
    float* cur = lds[0];
    float* nxt = lds[1];
    __syncthreads();   // the previous tile's readers are done with both buffers
    win_start((z0 > 0 ? z0 - 1 : z0) >> 1);
    load_plane(z0);
    float vm = 0.f;
    if (z0 > 0) {
      const float um = valid ? u[i - plane] : 0.f;
      win_to(z0 - 1);
      vm = valid ? um + pe(wi, z0 - 1) : 0.f;
    }
    float cd = 0.f;
    RT cr = (RT)0;
    if (valid) {
      cd = dinv[i];
      cr = r[i];
    }
    store_plane(cur, z0);
    if (z0 + 1 < G.nz) load_plane(z0 + 1);
    __syncthreads();
    float vc = cur[o];
    for (int z = z0; z < z1; ++z) {
      const bool zr = z + 1 < G.nz;
      const bool more = z + 1 < z1;
      if (zr) store_plane(nxt, z + 1);
      if (more && z + 2 < G.nz) load_plane(z + 2);
      float nd = 0.f;
      RT nr = (RT)0;
      if (more && valid) {
        nd = dinv[i + plane];
        nr = r[i + plane];
      }
      float s = 0.f;
      if (valid) {
        if (x > 0) s += G.gx(x - 1, y, z) * cur[o - 1];
        if (x + 1 < G.nx) s += G.gx(x, y, z) * cur[o + 1];
        if (y > 0) s += G.gy(x, y - 1, z) * cur[o - W];
        if (y + 1 < G.ny) s += G.gy(x, y, z) * cur[o + W];
      }
      __syncthreads();
      const float vp = zr ? nxt[o] : 0.f;
      if (valid) {
        if (z > 0) s += G.gz(x, y, z - 1) * vm;
        if (zr) s += G.gz(x, y, z) * vp;
        out[i] = (1.f - omega) * vc + omega * cd * ((float)cr + s);
      }
      vm = vc;
      vc = vp;
      cd = nd;
      cr = nr;
      float* tmp = cur;
      cur = nxt;
      nxt = tmp;
      i += plane;
    }
  }
}
// One weighted-Jacobi sweep out = in + omega D^-1 (r - A in) (level 0's third
// pre- and post-sweep).
template <bool L0, typename RT>
__global__ void __launch_bounds__(kBlock) k_mg_sweep(MgLevel Lk, float omega, const float* __restrict__ in,
                                                     float* __restrict__ out, const RT* __restrict__ r,
                                                     const SolveScal* ss) {
  __shared__ float lds[2][kPlaneMaxF];
  FOR_MY_TILES(Lk.ntiles) {
    const Tile t = Lk.tiles[ti];
    if (ss[t.rep].done) continue;
    const MgRep m = Lk.reps[t.rep];
    const Geo<L0> G = geo_of<L0>(m);
    const OpU<RT> op{in, Lk.dinv, r};
    mg_plane(G, t, m.tx, m.off, lds, op,
             [&](int, long long i, float v, float s, const CtrDR<RT>& c) {
               out[i] = (1.f - omega) * v + omega * c.dinv * ((float)c.r + s);
             });
  }
}

template <bool L0, typename RT, typename ST>
__global__ void __launch_bounds__(kBlock) k_mg_post2(MgLevel Lk, float omega, const float* __restrict__ in,
                                                     const RT* __restrict__ r, SolverBufsT<ST> sb) {
  __shared__ double lds4[4];
  __shared__ float lds[2][kPlaneMaxF];
  FOR_MY_TILES(Lk.ntiles) {
    const Tile t = Lk.tiles[ti];
    if (sb.ss[t.rep].done) continue;
    const MgRep m = Lk.reps[t.rep];
    const Geo<L0> G = geo_of<L0>(m);
    double rz = 0.0;
    // level 0 reads the FP64 residual (for r.z): the cycle works on r sc
    const double sc = L0 ? sb.ss[t.rep].sc : 1.0, isc = L0 ? sb.ss[t.rep].isc : 1.0;
    {
      const OpU<RT> op{in, Lk.dinv, r};
      mg_plane(G, t, m.tx, m.off, lds, op,
               [&](int, long long i, float u4, float s, const CtrDR<RT>& c) {
                 const float rs = L0 ? (float)((double)c.r * sc) : (float)c.r;
                 const float u5 = (1.f - omega) * u4 + omega * c.dinv * (rs + s);
                 if (L0) {
                   sb.z32[i] = u5;
                   rz += (double)c.r * ((double)u5 * isc);
                 } else {
                   Lk.u[i] = u5;
                 }
               });
    }
    if (L0) {
      // level 0: partial r.z of this tile (finished by the RED_RZ reduce)
      rz = block_sum(rz, lds4);
      store_partials(sb.partial + (size_t)ti * 3, rz, 0.0, 0.0);
    }
  }
}

// ---- level 0: three stencil stages per pass (temporal blocking) ---------------
//
// Level 0's couplings are uniform (a), so a sweep needs only the sum of the
// six neighbours.  Each kernel below runs three dependent stencil stages over
// a tile in one pass.  A tile of tx x ty output columns (kF3Block of them)
// over [z0, z1) is extended by three rings of columns in x and y
// (EX = tx + 6, EY = ty + 6).  Stage 0 forms its values on every column from
// global memory; stage s = 1, 2, 3 on the columns of rings < 4 - s (ring 0:
// the tile's own columns), from stage s-1's values.  In the step for plane z
// the stages work on the planes z+3, z+2, z+1 and z.
//
// Each thread owns one tile column (lane layout of the other stencil
// kernels) and at most one ring column: ring columns go to the threads in
// order, ring 1 first, so that a wavefront's ring columns mostly share a ring
// and the wavefront skips the stages its ring does not need (dealt round
// robin over the wavefronts instead, every wavefront ran all three).  A column's values of the planes around the current ones (its
// own z-neighbours, and r and D^-1 of the four planes in flight) stay in the
// owner's registers; only the x/y neighbours go through LDS, one plane per
// stage, double buffered: stage s in step z reads the plane stage s-1 wrote in
// step z-1, so one barrier per step orders everything.  Values outside the
// lattice are 0, which makes the neighbour sum the sum over the existing
// faces.
//   pre:  stage 0 u1 = w0 D^-1 r; stages 1, 2 sweeps (w1, w2), u3 written to
//         level 0's u; stage 3 the residual r - A u3, summed over the 2 x 2 x 2
//         children into level 1's r.
//   post: stage 0 u3 + P e; stages 1, 2, 3 sweeps (w2, w1, w0); stage 3's
//         plane is the CG's z (FP32, scaled) and feeds its r.z partial.
// The intermediate iterates never leave the workgroup: the pre-smoothing
// reads r and D^-1 once and writes u3 and r1 (12.5 B per voxel instead of
// 40.5 B over three kernels), the post-smoothing reads u3, e, r, D^-1 and the
// stored r once and writes z (16.5 B + one stored value, instead of 44.5 B +
// one).  Ring columns are computed by every tile that needs them, with the
// same arithmetic.  The fused tiles are dealt to the XCDs in runs of about
// eight tile rows (ftile_of), so neighbouring tiles' halo reads meet in L2.
constexpr int kF3Max = 848;   // extended plane: (32 + 6)(16 + 6) = (16 + 6)(32 + 6) = 836

// Weights of a fused pass's sweeps, in stage order.
struct F3W {
  float w[3];
};

struct F3Own {
  int EX;
  int p[2];      // LDS index of the owned columns: tile column, ring column (-1: none)
  int ring1;     // ring of the ring column (1..R; R + 1: none)
  int col[2];    // column within a plane (-1: outside the lattice)
};

// Ring column k (rings 1..R in turn; each ring top row, bottom row, left and
// right column) of a tx x ty tile extended by R rings: LDS index and ring,
// or ring R + 1 if none.
__device__ inline void f3_ring_cell(int k, int tx, int ty, int R, int EX, int& p, int& ring) {
  for (int rho = 1; rho <= R; ++rho) {
    const int w = tx + 2 * rho, h = ty + 2 * rho - 2, n = 2 * w + 2 * h;
    if (k < n) {
      const int o = R - rho;   // the ring's first row and column in the extended tile
      int hx, hy;
      if (k < w) {
        hx = o + k;
        hy = o;
      } else if (k < 2 * w) {
        hx = o + k - w;
        hy = o + h + 1;
      } else if (k < 2 * w + h) {
        hx = o;
        hy = o + 1 + k - 2 * w;
      } else {
        hx = o + w - 1;
        hy = o + 1 + k - 2 * w - h;
      }
      p = hy * EX + hx;
      ring = rho;
      return;
    }
    k -= n;
  }
  p = -1;
  ring = R + 1;
}

__device__ inline F3Own f3_own(const Tile& t, const MgRep& m, int R) {
  F3Own f;
  const int tx = m.tx, ty = kF3Block / tx;
  f.EX = tx + 2 * R;
  const int q = (int)threadIdx.x;
  f.p[0] = (q / tx + R) * f.EX + q % tx + R;
  f3_ring_cell(q, tx, ty, R, f.EX, f.p[1], f.ring1);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    f.col[j] = -1;
    if (f.p[j] >= 0) {
      const int x = t.x0 + f.p[j] % f.EX - R, y = t.y0 + f.p[j] / f.EX - R;
      if (x >= 0 && x < m.nx && y >= 0 && y < m.ny) f.col[j] = x + m.nx * y;
    }
  }
  return f;
}

// Shift a plane history (index 0 the newest).  (Unrolling the steps so that
// the history slots become compile-time indices removes these moves but holds
// more registers, and measured slower; so did compile-time tile widths.)
template <int N>
__device__ inline void f3_push(float (&h)[N], float v) {
#pragma unroll
  for (int k = N - 1; k > 0; --k) h[k] = h[k - 1];
  h[0] = v;
}

// Sum of the x/y neighbours of LDS cell p in plane buffer b.
__device__ inline float f3_xy(const float* b, int p, int EX) {
  return (b[p - 1] + b[p + 1]) + (b[p - EX] + b[p + EX]);
}

// ring of slot j's column (slot 0: the tile column)
#define F3_RING(j) ((j) == 0 ? 0 : f.ring1)

// Pre-smoothing and restriction of a uniform level (level 0, or a coarser
// level whose cells are all full 2^k-cubes: coupling a 2^k) in one pass: S
// stages (S = 3 at level 0, 2 below): u1 = w[0] D^-1 r, then sweeps w[1..S-1]
// (the last one's tile cells written to u), then the residual r - A u summed
// over the 2 x 2 x 2 children into the next level's r.
template <int S>
__global__ void __launch_bounds__(kF3Block) k_mg_prefused(MgLevel Lk, MgLevel Lc, F3W w, float ascale,
                                                          const float* __restrict__ r, const SolveScal* ss) {
  __shared__ float sV[S][2][kF3Max];
  const int ti = ftile_of(Lk.nftiles, Lk.fchunk);
  if (ti < 0) return;
  const Tile t = Lk.ftiles[ti];
  if (ss[t.rep].done) return;
  const MgRep m = Lk.reps[t.rep];
  const MgRep mc = Lc.reps[t.rep];
  const F3Own f = f3_own(t, m, S);
  const int EX = f.EX, nz = m.nz, tx = m.tx;
  const float a = m.a * ascale;
  const int plane = m.nx * m.ny;   // a system's level holds < 2^31 cells
  const float* __restrict__ rS = r + m.off;
  const float* __restrict__ dS = Lk.dinv + m.off;
  float* __restrict__ uS = Lk.u + m.off;
  const int z0 = t.z0, z1 = t.z1;
  float rh[2][S + 1], dh[2][S + 1];   // r, D^-1 of planes z+S .. z (newest first)
  float hs[S][2][3];                  // stage outputs, newest first
#pragma unroll
  for (int j = 0; j < 2; ++j) {
#pragma unroll
    for (int k = 0; k <= S; ++k) rh[j][k] = dh[j][k] = 0.f;
#pragma unroll
    for (int st = 0; st < S; ++st)
#pragma unroll
      for (int k = 0; k < 3; ++k) hs[st][j][k] = 0.f;
  }
  float nr[2], nd[2];   // stage-0 operands of the next plane
  auto fetch = [&](int z) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      nr[j] = 0.f;
      nd[j] = 0.f;
      if (f.col[j] >= 0 && z >= 0 && z < nz) {
        const int i = plane * z + f.col[j];
        nr[j] = rS[i];
        nd[j] = dS[i];
      }
    }
  };
  const int lx = (int)threadIdx.x % tx, ly = (int)threadIdx.x / tx;
  const int x = t.x0 + lx, y = t.y0 + ly;
  const bool lead = ((lx | ly) & 1) == 0 && f.col[0] >= 0;
  float acc = 0.f;
  fetch(z0 - S);
  for (int zz = z0 - 2 * S; zz < z1; ++zz) {
    const int wb = (zz + 2 * S) & 1, rb = wb ^ 1;   // write this step's planes, read the last step's
    {   // stage 0 at plane zz + S
      const int z = zz + S;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (F3_RING(j) > S) continue;
        f3_push(rh[j], nr[j]);
        f3_push(dh[j], nd[j]);
        const float v = w.w[0] * nd[j] * nr[j];
        f3_push(hs[0][j], v);
        sV[0][wb][f.p[j]] = v;
      }
      if (z + 1 <= z1 + S - 1) fetch(z + 1);
    }
#pragma unroll
    for (int st = 1; st < S; ++st) {   // sweep st at plane zz + S - st (rings 0 .. S - st)
      const int z = zz + S - st;
      if (z >= z0 - (S - st) && z <= z1 - 1 + (S - st)) {
        const bool in = z >= 0 && z < nz;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (F3_RING(j) > S - st) continue;
          const float nb = f3_xy(sV[st - 1][rb], f.p[j], EX) + (hs[st - 1][j][2] + hs[st - 1][j][0]);
          float v = (1.f - w.w[st]) * hs[st - 1][j][1] + w.w[st] * dh[j][st] * (rh[j][st] + a * nb);
          const bool ok = in && f.col[j] >= 0;
          v = ok ? v : 0.f;
          if (st == S - 1 && j == 0 && ok && z >= z0 && z < z1) uS[plane * z + f.col[0]] = v;
          f3_push(hs[st][j], v);
          sV[st][wb][f.p[j]] = v;
        }
      }
    }
    if (zz >= z0) {   // stage S at plane zz: r - A u, summed into the next level's r
      const int z = zz;
      float res = 0.f;
      if (f.col[0] >= 0) {
        const float nb = f3_xy(sV[S - 1][rb], f.p[0], EX) + (hs[S - 1][0][2] + hs[S - 1][0][0]);
        res = rh[0][S] - hs[S - 1][0][1] * __builtin_amdgcn_rcpf(dh[0][S]) + a * nb;
      }
      float q = res + __shfl_xor(res, 1, 64);
      q = q + __shfl_xor(q, tx, 64);
      acc += q;
      if ((z & 1) || z + 1 == nz) {
        if (lead)
          Lc.r[mc.off + (x >> 1) + (long long)mc.nx * ((y >> 1) + (long long)mc.ny * (z >> 1))] = acc;
        acc = 0.f;
      }
    }
    __syncthreads();
  }
}

// Prolongation and post-smoothing of a uniform level in one pass: stage 0
// u + P e (e the next level's correction), then S sweeps w[0..S-1].  ZOUT
// (level 0): the last sweep is the CG's z (FP32, scaled) and feeds the tile's
// r.z partial; otherwise it is written to out.
template <int S, bool ZOUT, typename RT, typename ST>
__global__ void __launch_bounds__(kF3Block) k_mg_postfused(MgLevel Lk, MgLevel Lc, const float* __restrict__ e,
                                                           F3W w, float ascale, const float* __restrict__ r,
                                                           const RT* __restrict__ r64, float* __restrict__ out,
                                                           SolverBufsT<ST> sb) {
  __shared__ double lds8[kF3Block / 64];
  __shared__ float sV[S][2][kF3Max];
  __shared__ float sE[4][kF3Max];   // coarse plane Z interpolated in x, y (slot Z & 3); owner-private
  const int ti = ftile_of(Lk.nftiles, Lk.fchunk);
  if (ti < 0) return;
  const Tile t = Lk.ftiles[ti];
  if (sb.ss[t.rep].done) return;
  const MgRep m = Lk.reps[t.rep];
  const MgRep mc = Lc.reps[t.rep];
  const F3Own f = f3_own(t, m, S);
  const int EX = f.EX, nz = m.nz;
  const float a = m.a * ascale;
  const int plane = m.nx * m.ny;
  const float* __restrict__ rS = r + m.off;
  const float* __restrict__ dS = Lk.dinv + m.off;
  const float* __restrict__ uS = Lk.u + m.off;
  const int z0 = t.z0, z1 = t.z1;
  const double isc = ZOUT ? sb.ss[t.rep].isc : 1.0;
  const float* __restrict__ eb = e + mc.off;
  const int csz = mc.nx * mc.ny;
  // E of coarse plane Z at the owned columns
  auto make_e = [&](int Z) {
    const float* b = eb + csz * Z;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (f.col[j] < 0) continue;
      int Ix, Jx, Iy, Jy;
      float wx, wy;
      lin_axis(t.x0 + f.p[j] % EX - S, m.nx, mc.nx, Ix, Jx, wx);
      lin_axis(t.y0 + f.p[j] / EX - S, m.ny, mc.ny, Iy, Jy, wy);
      const float g0 = b[Iy * mc.nx + Ix], g1 = b[Iy * mc.nx + Jx];
      const float g2 = b[Jy * mc.nx + Ix], g3 = b[Jy * mc.nx + Jx];
      const float e0 = (1.f - wx) * g0 + wx * g1;
      const float e1 = (1.f - wx) * g2 + wx * g3;
      sE[Z & 3][f.p[j]] = (1.f - wy) * e0 + wy * e1;
    }
  };
  int ehi = -(1 << 20);   // highest coarse plane in sE
  float rh[2][S + 1], dh[2][S + 1];
  float hs[S][2][3];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
#pragma unroll
    for (int k = 0; k <= S; ++k) rh[j][k] = dh[j][k] = 0.f;
#pragma unroll
    for (int st = 0; st < S; ++st)
#pragma unroll
      for (int k = 0; k < 3; ++k) hs[st][j][k] = 0.f;
  }
  float nu[2], nr[2], nd[2];
  auto fetch = [&](int z) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      nu[j] = 0.f;
      nr[j] = 0.f;
      nd[j] = 0.f;
      if (f.col[j] >= 0 && z >= 0 && z < nz) {
        const int i = plane * z + f.col[j];
        nu[j] = uS[i];
        nr[j] = rS[i];
        nd[j] = dS[i];
      }
    }
  };
  RT r64n = (RT)0;   // the stored r of the tile column, next output plane
  auto fetch64 = [&](int z) {
    if (ZOUT && f.col[0] >= 0 && z >= z0 && z < z1) r64n = r64[m.off + plane * z + f.col[0]];
  };
  double rz = 0.0;
  fetch(z0 - S);
  for (int zz = z0 - 2 * S; zz < z1; ++zz) {
    const int wb = (zz + 2 * S) & 1, rb = wb ^ 1;
    const RT r64c = r64n;
    fetch64(zz + 1);
    {   // stage 0 at plane zz + S: u + P e
      const int z = zz + S;
      int Iz = 0, Jz = 0;
      float wz = 0.f;
      const bool in = z >= 0 && z < nz;
      if (in) {
        lin_axis(z, nz, mc.nz, Iz, Jz, wz);
        if (ehi < min(Iz, Jz) - 1) ehi = min(Iz, Jz) - 1;
        while (ehi < max(Iz, Jz)) make_e(++ehi);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (F3_RING(j) > S) continue;
        f3_push(rh[j], nr[j]);
        f3_push(dh[j], nd[j]);
        // branch-free: with Jz == Iz, wz is 0 and the sum is eI exactly
        const float eI = sE[Iz & 3][f.p[j]], eJ = sE[Jz & 3][f.p[j]];
        float v = nu[j] + ((1.f - wz) * eI + wz * eJ);
        v = (in && f.col[j] >= 0) ? v : 0.f;
        f3_push(hs[0][j], v);
        sV[0][wb][f.p[j]] = v;
      }
      if (z + 1 <= z1 + S - 1) fetch(z + 1);
    }
#pragma unroll
    for (int st = 1; st < S; ++st) {   // sweep st at plane zz + S - st (rings 0 .. S - st)
      const int z = zz + S - st;
      if (z >= z0 - (S - st) && z <= z1 - 1 + (S - st)) {
        const bool in = z >= 0 && z < nz;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (F3_RING(j) > S - st) continue;
          const float nb = f3_xy(sV[st - 1][rb], f.p[j], EX) + (hs[st - 1][j][2] + hs[st - 1][j][0]);
          float v = (1.f - w.w[st - 1]) * hs[st - 1][j][1] + w.w[st - 1] * dh[j][st] * (rh[j][st] + a * nb);
          v = (in && f.col[j] >= 0) ? v : 0.f;
          f3_push(hs[st][j], v);
          sV[st][wb][f.p[j]] = v;
        }
      }
    }
    if (zz >= z0 && f.col[0] >= 0) {   // the last sweep at plane zz
      const float nb = f3_xy(sV[S - 1][rb], f.p[0], EX) + (hs[S - 1][0][2] + hs[S - 1][0][0]);
      const float v = (1.f - w.w[S - 1]) * hs[S - 1][0][1] + w.w[S - 1] * dh[0][S] * (rh[0][S] + a * nb);
      if constexpr (ZOUT) {
        sb.z32[m.off + plane * zz + f.col[0]] = v;
        rz += (double)r64c * ((double)v * isc);
      } else {
        out[m.off + plane * zz + f.col[0]] = v;
      }
    }
    __syncthreads();
  }
  if constexpr (ZOUT) {   // the tile's r.z partial (fixed order)
    for (int o = 32; o > 0; o >>= 1) rz += __shfl_xor(rz, o, 64);
    if ((threadIdx.x & 63) == 0) lds8[threadIdx.x >> 6] = rz;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tsum = 0.0;
      for (int k = 0; k < kF3Block / 64; ++k) tsum += lds8[k];
      store_partials(sb.partial + (size_t)ti * 3, tsum, 0.0, 0.0);
    }
  }
}

#undef F3_RING

// ---- coarse levels: one workgroup per system, in LDS --------------------------

struct CoarseLevel {
  Geo<false> G;
  int n;
  float rnx, rny;   // 1/nx, 1/ny (coordinates without integer division)
  // LDS: two Jacobi iterates and the residual, [ua | ub | r]; D^-1 and the
  // couplings to the +x/+y/+z neighbour (0 at the edge), [D^-1 | gx | gy | gz],
  // the level's part of the system's precomputed block copied into LDS.
  float *ua, *ub, *r, *dinv, *gx, *gy, *gz;
};

// Level j of a system's coarse solve (LDS pointers and geometry).
__device__ inline CoarseLevel coarse_level(const MgCoarseRep& cr, float* lds, int j, float a) {
  CoarseLevel L;
  L.G.nx = cr.dims[j][0];
  L.G.ny = cr.dims[j][1];
  L.G.nz = cr.dims[j][2];
  L.G.k = cr.kc + j;
  L.G.n0x = cr.n0[0];
  L.G.n0y = cr.n0[1];
  L.G.n0z = cr.n0[2];
  L.G.a = a;
  L.n = L.G.nx * L.G.ny * L.G.nz;
  L.rnx = 1.f / (float)L.G.nx;
  L.rny = 1.f / (float)L.G.ny;
  L.ua = lds + cr.pre_len + cr.lds_off[j];
  L.ub = L.ua + L.n;
  L.r = L.ub + L.n;
  L.dinv = lds + cr.pre_lev[j];
  L.gx = L.dinv + L.n;
  L.gy = L.gx + L.n;
  L.gz = L.gy + L.n;
  return L;
}

// Coordinates of cell t (t < 2^13): the float quotient (t + 1/2) / nx is at
// least 1/(2 nx) from an integer and its rounding error far below that; the
// fix-ups only guard the argument.
__device__ inline void cell_xyz(const CoarseLevel& L, int t, int& x, int& y, int& z) {
  int q = (int)(((float)t + 0.5f) * L.rnx);
  x = t - q * L.G.nx;
  if (x < 0) {
    --q;
    x += L.G.nx;
  } else if (x >= L.G.nx) {
    ++q;
    x -= L.G.nx;
  }
  z = (int)(((float)q + 0.5f) * L.rny);
  y = q - z * L.G.ny;
  if (y < 0) {
    --z;
    y += L.G.ny;
  } else if (y >= L.G.ny) {
    ++z;
    y -= L.G.ny;
  }
}

// Neighbours of cell t in LDS, branch-free: indices clamped to t where a
// face is missing and the coupling of a missing face 0, so all reads of a
// stencil are issued together instead of one per taken branch.  The stored
// +x/+y/+z couplings are already 0 at the upper edges.
struct CoarseNb {
  int xm, xp, ym, yp, zm, zp;   // neighbour indices (t where absent)
  float fxm, fym, fzm;          // 1 where the lower neighbour exists, else 0
};

__device__ inline CoarseNb coarse_nb(const CoarseLevel& L, int t, int x, int y, int z) {
  const int nx = L.G.nx, plane = nx * L.G.ny;
  CoarseNb b;
  b.xm = x > 0 ? t - 1 : t;
  b.xp = x + 1 < nx ? t + 1 : t;
  b.ym = y > 0 ? t - nx : t;
  b.yp = y + 1 < L.G.ny ? t + nx : t;
  b.zm = z > 0 ? t - plane : t;
  b.zp = z + 1 < L.G.nz ? t + plane : t;
  b.fxm = x > 0 ? 1.f : 0.f;
  b.fym = y > 0 ? 1.f : 0.f;
  b.fzm = z > 0 ? 1.f : 0.f;
  return b;
}

// sum_J g_IJ V(J) over the existing neighbours, in the order -x, +x, -y, +y, -z, +z
template <typename VF>
__device__ inline float lds_nbsum_f(const CoarseLevel& L, const CoarseNb& b, int t, VF V) {
  const float gxm = b.fxm * L.gx[b.xm], gym = b.fym * L.gy[b.ym], gzm = b.fzm * L.gz[b.zm];
  float s = gxm * V(b.xm);
  s += L.gx[t] * V(b.xp);
  s += gym * V(b.ym);
  s += L.gy[t] * V(b.yp);
  s += gzm * V(b.zm);
  s += L.gz[t] * V(b.zp);
  return s;
}

__device__ inline float lds_nbsum(const CoarseLevel& L, const float* v, int t, int x, int y, int z) {
  const CoarseNb b = coarse_nb(L, t, x, y, z);
  return lds_nbsum_f(L, b, t, [&](int j) { return v[j]; });
}

// The cells of a level dealt to the workgroup's threads: t = thread + m * block.
#define FOR_MY_CELLS(L, t) for (int t = (int)threadIdx.x; t < (L).n; t += kCoarseThreads)

// One phase over the n cells of a level: value(t) of the cells a thread
// holds is formed first (their LDS reads in flight together; tail slots repeat
// cell n-1), then store(t, value) for the cells that exist; batches of four
// cells per thread.  A phase reads no array it stores to, other than a cell's
// own entry.
template <int M, typename VF, typename SF>
__device__ inline void coarse_phase_m(int base, int n, VF value, SF store) {
  float v[M];
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = value(min(base + (int)threadIdx.x + m * kCoarseThreads, n - 1));
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int t = base + (int)threadIdx.x + m * kCoarseThreads;
    if (t < n) store(t, v[m]);
  }
}

template <typename VF, typename SF>
__device__ inline void coarse_phase(int n, VF value, SF store) {
  if (n <= kCoarseThreads) {
    if ((int)threadIdx.x < n) store((int)threadIdx.x, value((int)threadIdx.x));
  } else if (n <= 2 * kCoarseThreads) {
    coarse_phase_m<2>(0, n, value, store);
  } else {
    for (int b = 0; b < n; b += 4 * kCoarseThreads) coarse_phase_m<4>(b, n, value, store);
  }
}

// One weighted-Jacobi sweep, src -> dst (different buffers, so no barrier
// between reading and writing).
__device__ inline void lds_sweep(const CoarseLevel& L, const float* src, float* dst, float omega) {
  coarse_phase(
      L.n,
      [&](int t) {
        int x, y, z;
        cell_xyz(L, t, x, y, z);
        return (1.f - omega) * src[t] + omega * L.dinv[t] * (L.r[t] + lds_nbsum(L, src, t, x, y, z));
      },
      [&](int t, float v) { dst[t] = v; });
}

// Once per solve, one workgroup per system: coarse reaction terms of the
// one-workgroup levels (summed from level kc, kept in the LDS ua slots), then
// each level's couplings and D^-1 into the system's precomputed block.
__global__ void __launch_bounds__(kCoarseThreads) k_mg_coarse_prep(const MgCoarseRep* coarse,
                                                                   const float* const* lev_c,
                                                                   float* __restrict__ pre) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  const int rep = blockIdx.x;
  const MgCoarseRep& cr = coarse[rep];
  const float a = cr.a;
  const int J = cr.nlev;
  {
    const CoarseLevel L = coarse_level(cr, lds, 0, a);
    const float* gc = lev_c[cr.kc] + cr.off_kc;
    for (int t = threadIdx.x; t < L.n; t += kCoarseThreads) L.ua[t] = gc[t];
  }
  __syncthreads();
  for (int j = 1; j < J; ++j) {
    const CoarseLevel F = coarse_level(cr, lds, j - 1, a);
    const CoarseLevel C = coarse_level(cr, lds, j, a);
    for (int t = threadIdx.x; t < C.n; t += kCoarseThreads) {
      int X, Y, Z;
      cell_xyz(C, t, X, Y, Z);
      float s = 0.f;
      for (int dz = 0; dz < 2 && 2 * Z + dz < F.G.nz; ++dz)
        for (int dy = 0; dy < 2 && 2 * Y + dy < F.G.ny; ++dy)
          for (int dx = 0; dx < 2 && 2 * X + dx < F.G.nx; ++dx)
            s += F.ua[(2 * X + dx) + F.G.nx * ((2 * Y + dy) + F.G.ny * (2 * Z + dz))];
      C.ua[t] = s;
    }
    __syncthreads();
  }
  for (int j = 0; j < J; ++j) {
    const CoarseLevel L = coarse_level(cr, lds, j, a);
    float* g = pre + cr.pre_off + cr.pre_lev[j];
    for (int t = threadIdx.x; t < L.n; t += kCoarseThreads) {
      int x, y, z;
      cell_xyz(L, t, x, y, z);
      g[t] = 1.f / (L.ua[t] + L.G.gsum(x, y, z));
      g[L.n + t] = x + 1 < L.G.nx ? L.G.gx(x, y, z) : 0.f;
      g[2 * L.n + t] = y + 1 < L.G.ny ? L.G.gy(x, y, z) : 0.f;
      g[3 * L.n + t] = z + 1 < L.G.nz ? L.G.gz(x, y, z) : 0.f;
    }
  }
}

// The V-cycle of levels kc.. of one system in LDS (one workgroup per system),
// the same cycle as the multi-workgroup levels: two sweeps, restriction by
// aggregate sums, ..., the one-cell level solved exactly, cell-centred linear
// prolongation, two sweeps; the correction of level kc is written to that
// level's global u.  Every level's final iterate is left in its ua.
__global__ void __launch_bounds__(kCoarseThreads) k_mg_coarse(const MgCoarseRep* coarse,
                                                              float wa, float wb,
                                                              const float* const* lev_r,
                                                              float* const* lev_u,
                                                              const float* __restrict__ pre,
                                                              const SolveScal* ss) {
  extern __shared__ __attribute__((aligned(16))) float lds[];
  __shared__ MgCoarseRep s_cr;
  const int rep = blockIdx.x;
  // the system's descriptor into LDS (every later phase reads it there
  // instead of from global memory)
  {
    static_assert(sizeof(MgCoarseRep) % 4 == 0 && sizeof(MgCoarseRep) / 4 <= kCoarseThreads, "descriptor copy");
    constexpr int nw = (int)(sizeof(MgCoarseRep) / 4);
    const int* src = reinterpret_cast<const int*>(coarse + rep);
    const int v = (int)threadIdx.x < nw ? src[threadIdx.x] : 0;
    if (ss[rep].done) return;
    if ((int)threadIdx.x < nw) reinterpret_cast<int*>(&s_cr)[threadIdx.x] = v;
  }
  __syncthreads();
  const MgCoarseRep& cr = s_cr;
  const float a = cr.a;
  const int J = cr.nlev;
  // r of level kc, and the precomputed block (D^-1 and the couplings of every
  // level), into LDS; each pass issues all of its global loads before its
  // first LDS store (one memory latency per pass, not one per element)
  {
    const CoarseLevel L = coarse_level(cr, lds, 0, a);
    const float* gr = cr.r_kc;
    float rv[kCoarseMaxCellsPerThread];
#pragma unroll
    for (int m = 0; m < kCoarseMaxCellsPerThread; ++m) {
      const int t = (int)threadIdx.x + m * kCoarseThreads;
      rv[m] = gr[min(t, L.n - 1)];
    }
    const float4* src = reinterpret_cast<const float4*>(pre + cr.pre_off);
    float4* dst = reinterpret_cast<float4*>(lds);
    const int n4 = cr.pre_len >> 2;
    constexpr int kBatch = 6;
    for (int b = 0; b < n4; b += kBatch * kCoarseThreads) {
      float4 v[kBatch];
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int i = b + (int)threadIdx.x + k * kCoarseThreads;
        v[k] = src[min(i, n4 - 1)];
      }
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int i = b + (int)threadIdx.x + k * kCoarseThreads;
        if (i < n4) dst[i] = v[k];
      }
    }
#pragma unroll
    for (int m = 0; m < kCoarseMaxCellsPerThread; ++m) {
      const int t = (int)threadIdx.x + m * kCoarseThreads;
      if (t < L.n) L.r[t] = rv[m];
    }
  }
  __syncthreads();
  // down: u2 of the two sweeps from zero (u1 = w D^-1 r, formed on the fly at
  // the neighbours), then the aggregate sums of r - A u2
  for (int j = 0; j + 1 < J; ++j) {
    const CoarseLevel L = coarse_level(cr, lds, j, a);
    coarse_phase(
        L.n,
        [&](int t) {
          int x, y, z;
          cell_xyz(L, t, x, y, z);
          const CoarseNb nb = coarse_nb(L, t, x, y, z);
          const float s = lds_nbsum_f(L, nb, t, [&](int i) { return L.dinv[i] * L.r[i]; });
          const float d = L.dinv[t], rr = L.r[t];
          const float u1 = wa * d * rr;
          return (1.f - wb) * u1 + wb * d * (rr + wa * s);
        },
        [&](int t, float v) { L.ua[t] = v; });
    __syncthreads();
    const CoarseLevel C = coarse_level(cr, lds, j + 1, a);
    FOR_MY_CELLS(C, t) {
      int X, Y, Z;
      cell_xyz(C, t, X, Y, Z);
      // the up to eight children, every one evaluated (absent ones at a
      // clamped index) and weighted 0 or 1, in the order x, then y, then z
      float s = 0.f;
#pragma unroll
      for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const bool in = 2 * X + dx < L.G.nx && 2 * Y + dy < L.G.ny && 2 * Z + dz < L.G.nz;
            const int x = in ? 2 * X + dx : 2 * X, y = in ? 2 * Y + dy : 2 * Y, z = in ? 2 * Z + dz : 2 * Z;
            const int f = x + L.G.nx * (y + L.G.ny * z);
            const float res = L.r[f] - L.ua[f] / L.dinv[f] + lds_nbsum(L, L.ua, f, x, y, z);
            s += in ? res : 0.f;
          }
      C.r[t] = s;
    }
    __syncthreads();
  }
  // coarsest: one cell and no faces, so u = r / c exactly; larger: sweeps
  {
    const CoarseLevel L = coarse_level(cr, lds, J - 1, a);
    FOR_MY_CELLS(L, t) L.ua[t] = L.dinv[t] * L.r[t];
    __syncthreads();
    if (L.n > 1) {
      for (int it = 0; it < 15; ++it) {
        lds_sweep(L, L.ua, L.ub, wa);
        __syncthreads();
        lds_sweep(L, L.ub, L.ua, wb);
        __syncthreads();
      }
    }
  }
  // up: u3 = u2 + P e, two sweeps (the last of level kc straight to global)
  for (int j = J - 2; j >= 0; --j) {
    const CoarseLevel L = coarse_level(cr, lds, j, a);
    const CoarseLevel C = coarse_level(cr, lds, j + 1, a);
    coarse_phase(L.n, [&](int t) {
      int x, y, z;
      cell_xyz(L, t, x, y, z);
      int Ix, Jx, Iy, Jy, Iz, Jz;
      float wx, wy, wz;
      lin_axis(x, L.G.nx, C.G.nx, Ix, Jx, wx);
      lin_axis(y, L.G.ny, C.G.ny, Iy, Jy, wy);
      lin_axis(z, L.G.nz, C.G.nz, Iz, Jz, wz);
      const int sy = C.G.nx, sz = C.G.nx * C.G.ny;
      const float* e = C.ua;
      // x first along each coarse row, then y, then z (the global levels' order)
      const float r00 = (1.f - wx) * e[Iz * sz + Iy * sy + Ix] + wx * e[Iz * sz + Iy * sy + Jx];
      const float r01 = (1.f - wx) * e[Iz * sz + Jy * sy + Ix] + wx * e[Iz * sz + Jy * sy + Jx];
      const float r10 = (1.f - wx) * e[Jz * sz + Iy * sy + Ix] + wx * e[Jz * sz + Iy * sy + Jx];
      const float r11 = (1.f - wx) * e[Jz * sz + Jy * sy + Ix] + wx * e[Jz * sz + Jy * sy + Jx];
      const float p0 = (1.f - wy) * r00 + wy * r01;
      const float p1 = (1.f - wy) * r10 + wy * r11;
      return L.ua[t] + ((1.f - wz) * p0 + wz * p1);
    }, [&](int t, float v) { L.ua[t] = v; });
    __syncthreads();
    lds_sweep(L, L.ua, L.ub, wb);
    __syncthreads();
    if (j > 0) {
      lds_sweep(L, L.ub, L.ua, wa);
      __syncthreads();
    } else {
      lds_sweep(L, L.ub, cr.u_kc, wa);
    }
  }
  if (J == 1) {   // level kc is the one-cell level itself
    const CoarseLevel L = coarse_level(cr, lds, 0, a);
    float* gu = cr.u_kc;
    FOR_MY_CELLS(L, t) gu[t] = L.ua[t];
  }
}

// ---- launchers -------------------------------------------------------------

hipError_t mg_set_coarse_lds(int bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_mg_coarse, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_mg_coarse_prep, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <typename T>
void launch_mg_prepare(hipStream_t s, const Work& w, const MgBufs& mg, const T* c) {
  // level 0's D^-1 comes with level 1's c (k_mg_coarsen<true>); a level 1 with
  // no restriction tiles would leave it to k_mg_prep0
  if (mg.lev[0].ntiles && !mg.lev[1].nrtiles)
    hca_launch(k_mg_prep0<T>, dim3(grid_tiles(mg.lev[0].ntiles, w.max_blocks)), dim3(kBlock), 0, s, mg.lev[0], c);
  for (int k = 0; k < mg.nlev_glob; ++k) {
    const MgLevel& Lc = mg.lev[k + 1];
    if (!Lc.nrtiles) continue;
    if (k == 0)
      hca_launch(k_mg_coarsen<true, T>, dim3(grid_tiles(Lc.nrtiles, w.max_blocks)), dim3(kBlock), 0, s, mg.lev[k], Lc, c);
    else
      hca_launch(k_mg_coarsen<false, T>, dim3(grid_tiles(Lc.nrtiles, w.max_blocks)), dim3(kBlock), 0, s, mg.lev[k], Lc, c);
  }
  hca_launch(k_mg_coarse_prep, dim3(w.nreps), dim3(kCoarseThreads), mg.coarse_lds_bytes, s, mg.coarse,
             (const float* const*)mg.lev_c, mg.coarse_pre);
}

template <typename T>
void launch_mg_vcycle(hipStream_t s, const Work& w, const MgBufs& mg, const SolverBufsT<T>& sb,
                      MgHook hook, void* hctx) {
  // levels >= 1: pre-sweeps with weights (wa, wb), post-sweeps with (wb, wa);
  // level 0: three sweeps (w0[0], w0[1], w0[2]) before, reversed after
  const float wa = mg.w_a, wb = mg.w_b;
  const float* w0 = mg.w0;
  const SolveScal* ss = sb.ss;
  auto H = [&](int seg, int begin) {
    if (hook) hook(hctx, seg, begin);
  };
  // a level's correction: its u, or its ualt where its post-smoothing ran fused
  auto corr = [&](int k) -> const float* {
    return (mg.fused && k < mg.nlev_glob && mg.lev[k].nftiles) ? mg.lev[k].ualt : mg.lev[k].u;
  };
  if (mg.fused) {
    const MgLevel& L = mg.lev[0];
    const MgLevel& C = mg.lev[1];
    H(MG_PRE3_0, 1);
    hca_launch(k_mg_prefused<3>, dim3(grid_ftiles(L.nftiles, L.fchunk)), dim3(kF3Block), 0, s, L, C,
               F3W{{w0[0], w0[1], w0[2]}}, 1.f, (const float*)sb.r32, ss);
    H(MG_PRE3_0, 0);
  } else {
    const MgLevel& L = mg.lev[0];
    const MgLevel& C = mg.lev[1];
    H(MG_PRE0, 1);
    hca_launch((k_mg_pre<true, float>), dim3(grid_tiles(L.ntiles, w.max_blocks)), dim3(kBlock), 0, s, L, w0[0],
               w0[1], (const float*)sb.r32, L.ualt, ss);
    H(MG_PRE0, 0);
    H(MG_SWEEP0, 1);
    hca_launch((k_mg_sweep<true, float>), dim3(grid_tiles(L.ntiles, w.max_blocks)), dim3(kBlock), 0, s, L, w0[2],
               (const float*)L.ualt, L.u, (const float*)sb.r32, ss);
    H(MG_SWEEP0, 0);
    H(MG_RESTRICT0, 1);
    hca_launch((k_mg_restrict<true, float>), dim3(grid_tiles(L.ntiles, w.max_blocks)), dim3(kBlock), 0, s, L, C,
                       (const float*)sb.r32, ss);
    H(MG_RESTRICT0, 0);
  }
  if (mg.nlev_glob > 1) {
    H(MG_DOWN, 1);
    for (int k = 1; k < mg.nlev_glob; ++k) {
      const MgLevel& L = mg.lev[k];
      const MgLevel& C = mg.lev[k + 1];
      if (!L.ntiles) continue;
      if (mg.fused && L.nftiles) {
        hca_launch(k_mg_prefused<2>, dim3(grid_ftiles(L.nftiles, L.fchunk)), dim3(kF3Block), 0, s, L, C,
                   F3W{{wa, wb, 0.f}}, (float)(1 << k), (const float*)L.r, ss);
        continue;
      }
      hca_launch((k_mg_pre<false, float>), dim3(grid_tiles(L.ntiles, w.max_blocks)), dim3(kBlock), 0, s, L, wa, wb,
                 (const float*)L.r, L.u, ss);
      hca_launch((k_mg_restrict<false, float>), dim3(grid_tiles(L.ntiles, w.max_blocks)), dim3(kBlock), 0, s, L, C,
                 (const float*)L.r, ss);
    }
    H(MG_DOWN, 0);
  }
  H(MG_COARSE, 1);
  hca_launch(k_mg_coarse, dim3(w.nreps), dim3(kCoarseThreads), mg.coarse_lds_bytes, s, mg.coarse, wa, wb,
             (const float* const*)mg.lev_r, (float* const*)mg.lev_u, (const float*)mg.coarse_pre, ss);
  H(MG_COARSE, 0);
  if (mg.nlev_glob > 1) {
    H(MG_UP, 1);
    for (int k = mg.nlev_glob - 1; k >= 1; --k) {
      const MgLevel& L = mg.lev[k];
      const MgLevel& C = mg.lev[k + 1];
      if (!L.ntiles) continue;
      if (mg.fused && L.nftiles) {
        hca_launch((k_mg_postfused<2, false, T, T>), dim3(grid_ftiles(L.nftiles, L.fchunk)), dim3(kF3Block), 0, s,
                   L, C, corr(k + 1), F3W{{wb, wa, 0.f}}, (float)(1 << k), (const float*)L.r, (const T*)nullptr,
                   L.ualt, sb);
        continue;
      }
      hca_launch((k_mg_post1<false, float>), dim3(grid_tiles(L.ntiles, w.max_blocks)), dim3(kBlock), 0, s, L, C,
                 corr(k + 1), wb, (const float*)L.r, ss);
      hca_launch((k_mg_post2<false, float, T>), dim3(grid_tiles(L.ntiles, w.max_blocks)), dim3(kBlock), 0, s, L, wa,
                 (const float*)L.ualt, (const float*)L.r, sb);
    }
    H(MG_UP, 0);
  }
  if (mg.fused) {
    const MgLevel& L = mg.lev[0];
    const MgLevel& C = mg.lev[1];
    H(MG_POST3_0, 1);
    hca_launch((k_mg_postfused<3, true, T, T>), dim3(grid_ftiles(L.nftiles, L.fchunk)), dim3(kF3Block), 0, s, L,
               C, corr(1), F3W{{w0[2], w0[1], w0[0]}}, 1.f, (const float*)sb.r32, (const T*)sb.r,
               (float*)nullptr, sb);
    H(MG_POST3_0, 0);
    launch_cg_reduce(s, w, sb, RED_RZF, 0.0, 0);
  } else {
    const MgLevel& L = mg.lev[0];
    const MgLevel& C = mg.lev[1];
    H(MG_POST1_0, 1);
    hca_launch((k_mg_post1<true, float>), dim3(grid_tiles(L.ntiles, w.max_blocks)), dim3(kBlock), 0, s, L, C,
               corr(1), w0[2], (const float*)sb.r32, ss);
    H(MG_POST1_0, 0);
    H(MG_SWEEP0, 1);
    hca_launch((k_mg_sweep<true, float>), dim3(grid_tiles(L.ntiles, w.max_blocks)), dim3(kBlock), 0, s, L, w0[1],
               (const float*)L.ualt, L.u, (const float*)sb.r32, ss);
    H(MG_SWEEP0, 0);
    H(MG_POST2_0, 1);
    hca_launch((k_mg_post2<true, T, T>), dim3(grid_tiles(L.ntiles, w.max_blocks)), dim3(kBlock), 0, s, L, w0[0],
               (const float*)L.u, (const T*)sb.r, sb);
    H(MG_POST2_0, 0);
    launch_cg_reduce(s, w, sb, RED_RZ, 0.0, 0);
  }
}

template void launch_mg_prepare<double>(hipStream_t, const Work&, const MgBufs&, const double*);
template void launch_mg_prepare<float>(hipStream_t, const Work&, const MgBufs&, const float*);
template void launch_mg_vcycle<double>(hipStream_t, const Work&, const MgBufs&,
                                       const SolverBufsT<double>&, MgHook, void*);
template void launch_mg_vcycle<float>(hipStream_t, const Work&, const MgBufs&,
                                      const SolverBufsT<float>&, MgHook, void*);

}  // namespace hca
