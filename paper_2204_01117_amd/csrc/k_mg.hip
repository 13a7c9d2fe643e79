// Geometric multigrid V-cycle used as the CG preconditioner.
//
// Cell-centred hierarchy: every axis of at least 4 cells is halved (an odd
// axis of n cells gets ceil(n/2) coarse cells, the last one with a single
// child); levels stop at <= 64 cells (or when no axis halves).
// Prolongation P is trilinear between cell centres (per halved axis: 3/4 of
// the parent and 1/4 of the parent's neighbour on the child's side; past a
// domain side the neighbour is the parent's mirror image, + for a Neumann
// side and - for an outlet, where the correction vanishes).  Restriction is
// its transpose R = P^T / m (m = children per coarse cell), so interior
// weights are (1, 3, 3, 1)/8 per halved axis.  Coarse operators are the
// 7-point stencil re-discretised with the coarse spacing (weights / 4 per
// halved axis) and the same boundary rows.  Smoothing: one damped-Jacobi
// sweep before (from zero) and one after the coarse correction, so the
// V-cycle is a fixed symmetric positive-definite operator, as PCG requires.
// The coarsest level is solved with its exact dense inverse (<= 512 cells)
// or, failing that, with a fixed number of Jacobi sweeps.
//
// Kernels of one application: restrict level 0 -> 1 (block 0 also decides
// whether the solve has finished), restrict down to the first small level,
// one single-workgroup kernel for all small levels, prolongate + smooth back
// up, and the fine-level prolongation + smoothing that writes z and the
// partials of r.z.  The level kernels stage their tiles in LDS.
#include <cmath>
#include <cstdlib>
#include <vector>

#include "pressure_common.h"

namespace uf {

constexpr int kMgMaxLevels = 16;
constexpr int kTailThreads = 1024;
constexpr int kDenseMax = 512;           // largest coarsest level with an exact inverse
constexpr long long kCoarsestCells = 64; // coarsening stops at levels this small
constexpr int kCoarseSweeps = 10;        // Jacobi sweeps when there is no exact inverse
// Jacobi weight, chosen by PCG iteration counts (0.8 and 0.9 within 10%).
constexpr double kJacobiOmega = 0.8;

template <class T>
struct MgLvl {
  Layout L;
  T w[3];
  T omd_in;   // om / D of an interior cell
  int c[3];   // axis halved towards the next level
  T* r;       // right-hand side
  T* x;       // result (z on level 0)
  T* t;       // scratch: level 0 = residual of the pre-smoothed problem
};

// Scalars shared by every level.  Kernels get these and the descriptors of
// the one or two levels they touch as separate by-value arguments (a
// dynamically indexed table in the arguments would live in scratch memory).
template <class T>
struct MgCommon {
  int bc[6];
  T om;       // Jacobi weight
  T sgn[6];   // mirror sign of a correction across each side: -1 outlet, +1 otherwise
};

__host__ __device__ static inline long long ncells(const Layout& L) { return (long long)L.nx * L.ny * L.nz; }

__device__ __forceinline__ void decode(int idx, const Layout& L, int& i, int& j, int& k) {
  k = idx % L.nz;
  const int r = idx / L.nz;
  j = r % L.ny;
  i = r / L.ny;
}

__device__ __forceinline__ bool deep_inside(const Layout& L, int i, int j, int k) {
  return i >= 2 && i < L.nx - 2 && j >= 2 && j < L.ny - 2 && k >= 2 && k < L.nz - 2;
}

// om / D at a cell of level F; 0 outside the level, so that a ghost (whose
// r is zero) contributes nothing.  Interior cells share one constant.
template <class T>
__device__ __forceinline__ T omd(const MgCommon<T>& K, const MgLvl<T>& F, int i, int j, int k) {
  const Layout& L = F.L;
  if ((unsigned)i >= (unsigned)L.nx || (unsigned)j >= (unsigned)L.ny || (unsigned)k >= (unsigned)L.nz) return T(0);
  if (i > 0 && i < L.nx - 1 && j > 0 && j < L.ny - 1 && k > 0 && k < L.nz - 1) return F.omd_in;
  return K.om / diag_w(K.bc, L, F.w, i, j, k);
}

// Residual of the pre-smoothed problem at cell (i,j,k) of level F:
// r - A e with e = om D^-1 r (one Jacobi sweep from zero), i.e.
//   (1 - om) r + sum_a w_a (e_{+a} + e_{-a}).
template <class T>
__device__ __forceinline__ T smoothed_residual(const MgCommon<T>& K, const MgLvl<T>& F, const T* __restrict__ r, int i,
                                               int j, int k) {
  const Layout& L = F.L;
  const long long o = L.at(i, j, k);
  T s;
  if (deep_inside(L, i, j, k)) {
    s = F.omd_in * (F.w[0] * (r[o + L.SX] + r[o - L.SX]) + F.w[1] * (r[o + L.PZ] + r[o - L.PZ]) +
                    F.w[2] * (r[o + 1] + r[o - 1]));
  } else {
    auto e_at = [&](int ii, int jj, int kk) -> T { return omd(K, F, ii, jj, kk) * r[L.at(ii, jj, kk)]; };
    s = F.w[0] * (e_at(i + 1, j, k) + e_at(i - 1, j, k)) + F.w[1] * (e_at(i, j + 1, k) + e_at(i, j - 1, k)) +
        F.w[2] * (e_at(i, j, k + 1) + e_at(i, j, k - 1));
  }
  return (T(1) - K.om) * r[o] + s;
}

// Trilinear prolongation along one axis: a child f takes w0 x[i0] + w1 x[i1].
template <class T>
struct Tap2 {
  int i0, i1;
  T w0, w1;
};

template <class T>
__device__ __forceinline__ Tap2<T> ptap(int f, int c, int nc, T slo, T shi) {
  if (!c) return Tap2<T>{f, f, T(1), T(0)};
  const int I = f >> 1;
  const int J = (f & 1) ? I + 1 : I - 1;
  if (J < 0) return Tap2<T>{I, I, T(0.75) + T(0.25) * slo, T(0)};
  if (J >= nc) return Tap2<T>{I, I, T(0.75) + T(0.25) * shi, T(0)};
  return Tap2<T>{I, J, T(0.75), T(0.25)};
}

// (P x_c) at cell (i, j, k) of level F (inside the level).
template <class T>
__device__ __forceinline__ T prolong(const MgCommon<T>& K, const MgLvl<T>& F, const MgLvl<T>& C, int i, int j, int k) {
  const Tap2<T> a = ptap(i, F.c[0], C.L.nx, K.sgn[0], K.sgn[1]);
  const Tap2<T> b = ptap(j, F.c[1], C.L.ny, K.sgn[2], K.sgn[3]);
  const Tap2<T> c = ptap(k, F.c[2], C.L.nz, K.sgn[4], K.sgn[5]);
  const T* __restrict__ x = C.x;
  const Layout& L = C.L;
  auto row = [&](int I, int J) { return c.w0 * x[L.at(I, J, c.i0)] + c.w1 * x[L.at(I, J, c.i1)]; };
  return a.w0 * (b.w0 * row(a.i0, b.i0) + b.w1 * row(a.i0, b.i1)) +
         a.w1 * (b.w0 * row(a.i1, b.i0) + b.w1 * row(a.i1, b.i1));
}

// Restriction weights along one axis for coarse index I: fine cells
// f = 2I-1 .. 2I+2 with weight P(f, I) / 2 on a halved axis (taps past the
// level get weight 0 and an index clamped into the level, so that a reader
// of a compact array without ghosts never leaves it: a value read there
// from memory nobody wrote, if NaN, would survive the zero weight), or
// f = I alone.  Fixed tap positions keep the arrays in registers.
template <class T>
__device__ __forceinline__ int rtaps(int I, int c, int nc, int nf, T slo, T shi, int f[4], T w[4]) {
  if (!c) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      f[q] = I;
      w[q] = q == 0 ? T(1) : T(0);
    }
    return 1;
  }
  f[0] = 2 * I - 1 >= 0 ? 2 * I - 1 : 2 * I;
  w[0] = 2 * I - 1 >= 0 ? T(0.125) : T(0);
  f[1] = 2 * I;
  w[1] = T(0.5) * (T(0.75) + (I == 0 ? T(0.25) * slo : T(0)));
  // an odd fine axis (nf = 2 nc - 1) has no right child under its last coarse cell
  f[2] = 2 * I + 1 < nf ? 2 * I + 1 : 2 * I;
  w[2] = 2 * I + 1 < nf ? T(0.5) * (T(0.75) + (I == nc - 1 ? T(0.25) * shi : T(0))) : T(0);
  f[3] = 2 * I + 2 < nf ? 2 * I + 2 : f[2];
  w[3] = 2 * I + 2 < nf ? T(0.125) : T(0);
  return 4;
}

// (R res)(I, J, Kc) = sum over fine f of P(f, I)/m res_f.
template <class T, class Res>
__device__ __forceinline__ T restrict_at(const MgCommon<T>& K, const MgLvl<T>& F, const MgLvl<T>& C, int I, int J,
                                         int Kc, Res res) {
  int fi[4], fj[4], fk[4];
  T wi[4], wj[4], wk[4];
  const int ni = rtaps(I, F.c[0], C.L.nx, F.L.nx, K.sgn[0], K.sgn[1], fi, wi);
  const int nj = rtaps(J, F.c[1], C.L.ny, F.L.ny, K.sgn[2], K.sgn[3], fj, wj);
  const int nk = rtaps(Kc, F.c[2], C.L.nz, F.L.nz, K.sgn[4], K.sgn[5], fk, wk);
  T acc = T(0);
#pragma unroll 1
  for (int a = 0; a < 4; ++a) {
    if (a >= ni) break;
    T sa = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (b >= nj) break;
      T sb = T(0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q >= nk) break;
        sb += wk[q] * res(fi[a], fj[b], fk[q]);
      }
      sa += wj[b] * sb;
    }
    acc += wi[a] * sa;
  }
  return acc;
}

// t = om D^-1 r + P x_c at a cell of level F; 0 outside the level.
template <bool COARSE, class T>
__device__ __forceinline__ T pre_plus_coarse(const MgCommon<T>& K, const MgLvl<T>& F, const MgLvl<T>& C, int i, int j,
                                             int k) {
  const Layout& L = F.L;
  if ((unsigned)i >= (unsigned)L.nx || (unsigned)j >= (unsigned)L.ny || (unsigned)k >= (unsigned)L.nz) return T(0);
  T v = omd(K, F, i, j, k) * F.r[L.at(i, j, k)];
  if (COARSE) v += prolong(K, F, C, i, j, k);
  return v;
}

// ----------------------------------------------------------------- kernels

__device__ __forceinline__ bool inside(const Layout& L, int i, int j, int k) {
  return (unsigned)i < (unsigned)L.nx && (unsigned)j < (unsigned)L.ny && (unsigned)k < (unsigned)L.nz;
}

// Index clamped into the padded extent [-1, n + 1] of an axis.  Every
// vector the level kernels read this way (CG residuals, level right-hand
// sides and corrections) has zero ghosts, so positions past the level read
// as 0 without a branch.
__device__ __forceinline__ int clampg(int i, int n) { return min(max(i, -1), n + 1); }

// Walk of a DI x DJ x DK box (k fastest) by NT threads: a thread takes a
// (jj, kk) column of the plane and the entries ii = g, g + STEP, ... of it
// (STEP > 1 only when the plane has fewer entries than threads).
template <int DI, int DJ, int DK, int NT>
struct BoxWalk {
  static constexpr int P = DJ * DK;
  static constexpr int STEP = P >= NT ? 1 : NT / P;
  static constexpr int U = (DI + STEP - 1) / STEP;   // entries per column and thread
  template <class Fn>
  __device__ __forceinline__ static void run(Fn f) {
    if (P >= NT) {
      for (int pidx = threadIdx.x; pidx < P; pidx += NT) f(pidx / DK, pidx % DK, 0);
    } else {
      const int g = threadIdx.x / P;
      if (g < STEP) {
        const int pidx = threadIdx.x - g * P;
        f(pidx / DK, pidx % DK, g);
      }
    }
  }
};

// LDS copy of a DI x DJ x DK box of a level vector from (lo0, lo1, lo2),
// each entry scaled by scale(ii, jj, kk) (positions past the level read 0).
template <int DI, int DJ, int DK, int NT, class T, class Scale>
__device__ __forceinline__ void stage_box(T* __restrict__ s, const T* __restrict__ src, const Layout& L, int lo0,
                                          int lo1, int lo2, Scale scale) {
  using W = BoxWalk<DI, DJ, DK, NT>;
  W::run([&](int jj, int kk, int g) {
    const long long base = (long long)(clampg(lo1 + jj, L.ny) + 1) * L.PZ + (clampg(lo2 + kk, L.nz) + 1);
    T v[W::U];
#pragma unroll
    for (int u = 0; u < W::U; ++u) {
      const int ii = g + u * W::STEP;
      v[u] = ii < DI ? src[(long long)(clampg(lo0 + ii, L.nx) + 1) * L.SX + base] : T(0);
    }
#pragma unroll
    for (int u = 0; u < W::U; ++u) {
      const int ii = g + u * W::STEP;
      if (ii < DI) s[(ii * DJ + jj) * DK + kk] = scale(ii, jj, kk) * v[u];
    }
  });
}

// The same for the vector a - alpha b (the residual after a CG update),
// formed exactly as the update forms it.
template <int DI, int DJ, int DK, int NT, class T, class Scale>
__device__ __forceinline__ void stage_box_axpy(T* __restrict__ s, const T* __restrict__ a, const T* __restrict__ b,
                                               T alpha, const Layout& L, int lo0, int lo1, int lo2, Scale scale) {
  using W = BoxWalk<DI, DJ, DK, NT>;
  W::run([&](int jj, int kk, int g) {
    const long long base = (long long)(clampg(lo1 + jj, L.ny) + 1) * L.PZ + (clampg(lo2 + kk, L.nz) + 1);
    T va[W::U], vb[W::U];
#pragma unroll
    for (int u = 0; u < W::U; ++u) {
      const int ii = g + u * W::STEP;
      const long long o = (long long)(clampg(lo0 + ii, L.nx) + 1) * L.SX + base;
      va[u] = ii < DI ? a[o] : T(0);
      vb[u] = ii < DI ? b[o] : T(0);
    }
#pragma unroll
    for (int u = 0; u < W::U; ++u) {
      const int ii = g + u * W::STEP;
      if (ii < DI) s[(ii * DJ + jj) * DK + kk] = scale(ii, jj, kk) * (va[u] - alpha * vb[u]);
    }
  });
}

// Boundary class of a position along one axis of n cells: bit 0 = first
// cell (or before), bit 1 = last cell (or after).  A cell's D and om/D
// depend only on its three classes (64 combinations).
__device__ __forceinline__ int bclass(int i, int n) { return (i <= 0 ? 1 : 0) | (i >= n - 1 ? 2 : 0); }

__device__ __forceinline__ int cls3(const Layout& L, int i, int j, int k) {
  return (bclass(i, L.nx) << 4) | (bclass(j, L.ny) << 2) | bclass(k, L.nz);
}

// D of class c of level F: per axis, the weight once for each side that is
// not a domain side, or is an outlet side.
template <class T>
__device__ __forceinline__ T class_diag(const MgCommon<T>& K, const MgLvl<T>& F, int c) {
  const int cx = c >> 4, cy = (c >> 2) & 3, cz = c & 3;
  const T dx = F.w[0] * (T(!(cx & 1) || K.bc[0] == OUTLET) + T(!(cx & 2) || K.bc[1] == OUTLET));
  const T dy = F.w[1] * (T(!(cy & 1) || K.bc[2] == OUTLET) + T(!(cy & 2) || K.bc[3] == OUTLET));
  const T dz = F.w[2] * (T(!(cz & 1) || K.bc[4] == OUTLET) + T(!(cz & 2) || K.bc[5] == OUTLET));
  return dx + dy + dz;
}

// Tables of D and om/D by class, filled by threads 0..63 of the block.
template <class T>
__device__ __forceinline__ void fill_class_tables(const MgCommon<T>& K, const MgLvl<T>& F, T* tab_d, T* tab_omd) {
  if (threadIdx.x < 64) {
    const T D = class_diag(K, F, threadIdx.x);
    if (tab_d) tab_d[threadIdx.x] = D;
    tab_omd[threadIdx.x] = D > T(0) ? K.om / D : T(0);
  }
}

// Persistent level kernels: a block walks tiles xcd * per + lid + it * nbx
// (workgroups are dealt to the 8 XCDs round-robin), so the tiles in flight
// on one XCD are neighbours and their halos meet in that XCD's L2.  The
// next tile's box is loaded into registers while the current one is
// processed.
struct TileWalk {
  int t, end, step;
  // G: the blocks that walk tiles (blocks past them have other work)
  __device__ __forceinline__ explicit TileWalk(int nt, int G = gridDim.x) {
    if (G >= 8 && (G & 7) == 0) {
      const int xcd = blockIdx.x & 7, lid = blockIdx.x >> 3, per = (nt + 7) >> 3;
      t = xcd * per + lid;
      end = min(nt, (xcd + 1) * per);
      step = G >> 3;
    } else {
      t = blockIdx.x;
      end = nt;
      step = G;
    }
  }
};

// Tile origin (first cell per axis) of tile t; tiles are numbered with k
// fastest.
__device__ __forceinline__ void tile_origin(int t, int3 nt3, int3 tile, int& x0, int& y0, int& z0) {
  z0 = (t % nt3.x) * tile.z;
  y0 = ((t / nt3.x) % nt3.y) * tile.y;
  x0 = (t / (nt3.x * nt3.y)) * tile.x;
}

constexpr int kLevelBlocksPerCU = 4;   // resident blocks per CU targeted by the level kernels
constexpr int kCUs = 256;

// Coarse tile of the restriction kernel: one next-level cell per thread.
template <class T>
struct RTile {
  static constexpr int CI = 4, CJ = 4, CK = sizeof(T) == 4 ? 16 : 8;
  // fine residual box: 2C + 2 cells per axis (halved axis: from 2X - 1;
  // an axis that is not halved uses its first C entries, from X)
  static constexpr int EI = 2 * CI + 2, EJ = 2 * CJ + 2, EK = 2 * CK + 2;
};

// Restriction, tile by tile of next-level cells: e = om D^-1 r (the
// pre-smoothing sweep from zero) over the tile's footprint and a one-cell
// halo is staged in LDS, the residual of the pre-smoothed problem
//   r - A e = (1 - om) r + sum_a w_a (e_{+a} + e_{-a}),  (1 - om) r = a_c e
// (a_c = (1 - om) D / om by boundary class) is formed over the footprint,
// then restricted.  mode 0: skip when flags[m] is set; 1: block 0 decides
// whether the solve has finished and publishes flags[m] (first kernel of a
// preconditioner application; after convergence the work here is wasted,
// not wrong); 2: unconditional.
// The CG update of iteration t, folded into the level-0 restriction of the
// preconditioner application that follows it: x += alpha d and
// r_{t+1} = r_t - alpha q (into F.r) on the fine cells whose parents are in
// the block's tiles, the r.r partials, and the restriction of the
// pre-smoothed r_{t+1} formed from r_t and q directly.  (The marching
// kernel below leaves x += alpha d to k_cg_xupd.)
template <class T>
struct CgUpd {
  T* X;
  const T* Rin;   // r_t
  const T* D;     // d_t
  const T* Q;     // q = A d_t
  int t;
};

template <bool CGU, class T>
__global__ __launch_bounds__(256) void k_mg_restrict(MgCommon<T> K, MgLvl<T> F, MgLvl<T> C, int has_coarse, CgCtl c,
                                                     int m, int mode, int3 nt3, CgUpd<T> upd) {
  using Rt = RTile<T>;
  constexpr int EI = Rt::EI, EJ = Rt::EJ, EK = Rt::EK;
  constexpr int QI = EI + 2, QJ = EJ + 2, QK = EK + 2;   // e box: the residual box and a 1-cell halo
  __shared__ T sres[EI * EJ * EK];
  __shared__ T se[QI * QJ * QK];
  __shared__ T tab_omd[64];
  __shared__ T tab_a[64];
  // mode 0: the flag is loaded now and tested once the first box is staged,
  // so that its latency overlaps the box loads.  mode 1: one block past the
  // tile walkers takes the decision, off the tiles' critical path.
  const int skip = (!CGU && mode == 0) ? c.flags[m] : 0;
  const int gw = (!CGU && mode == 1 && has_coarse) ? (int)gridDim.x - 1 : (int)gridDim.x;
  if (!CGU && mode == 1) {
    if ((int)blockIdx.x == (has_coarse ? gw : 0)) {
      const bool done = precond_skip(c, m);
      if (threadIdx.x == 0) c.flags[m] = done;
    }
    if ((int)blockIdx.x >= gw) return;
  }
  T alpha = T(0);
  if constexpr (CGU) {
    // the same decision and alpha as the stand-alone update kernel
    double rz = 0.0, dq = 0.0;
    bool run = iteration_open(c, upd.t);
    if (run) {
      rz = c.st->rzh[upd.t & 1];
      run = rz_allows(c, rz);
    }
    if (run) {
      dq = slot_sum(c.part + (size_t)S_DQ * c.stride, c.nb_dq);
      run = dq > 0.0 && isfinite(dq);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      c.exec[upd.t] = run;
      if (run) c.st->iter = upd.t + 1;
    }
    if (!run) return;
    alpha = (T)(rz / dq);
  }
  if (!has_coarse) return;
  if (threadIdx.x < 64) {
    const T D = class_diag(K, F, threadIdx.x);
    tab_omd[threadIdx.x] = D > T(0) ? K.om / D : T(0);
    tab_a[threadIdx.x] = (T(1) - K.om) * D / K.om;
  }
  const Layout& L = F.L;
  const int3 ct = make_int3(Rt::CI, Rt::CJ, Rt::CK);
  const int nt = nt3.x * nt3.y * nt3.z;
  // first fine cell of the residual box of a tile with coarse origin X0
  auto box_lo = [&](int X0, int a) { return F.c[a] ? 2 * X0 - 1 : X0; };
  double acc[1] = {0.0};
  for (TileWalk w(nt, gw); w.t < w.end; w.t += w.step) {
    int X0, Y0, Z0;
    tile_origin(w.t, nt3, ct, X0, Y0, Z0);
    const int lo0 = box_lo(X0, 0), lo1 = box_lo(Y0, 1), lo2 = box_lo(Z0, 2);
    __syncthreads();   // the previous tile is done with the LDS; tables are in place
    auto omd_at = [&](int ii, int jj, int kk) { return tab_omd[cls3(L, lo0 - 1 + ii, lo1 - 1 + jj, lo2 - 1 + kk)]; };
    // CGU: the fine cells whose parents are in this tile (the tiles
    // partition the coarse cells, so these partition the fine ones); their
    // x and d are loaded before the box so that the loads overlap
    using WO = BoxWalk<2 * Rt::CI, 2 * Rt::CJ, 2 * Rt::CK, 256>;
    int f0 = 0, f1 = 0, f2 = 0, e0 = 0, e1 = 0, e2 = 0;
    T xv[WO::U], dv[WO::U], rv[WO::U], qv[WO::U];
    if constexpr (CGU) {
      f0 = F.c[0] ? 2 * X0 : X0;
      f1 = F.c[1] ? 2 * Y0 : Y0;
      f2 = F.c[2] ? 2 * Z0 : Z0;
      e0 = min(F.c[0] ? 2 * Rt::CI : Rt::CI, L.nx - f0);
      e1 = min(F.c[1] ? 2 * Rt::CJ : Rt::CJ, L.ny - f1);
      e2 = min(F.c[2] ? 2 * Rt::CK : Rt::CK, L.nz - f2);
      WO::run([&](int jj, int kk, int g) {
        const long long base = (long long)(f1 + min(jj, e1 - 1) + 1) * L.PZ + (f2 + min(kk, e2 - 1) + 1);
#pragma unroll
        for (int u = 0; u < WO::U; ++u) {
          const long long o = (long long)(f0 + min(g + u * WO::STEP, e0 - 1) + 1) * L.SX + base;
          xv[u] = upd.X[o];
          dv[u] = upd.D[o];
          rv[u] = upd.Rin[o];
          qv[u] = upd.Q[o];
        }
      });
      stage_box_axpy<QI, QJ, QK, 256>(se, upd.Rin, upd.Q, alpha, L, lo0 - 1, lo1 - 1, lo2 - 1, omd_at);
    } else {
      stage_box<QI, QJ, QK, 256>(se, F.r, L, lo0 - 1, lo1 - 1, lo2 - 1, omd_at);
    }
    if (skip) return;   // the solve has finished (uniform over the grid)
    if constexpr (CGU) {
      WO::run([&](int jj, int kk, int g) {
        if (jj >= e1 || kk >= e2) return;
        const long long base = (long long)(f1 + jj + 1) * L.PZ + (f2 + kk + 1);
#pragma unroll
        for (int u = 0; u < WO::U; ++u) {
          const int ii = g + u * WO::STEP;
          if (ii >= e0) break;
          const long long o = (long long)(f0 + ii + 1) * L.SX + base;
          upd.X[o] = xv[u] + alpha * dv[u];
          const T r = rv[u] - alpha * qv[u];
          F.r[o] = r;
          acc[0] += (double)r * (double)r;
        }
      });
    }
    __syncthreads();
    // residual over the footprint; entries outside the level are never
    // restricted from
    using WR = BoxWalk<EI, EJ, EK, 256>;
    WR::run([&](int jj, int kk, int g) {
      const int cyz = (bclass(lo1 + jj, L.ny) << 2) | bclass(lo2 + kk, L.nz);
      constexpr int sI = QJ * QK, sJ = QK;
#pragma unroll
      for (int u = 0; u < WR::U; ++u) {
        const int ii = g + u * WR::STEP;
        if (ii >= EI) break;
        const int q = ((ii + 1) * QJ + (jj + 1)) * QK + (kk + 1);
        sres[(ii * EJ + jj) * EK + kk] = tab_a[(bclass(lo0 + ii, L.nx) << 4) | cyz] * se[q] +
                                         F.w[0] * (se[q + sI] + se[q - sI]) + F.w[1] * (se[q + sJ] + se[q - sJ]) +
                                         F.w[2] * (se[q + 1] + se[q - 1]);
      }
    });
    __syncthreads();
    const int tk = threadIdx.x % Rt::CK, tj = (threadIdx.x / Rt::CK) % Rt::CJ, ti = threadIdx.x / (Rt::CK * Rt::CJ);
    const int I = X0 + ti, J = Y0 + tj, Kc = Z0 + tk;
    if (ti < Rt::CI && inside(C.L, I, J, Kc)) {
      T out;
      if (F.c[0] && F.c[1] && F.c[2]) {
        // every axis halved: the 4 x 4 x 4 fine taps of (I, J, Kc) start at
        // box entry (2 ti, 2 tj, 2 tk); taps past the level have weight 0
        // (their box entries hold finite values)
        T wi[4], wj[4], wk[4];
        auto wts = [&](int X, int nc, int nf, T slo, T shi, T (&w)[4]) {
          w[0] = 2 * X - 1 >= 0 ? T(0.125) : T(0);
          w[1] = T(0.5) * (T(0.75) + (X == 0 ? T(0.25) * slo : T(0)));
          w[2] = 2 * X + 1 < nf ? T(0.5) * (T(0.75) + (X == nc - 1 ? T(0.25) * shi : T(0))) : T(0);
          w[3] = 2 * X + 2 < nf ? T(0.125) : T(0);
        };
        wts(I, C.L.nx, L.nx, K.sgn[0], K.sgn[1], wi);
        wts(J, C.L.ny, L.ny, K.sgn[2], K.sgn[3], wj);
        wts(Kc, C.L.nz, L.nz, K.sgn[4], K.sgn[5], wk);
        const T* base = sres + ((2 * ti) * EJ + 2 * tj) * EK + 2 * tk;
        out = T(0);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          T sa = T(0);
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const T* row = base + (a * EJ + b) * EK;
            sa += wj[b] * (wk[0] * row[0] + wk[1] * row[1] + wk[2] * row[2] + wk[3] * row[3]);
          }
          out += wi[a] * sa;
        }
      } else {
        out = restrict_at(K, F, C, I, J, Kc, [&](int i, int j, int k) {
          return sres[((i - lo0) * EJ + (j - lo1)) * EK + (k - lo2)];
        });
      }
      C.r[C.L.at(I, J, Kc)] = out;
    }
  }
  if constexpr (CGU) {
    const int slots[1] = {S_RR};
    write_partials<1>(acc, c.part, c.stride, slots, (int)blockIdx.x);
    pad_partials(c, S_RR, (int)blockIdx.x, (int)gridDim.x);
  }
}

// ------------------------- level-0 update and restriction, marching in x ---
// The residual update of iteration t and the level-0 restriction of the
// application that follows -- what k_mg_restrict<true> computes but x +=
// alpha d, which k_cg_xupd does beside the coarse levels -- with the
// work laid out as a march along x: a block owns CJ x CK coarse (j, k)
// columns (their 2CJ x 2CK fine children) over a chunk of coarse x-planes
// and walks the fine planes in order.  Per fine plane it forms
// e = om D^-1 (r_t - alpha q) on the fine columns and two cells around them
// (its own cells from the values the update loads anyway), keeps the last
// three e planes in LDS, forms the residual of the pre-smoothed problem one
// plane behind, and adds that plane's y/z restriction into the two coarse
// planes it belongs to (x weights in tap order, as restrict_at adds them).
// r_t and q are read once per plane and band (the 3-D boxes of
// k_mg_restrict read them 2.5 times), and the block's working set is three
// planes.  Every axis must be halved towards the coarse level.
template <class T>
struct XTile {
  static constexpr int CJ = 8, CK = 32;            // coarse columns, one per thread
  static constexpr int FJ = 2 * CJ, FK = 2 * CK;   // fine columns, four per thread
  static constexpr int EJ = FJ + 4, EK = FK + 4;   // e plane: 2 cells around
  static constexpr int RJ = FJ + 2, RK = FK + 2;   // residual plane: 1 cell around
  static constexpr int NE = EJ * EK, NR = RJ * RK;
  static constexpr int NRING = NE - FJ * FK;       // e entries around the fine columns
  static constexpr int ROWS = 256 / FK;            // fine rows a pass of the block covers
};

// Restriction weights along one halved axis for coarse index X (taps 2X-1 ..
// 2X+2; those past the level get 0), as k_mg_restrict's.
template <class T>
__device__ __forceinline__ void rweights(int X, int nc, int nf, T slo, T shi, T w[4]) {
  w[0] = 2 * X - 1 >= 0 ? T(0.125) : T(0);
  w[1] = T(0.5) * (T(0.75) + (X == 0 ? T(0.25) * slo : T(0)));
  w[2] = 2 * X + 1 < nf ? T(0.5) * (T(0.75) + (X == nc - 1 ? T(0.25) * shi : T(0))) : T(0);
  w[3] = 2 * X + 2 < nf ? T(0.125) : T(0);
}

// Position (ej, ek) in the e plane of ring entry q (the entries that are
// not the block's fine columns): two full rows on each side, then two
// entries at each end of the rows in between.
template <class T>
__device__ __forceinline__ void ring_pos(int q, int& ej, int& ek) {
  using X = XTile<T>;
  if (q < 2 * X::EK) {
    ej = q / X::EK;
    ek = q - ej * X::EK;
  } else if (q < 4 * X::EK) {
    const int r = q - 2 * X::EK;
    ej = X::EJ - 2 + r / X::EK;
    ek = r % X::EK;
  } else {
    const int r = q - 4 * X::EK, c4 = r & 3;
    ej = 2 + (r >> 2);
    ek = c4 < 2 ? c4 : X::EK - 4 + c4;
  }
}

// CGU true: the residual update r -= alpha q of CG iteration upd.t (its
// decision and alpha as k_mg_restrict<true>'s), then the restriction of the
// pre-smoothed new residual; the iterate's update x += alpha d is left to
// k_cg_xupd, which runs beside the coarse levels.
// CGU false: the plain restriction of level F's r (what k_mg_restrict<false>
// computes), with k_mg_restrict's modes -- 0: skip when flags[m] is set;
// 1: the block past the tile walkers (logical block ntot) decides whether
// the solve has finished and publishes flags[m], the others work
// unconditionally; 2: unconditional.
template <bool CGU, class T>
__global__ __launch_bounds__(256) void k_mg_update_march(MgCommon<T> K, MgLvl<T> F, MgLvl<T> C, CgCtl c,
                                                         CgUpd<T> upd, int nci, int nkt, int nchunk, int ntot,
                                                         int m, int mode) {
  using X = XTile<T>;
  __shared__ T se[3][X::NE];
  __shared__ T sres[X::NR];
  __shared__ T tab_omd[64];
  __shared__ T tab_a[64];
  const int per = (int)(gridDim.x >> 3);
  const int lb = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  T alpha = T(0);
  if constexpr (CGU) {
    // the same decision and alpha as the stand-alone update kernel
    double rz = 0.0, dq = 0.0;
    bool run = iteration_open(c, upd.t);
    if (run) {
      rz = c.st->rzh[upd.t & 1];
      run = rz_allows(c, rz);
    }
    if (run) {
      dq = slot_sum(c.part + (size_t)S_DQ * c.stride, c.nb_dq);
      run = dq > 0.0 && isfinite(dq);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      c.exec[upd.t] = run;
      if (run) c.st->iter = upd.t + 1;
    }
    if (!run) return;
    alpha = (T)(rz / dq);
  } else {
    if (mode == 1 && lb == ntot) {
      const bool done = precond_skip(c, m);
      if (threadIdx.x == 0) c.flags[m] = done;
      return;
    }
    if (mode == 0 && c.flags[m]) return;   // the solve has finished (uniform over the grid)
  }
  if (threadIdx.x < 64) {
    const T D = class_diag(K, F, threadIdx.x);
    tab_omd[threadIdx.x] = D > T(0) ? K.om / D : T(0);
    tab_a[threadIdx.x] = (T(1) - K.om) * D / K.om;
  }
  const Layout& L = F.L;
  double acc_rr[1] = {0.0};
  // logical block lb: XCD-contiguous ranges of (j tile, k tile, chunk)
  if (lb < ntot) {
    const int tile = lb / nchunk, ch = lb - tile * nchunk;
    const int jt = tile / nkt, kt = tile - jt * nkt;
    const int J0 = jt * X::CJ, K0 = kt * X::CK;
    const int j0 = 2 * J0, k0 = 2 * K0;
    const int I0 = ch * nci, I1 = min(C.L.nx, I0 + nci);
    const int own0 = 2 * I0, own1 = min(2 * I1, L.nx);   // fine planes this block updates
    const int tid = threadIdx.x;
    const int kk = tid % X::FK, jr = tid / X::FK;
    const int k = k0 + kk;
    const int kg = clampg(k, L.nz);
    const bool kin = k < L.nz;
    // own column rows j0 + jr + ROWS u
    int jg[4];
    bool jin[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + jr + X::ROWS * u;
      jg[u] = clampg(j, L.ny);
      jin[u] = j < L.ny;
    }
    // ring entries of this thread (at most two)
    int rq[2], rjg[2], rkg[2], rpos[2];
    bool ron[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int q = tid + 256 * v;
      ron[v] = q < X::NRING;
      int ej = 0, ek = 0;
      if (ron[v]) ring_pos<T>(q, ej, ek);
      rq[v] = q;
      rjg[v] = clampg(j0 - 2 + ej, L.ny);
      rkg[v] = clampg(k0 - 2 + ek, L.nz);
      rpos[v] = ej * X::EK + ek;
    }
    // the coarse column of the restriction
    const int tj = tid / X::CK, tk = tid - tj * X::CK;
    const int J = J0 + tj, Kc = K0 + tk;
    const bool cin = J < C.L.ny && Kc < C.L.nz;
    T wj[4], wk[4];
    rweights(J, C.L.ny, L.ny, K.sgn[2], K.sgn[3], wj);
    rweights(Kc, C.L.nz, L.nz, K.sgn[4], K.sgn[5], wk);
    // plane values in registers: own r_t, q, ring r_t, q
    T orr[4], oq[4], rr_[2], rq_[2];
    // the residual read: r_t (with q for the update) or level F's r
    const T* __restrict__ rin = CGU ? upd.Rin : F.r;
    auto load_plane = [&](int f) {
      const int fg = clampg(f, L.nx);
      const long long base = (long long)(fg + 1) * L.SX;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const long long o = base + (long long)(jg[u] + 1) * L.PZ + (kg + 1);
        orr[u] = rin[o];
        if constexpr (CGU) oq[u] = upd.Q[o];
      }
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const long long o = base + (long long)(rjg[v] + 1) * L.PZ + (rkg[v] + 1);
        rr_[v] = ron[v] ? rin[o] : T(0);
        if constexpr (CGU) rq_[v] = ron[v] ? upd.Q[o] : T(0);
      }
    };
    const int fe0 = 2 * I0 - 2, fe1 = 2 * I1 + 1;   // e planes
    load_plane(fe0);
    // the (j, k) part of the boundary classes of the thread's own and ring
    // entries and of its residual entries, and the residual entries' e
    // positions: fixed for the whole march
    constexpr int NRU = (X::NR + 255) / 256;
    int ocyz[4], gcyz[2], qcyz[NRU], qpe[NRU];
#pragma unroll
    for (int u = 0; u < 4; ++u) ocyz[u] = (bclass(j0 + jr + X::ROWS * u, L.ny) << 2) | bclass(k, L.nz);
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int ej = rpos[v] / X::EK, ek = rpos[v] - ej * X::EK;
      gcyz[v] = (bclass(j0 - 2 + ej, L.ny) << 2) | bclass(k0 - 2 + ek, L.nz);
    }
#pragma unroll
    for (int u = 0; u < NRU; ++u) {
      const int q = min(tid + 256 * u, X::NR - 1);
      const int rj = q / X::RK, rk = q - rj * X::RK;
      qpe[u] = (rj + 1) * X::EK + rk + 1;
      qcyz[u] = (bclass(j0 - 1 + rj, L.ny) << 2) | bclass(k0 - 1 + rk, L.nz);
    }
    __syncthreads();   // tables in place
    T wi_cur[4], wi_prev[4];
    int Icur = I0;
    rweights(Icur, C.L.nx, L.nx, K.sgn[0], K.sgn[1], wi_cur);
    rweights(Icur - 1, C.L.nx, L.nx, K.sgn[0], K.sgn[1], wi_prev);
    T acc_cur = T(0), acc_prev = T(0);
    for (int f = fe0; f <= fe1; ++f) {
      T* e = se[(f + 3) % 3];
      const int cx = bclass(f, L.nx) << 4;
      const bool upd_plane = f >= own0 && f < own1;
      // own cells: the update, then e from the updated residual
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const T r = CGU ? orr[u] - alpha * oq[u] : orr[u];
        const int jj = jr + X::ROWS * u;
        e[(jj + 2) * X::EK + kk + 2] = tab_omd[cx | ocyz[u]] * r;
        if (CGU && upd_plane && jin[u] && kin) {
          const long long o = (long long)(f + 1) * L.SX + (long long)(jg[u] + 1) * L.PZ + (kg + 1);
          F.r[o] = r;
          acc_rr[0] += (double)r * (double)r;
        }
      }
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        if (!ron[v]) continue;
        e[rpos[v]] = tab_omd[cx | gcyz[v]] * (CGU ? rr_[v] - alpha * rq_[v] : rr_[v]);
      }
      if (f < fe1) load_plane(f + 1);
      __syncthreads();
      // residual of plane f - 1 from the e planes f - 2, f - 1, f
      const int fr = f - 1;
      if (fr < 2 * I0 - 1) continue;
      {
        const T* em = se[(fr + 2) % 3];
        const T* ec = se[(fr + 3) % 3];
        const T* ep = e;
        const int crx = bclass(fr, L.nx) << 4;
#pragma unroll
        for (int u = 0; u < NRU; ++u) {
          const int q = tid + 256 * u;
          if (q >= X::NR) break;
          const int pe = qpe[u];
          sres[q] = tab_a[crx | qcyz[u]] * ec[pe] + F.w[0] * (ep[pe] + em[pe]) +
                    F.w[1] * (ec[pe + X::EK] + ec[pe - X::EK]) + F.w[2] * (ec[pe + 1] + ec[pe - 1]);
        }
      }
      __syncthreads();
      // y/z restriction of the residual plane, added to its two coarse planes
      const int In = (fr + 1) >> 1;
      if (In != Icur) {
        // coarse plane Icur - 1 has all four taps
        if (cin && Icur - 1 >= I0 && Icur - 1 < I1) C.r[C.L.at(Icur - 1, J, Kc)] = acc_prev;
        acc_prev = acc_cur;
        acc_cur = T(0);
        Icur = In;
#pragma unroll
        for (int a = 0; a < 4; ++a) wi_prev[a] = wi_cur[a];
        rweights(Icur, C.L.nx, L.nx, K.sgn[0], K.sgn[1], wi_cur);
      }
      T sa = T(0);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const T* row = sres + (2 * tj + b) * X::RK + 2 * tk;
        sa += wj[b] * (wk[0] * row[0] + wk[1] * row[1] + wk[2] * row[2] + wk[3] * row[3]);
      }
      const int a = fr + 1 - 2 * Icur;   // 0 or 1 for Icur, a + 2 for Icur - 1
      acc_cur += wi_cur[a] * sa;
      acc_prev += wi_prev[a + 2] * sa;
    }
    if (cin && Icur - 1 >= I0 && Icur - 1 < I1) C.r[C.L.at(Icur - 1, J, Kc)] = acc_prev;
  }
  if constexpr (CGU) {
    const int slots[1] = {S_RR};
    write_partials<1>(acc_rr, c.part, c.stride, slots, (int)blockIdx.x);
    pad_partials(c, S_RR, (int)blockIdx.x, (int)gridDim.x);
  }
}

// x += alpha d of CG iteration t over the interior cells of level 0, the
// update the marching restriction leaves out: the decision (exec[t], which
// that kernel published) and alpha come from the same values as there, and
// the partial-sum reduction has the same 256-thread shape, so x gets the
// same bits as an update inside the restriction.  Launched on a stream of
// its own after the restriction; the iteration's end waits for it.
template <class T>
__global__ __launch_bounds__(256) void k_cg_xupd(Layout L, T* __restrict__ X, const T* __restrict__ D, CgCtl c,
                                                 int t) {
  if (!c.exec[t]) return;
  const double rz = c.st->rzh[t & 1];
  const double dq = slot_sum(c.part + (size_t)S_DQ * c.stride, c.nb_dq);
  const T alpha = (T)(rz / dq);
  // work items: 64-cell pieces of the (i, j) rows, one per wavefront at a
  // time (a grid has fewer than 2^31 padded cells: 32-bit indices)
  const unsigned nz = (unsigned)L.nz, ny = (unsigned)L.ny;
  const unsigned kc = (nz + 63u) >> 6;
  const unsigned items = (unsigned)L.nx * ny * kc;
  const unsigned lane = threadIdx.x & 63u;
  const unsigned nw = gridDim.x * 4u;
  for (unsigned it = blockIdx.x * 4u + (threadIdx.x >> 6); it < items; it += nw) {
    const unsigned w = __builtin_amdgcn_readfirstlane(it);
    const unsigned row = w / kc, k = (w - row * kc) * 64u + lane;
    const unsigned i = row / ny, j = row - i * ny;
    if (k < nz) {
      const long long o = L.at((int)i, (int)j, (int)k);
      X[o] = X[o] + alpha * D[o];
    }
  }
}

// Tile of the up/smoothing kernel (cells of its level per block of 256).
template <int TI_, int TJ_, int TK_>
struct UpTile {
  static constexpr int TI = TI_, TJ = TJ_, TK = TK_;
};
using UpBig = UpTile<8, 8, 32>;     // levels of >= kUpBigCells cells
using UpSmall = UpTile<4, 4, 16>;   // smaller levels: more tiles to spread
constexpr long long kUpBigCells = 1LL << 20;

// Prolongation + post-smoothing, tile by tile of level F: t = om D^-1 r +
// P x_c over the tile and a one-cell halo (LDS), then x = t + om D^-1
// (r - A t).  r of the box and the coarse values it needs are staged in LDS
// first.  HALF: every axis is halved towards C (the coarse box is then
// TI/2 + 4 wide per axis).  FINE: level 0, also writes the block's partial
// of r.z for the CG.
template <bool FINE, bool COARSE, bool HALF, class Tile, class T>
__global__ __launch_bounds__(256) void k_mg_upsmooth(MgCommon<T> K, MgLvl<T> F, MgLvl<T> C, CgCtl c, int m, int3 nt3) {
  constexpr int TI = Tile::TI, TJ = Tile::TJ, TK = Tile::TK;
  constexpr int HI = TI + 2, HJ = TJ + 2, HK = TK + 2, HN = HI * HJ * HK;
  // coarse box: parents of the fine box and their prolongation neighbours
  // (halved axis: from i0/2 - 2, TI/2 + 4 entries; otherwise the fine box)
  constexpr int XI = HALF ? TI / 2 + 4 : HI, XJ = HALF ? TJ / 2 + 4 : HJ, XK = HALF ? TK / 2 + 4 : HK;
  __shared__ T sr[HN];
  __shared__ T st[HN];
  __shared__ T sx[COARSE ? XI * XJ * XK : 1];
  __shared__ T tab_d[64];
  __shared__ T tab_omd[64];
  const int skip = c.flags[m];   // tested once the first boxes are staged
  fill_class_tables<T>(K, F, tab_d, tab_omd);
  const Layout& L = F.L;
  const int3 tt = make_int3(TI, TJ, TK);
  const int nt = nt3.x * nt3.y * nt3.z;
  auto clo = [&](int x0, int a) { return F.c[a] ? (x0 >> 1) - 2 : x0 - 1; };
  auto one = [](int, int, int) { return T(1); };
  double acc[1] = {0.0};
  for (TileWalk w(nt); w.t < w.end; w.t += w.step) {
    int i0, j0, k0;
    tile_origin(w.t, nt3, tt, i0, j0, k0);
    const int cl0 = clo(i0, 0), cl1 = clo(j0, 1), cl2 = clo(k0, 2);
    __syncthreads();   // the previous tile is done with the LDS; tables are in place
    stage_box<HI, HJ, HK, 256>(sr, F.r, L, i0 - 1, j0 - 1, k0 - 1, one);
    if (COARSE) stage_box<XI, XJ, XK, 256>(sx, C.x, C.L, cl0, cl1, cl2, one);
    if (skip) return;   // the solve has finished (uniform over the grid)
    __syncthreads();
    // t = om D^-1 r + P x_c over the box, 0 outside the level
    using WT = BoxWalk<HI, HJ, HK, 256>;
    if constexpr (COARSE && HALF && WT::STEP == 1 && TI % 2 == 0) {
      // Every axis halved and one thread per (jj, kk) column: the column's
      // coarse values are interpolated in (j, k) once (cv, by coarse x
      // index - cl0); a fine cell then takes its parent and x-neighbour
      // from cv.  The tile origin i0 is even, so for the box entry ii the
      // parent is cv[((ii - 1) >> 1) + 2] and the neighbour lies on the
      // child's side (+1 for odd i, i.e. even ii).
      WT::run([&](int jj, int kk, int) {
        const int j = j0 - 1 + jj, k = k0 - 1 + kk;
        const bool in_jk = (unsigned)j < (unsigned)L.ny && (unsigned)k < (unsigned)L.nz;
        const int cyz = (bclass(j, L.ny) << 2) | bclass(k, L.nz);
        const Tap2<T> b = ptap(j, 1, C.L.ny, K.sgn[2], K.sgn[3]);
        const Tap2<T> e = ptap(k, 1, C.L.nz, K.sgn[4], K.sgn[5]);
        const int r0 = (b.i0 - cl1) * XK, r1 = (b.i1 - cl1) * XK;
        const int q0 = e.i0 - cl2, q1 = e.i1 - cl2;
        T cv[XI];
#pragma clang loop unroll(full)
        for (int I = 1; I <= 6; ++I) {
          const T* sp = sx + I * XJ * XK;
          cv[I] = b.w0 * (e.w0 * sp[r0 + q0] + e.w1 * sp[r0 + q1]) + b.w1 * (e.w0 * sp[r1 + q0] + e.w1 * sp[r1 + q1]);
        }
#pragma clang loop unroll(full)
        for (int ii = 0; ii < HI; ++ii) {
          const int i = i0 - 1 + ii;
          const int Ir = ((ii - 1) >> 1) + 2;
          const int Jr = (ii % 2 == 0) ? Ir + 1 : Ir - 1;
          const int J = cl0 + Jr;   // neighbour's coarse x index
          T w0 = T(0.75), w1 = T(0.25);
          if (J < 0) {
            w0 = T(0.75) + T(0.25) * K.sgn[0];
            w1 = T(0);
          } else if (J >= C.L.nx) {
            w0 = T(0.75) + T(0.25) * K.sgn[1];
            w1 = T(0);
          }
          const int idx = (ii * HJ + jj) * HK + kk;
          T v = T(0);
          if (in_jk && (unsigned)i < (unsigned)L.nx)
            v = tab_omd[(bclass(i, L.nx) << 4) | cyz] * sr[idx] + w0 * cv[Ir] + w1 * cv[Jr];
          st[idx] = v;
        }
      });
    } else
    WT::run([&](int jj, int kk, int g) {
      const int j = j0 - 1 + jj, k = k0 - 1 + kk;
      const bool in_jk = (unsigned)j < (unsigned)L.ny && (unsigned)k < (unsigned)L.nz;
      const int cyz = (bclass(j, L.ny) << 2) | bclass(k, L.nz);
      const Tap2<T> b = ptap(j, F.c[1], C.L.ny, K.sgn[2], K.sgn[3]);
      const Tap2<T> e = ptap(k, F.c[2], C.L.nz, K.sgn[4], K.sgn[5]);
#pragma unroll
      for (int u = 0; u < WT::U; ++u) {
        const int ii = g + u * WT::STEP;
        if (ii >= HI) break;
        const int i = i0 - 1 + ii;
        const int idx = (ii * HJ + jj) * HK + kk;
        T v = T(0);
        if (in_jk && (unsigned)i < (unsigned)L.nx) {
          v = tab_omd[(bclass(i, L.nx) << 4) | cyz] * sr[idx];
          if (COARSE) {
            const Tap2<T> a = ptap(i, F.c[0], C.L.nx, K.sgn[0], K.sgn[1]);
            auto row = [&](int I, int J) {
              const int base = ((I - cl0) * XJ + (J - cl1)) * XK - cl2;
              return e.w0 * sx[base + e.i0] + e.w1 * sx[base + e.i1];
            };
            v += a.w0 * (b.w0 * row(a.i0, b.i0) + b.w1 * row(a.i0, b.i1)) +
                 a.w1 * (b.w0 * row(a.i1, b.i0) + b.w1 * row(a.i1, b.i1));
          }
        }
        st[idx] = v;
      }
    });
    __syncthreads();
    // x = t + om D^-1 (r - A t) on the tile
    using WZ = BoxWalk<TI, TJ, TK, 256>;
    WZ::run([&](int jj, int kk, int g) {
      const int j = j0 + jj, k = k0 + kk;
      if ((unsigned)j >= (unsigned)L.ny || (unsigned)k >= (unsigned)L.nz) return;
      const int cyz = (bclass(j, L.ny) << 2) | bclass(k, L.nz);
#pragma unroll
      for (int u = 0; u < WZ::U; ++u) {
        const int ii = g + u * WZ::STEP;
        const int i = i0 + ii;
        if (ii >= TI || i >= L.nx) break;
        const int q = ((ii + 1) * HJ + (jj + 1)) * HK + (kk + 1);
        const int cl = (bclass(i, L.nx) << 4) | cyz;
        const T tc = st[q];
        const T At = tab_d[cl] * tc - F.w[0] * (st[q + HJ * HK] + st[q - HJ * HK]) -
                     F.w[1] * (st[q + HK] + st[q - HK]) - F.w[2] * (st[q + 1] + st[q - 1]);
        const T rr = sr[q];
        const T z = tc + tab_omd[cl] * (rr - At);
        F.x[L.at(i, j, k)] = z;
        if (FINE) acc[0] += (double)rr * (double)z;
      }
    });
  }
  if (FINE && !skip) {
    const int slots[1] = {S_RZ0 + (m & 1)};
    write_partials<1>(acc, c.part, c.stride, slots, (int)blockIdx.x);
  }
}

// ---------------- level-0 prolongation and post-smoothing, marching in x ---
// What k_mg_upsmooth<true, true, true> computes on level 0, laid out as a
// march along x: a block owns 16 x 64 fine (j, k) columns over a chunk of
// planes.  Per coarse plane I it forms the y/z interpolation Y(I) of the
// correction on the columns and one cell around (the coarse taps of each
// position fixed for the whole march), keeping three such planes in LDS;
// per fine plane it forms t = om D^-1 r + P x_c from the two Y planes of
// its parent and the parent's neighbour, keeping three t planes in LDS
// (the own columns' t also in registers), and one plane behind it the
// smoothed z = t + om D^-1 (r - A t) and the r.z partial.  r is read once
// per plane and band, and one barrier separates the planes.  The kernel is
// bound by the latency of its per-plane steps: 512 threads of two columns
// each keep twice the wavefronts of 256 threads of four in flight (64
// registers instead of 93; 112 -> 98 us per launch at 512x512x128).
struct UTile {
  static constexpr int NTH = 512;                  // threads of a block
  static constexpr int FJ = 16, FK = 64;           // fine columns, NU per thread
  static constexpr int TJ = FJ + 2, TK = FK + 2;   // t and Y planes: 1 cell around
  static constexpr int NT = TJ * TK;
  static constexpr int ROWS = NTH / FK;
  static constexpr int NU = FJ / ROWS;
};

struct UpGeom {
  int nfi, nkt, nchunk, ntot;
};

static UpGeom up_geom(const Layout& L);

// The march applies to level 0 when every axis halves towards level 1, the
// columns fill the tile's depth and a chunk is at least 16 planes long (it
// forms t on two planes past its own).
static bool up_march(const Layout& L) {
  return L.nx >= 4 && L.ny >= 4 && L.nz >= UTile::FK && (long long)L.nx * L.ny * L.nz > kCoarsestCells &&
         up_geom(L).nfi >= 16;
}

static UpGeom up_geom(const Layout& L) {
  UpGeom u;
  const int njt = (L.ny + UTile::FJ - 1) / UTile::FJ;
  u.nkt = (L.nz + UTile::FK - 1) / UTile::FK;
  const int tiles = njt * u.nkt;
  const int want = std::max(1, std::min(L.nx, (1024 + tiles - 1) / tiles));
  u.nfi = (L.nx + want - 1) / want;
  u.nchunk = (L.nx + u.nfi - 1) / u.nfi;
  u.ntot = tiles * u.nchunk;
  return u;
}

template <class T>
__global__ __launch_bounds__(UTile::NTH) void k_mg_upsmooth_march(MgCommon<T> K, MgLvl<T> F, MgLvl<T> C, CgCtl c, int m,
                                                           int nfi, int nkt, int nchunk, int ntot) {
  using U = UTile;
  constexpr int NRING = U::NT - U::FJ * U::FK;   // region entries around the fine columns
  __shared__ T sy[3][U::NT];
  __shared__ T st[3][U::NT];
  __shared__ T tab_d[64];
  __shared__ T tab_omd[64];
  // coarse taps of the region's rows (y) and columns (z): offsets and weights
  __shared__ int rt_o[U::TJ][2];
  __shared__ T rt_w[U::TJ][2];
  __shared__ int ct_o[U::TK][2];
  __shared__ T ct_w[U::TK][2];
  if (c.flags[m]) return;   // the solve has finished (uniform over the grid)
  fill_class_tables<T>(K, F, tab_d, tab_omd);
  const Layout& L = F.L;
  const Layout& CL = C.L;
  double acc[1] = {0.0};
  const int per = (int)(gridDim.x >> 3);
  const int lb = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  if (lb < ntot) {
    const int tile = lb / nchunk, ch = lb - tile * nchunk;
    const int jt = tile / nkt, kt = tile - jt * nkt;
    const int j0 = jt * U::FJ, k0 = kt * U::FK;
    const int i0 = ch * nfi, i1 = min(L.nx, i0 + nfi);
    const int tid = threadIdx.x;
    if (tid < U::TJ) {
      const Tap2<T> b = ptap(j0 - 1 + tid, 1, CL.ny, K.sgn[2], K.sgn[3]);
      rt_o[tid][0] = (clampg(b.i0, CL.ny) + 1) * CL.PZ;
      rt_o[tid][1] = (clampg(b.i1, CL.ny) + 1) * CL.PZ;
      rt_w[tid][0] = b.w0;
      rt_w[tid][1] = b.w1;
    } else if (tid >= 64 && tid < 64 + U::TK) {
      const Tap2<T> e = ptap(k0 - 1 + tid - 64, 1, CL.nz, K.sgn[4], K.sgn[5]);
      ct_o[tid - 64][0] = clampg(e.i0, CL.nz) + 1;
      ct_o[tid - 64][1] = clampg(e.i1, CL.nz) + 1;
      ct_w[tid - 64][0] = e.w0;
      ct_w[tid - 64][1] = e.w1;
    }
    // the thread's region entries: its NU fine columns (rows jr + ROWS u)
    // and at most one entry of the ring around them (entry NU)
    constexpr int NU = U::NU, NV = NU + 1;
    const int kk = tid % U::FK, jr = tid / U::FK;
    int ej[NV], ek[NV];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      ej[u] = jr + U::ROWS * u + 1;
      ek[u] = kk + 1;
    }
    const bool ring = tid < NRING;
    {
      const int q = ring ? tid : 0;
      if (q < U::TK) {
        ej[NU] = 0;
        ek[NU] = q;
      } else if (q < 2 * U::TK) {
        ej[NU] = U::TJ - 1;
        ek[NU] = q - U::TK;
      } else {
        const int r = q - 2 * U::TK;
        ej[NU] = 1 + (r >> 1);
        ek[NU] = (r & 1) ? U::TK - 1 : 0;
      }
    }
    int pos[NV], cyz[NV];
    bool in[NV];
    long long ro[NV];   // offset of (j, k) within a fine plane (clamped into the ghosts)
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int j = j0 - 1 + ej[v], k = k0 - 1 + ek[v];
      pos[v] = ej[v] * U::TK + ek[v];
      cyz[v] = (bclass(j, L.ny) << 2) | bclass(k, L.nz);
      in[v] = (unsigned)j < (unsigned)L.ny && (unsigned)k < (unsigned)L.nz && (v < NU || ring);
      ro[v] = (long long)(clampg(j, L.ny) + 1) * L.PZ + (clampg(k, L.nz) + 1);
    }
    __syncthreads();   // tap tables in place
    // Y(I) at the region: the y/z interpolation of coarse plane I
    auto make_y = [&](int I) {
      T* y = sy[(I + 3) % 3];
      const T* xc = C.x + (long long)(clampg(I, CL.nx) + 1) * CL.SX;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (v == NU && !ring) continue;
        const int r0 = rt_o[ej[v]][0], r1 = rt_o[ej[v]][1], q0 = ct_o[ek[v]][0], q1 = ct_o[ek[v]][1];
        const T bw0 = rt_w[ej[v]][0], bw1 = rt_w[ej[v]][1], ew0 = ct_w[ek[v]][0], ew1 = ct_w[ek[v]][1];
        y[pos[v]] = bw0 * (ew0 * xc[r0 + q0] + ew1 * xc[r0 + q1]) + bw1 * (ew0 * xc[r1 + q0] + ew1 * xc[r1 + q1]);
      }
    };
    T rv[NV];
    auto load_r = [&](int i) {
      const T* rp = F.r + (long long)(clampg(i, L.nx) + 1) * L.SX;
#pragma unroll
      for (int v = 0; v < NV; ++v) rv[v] = (v < NU || ring) ? rp[ro[v]] : T(0);
    };
    const int ts = i0 - 1, te = i1;   // t planes of the chunk
    int ymax = (ts >> 1) + 1;
    for (int I = (ts >> 1) - 1; I <= ymax; ++I) make_y(I);
    load_r(ts);
    T tm[NU], tc[NU], tn[NU], rc[NU], rn[NU];   // own t(i-2), t(i-1), t(i); own r(i-1), r(i)
#pragma unroll
    for (int u = 0; u < NU; ++u) tm[u] = tc[u] = tn[u] = rc[u] = rn[u] = T(0);
    for (int i = ts; i <= te; ++i) {
      __syncthreads();   // the Y planes of plane i are in place; t slot i % 3 is free
      const Tap2<T> a = ptap(i, 1, CL.nx, K.sgn[0], K.sgn[1]);
      const T* ya = sy[(a.i0 + 3) % 3];
      const T* yb = sy[(a.i1 + 3) % 3];
      T* t = st[(i + 3) % 3];
      const bool iin = (unsigned)i < (unsigned)L.nx;
      const int cx = bclass(i, L.nx) << 4;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (v == NU && !ring) continue;
        const T tv = (iin && in[v]) ? tab_omd[cx | cyz[v]] * rv[v] + a.w0 * ya[pos[v]] + a.w1 * yb[pos[v]] : T(0);
        t[pos[v]] = tv;
        if (v < NU) {
          tn[v] = tv;
          rn[v] = rv[v];
        }
      }
      if (i < te) {
        load_r(i + 1);
        // an odd next plane needs the coarse plane past the ones held
        const int need = ((i + 1) & 1) ? ((i + 1) >> 1) + 1 : ((i + 1) >> 1);
        if (need > ymax) {
          ymax = need;
          make_y(ymax);
        }
      }
      __syncthreads();
      // z of plane i - 1 on the own columns, from t(i-2), t(i-1), t(i)
      const int iz = i - 1;
      if (iz >= i0 && iz < i1) {
        const T* tp = st[(iz + 3) % 3];
        const int czx = bclass(iz, L.nx) << 4;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          if (!in[u]) continue;
          const int cl = czx | cyz[u];
          const int q = pos[u];
          const T At = tab_d[cl] * tc[u] - F.w[0] * (tn[u] + tm[u]) - F.w[1] * (tp[q + U::TK] + tp[q - U::TK]) -
                       F.w[2] * (tp[q + 1] + tp[q - 1]);
          const T z = tc[u] + tab_omd[cl] * (rc[u] - At);
          F.x[(long long)(iz + 1) * L.SX + ro[u]] = z;
          acc[0] += (double)rc[u] * (double)z;
        }
      }
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        tm[u] = tc[u];
        tc[u] = tn[u];
        rc[u] = rn[u];
      }
    }
  }
  const int slots[1] = {S_RZ0 + (m & 1)};
  write_partials<1>(acc, c.part, c.stride, slots, (int)blockIdx.x);
}

// Levels of at most `cells` cells run in the single-workgroup kernel, with
// r, x and t of all of them in an LDS pool of `pool` cells per array (a
// hierarchy whose small levels need more takes the global-memory variant).
template <class T>
struct TailCfg;
template <>
struct TailCfg<float> {
  // larger small levels are faster as separate multi-block kernels (one
  // workgroup took 40 us for 8192 cells and below, the kernels 22 us)
  static constexpr long long cells = 1024;
  static constexpr int pool = 2048;
};
template <>
struct TailCfg<double> {
  static constexpr long long cells = 1024;
  static constexpr int pool = 2048;
};

// All levels from lt down to the coarsest and back in one workgroup, with
// every level's r, x and t in LDS (compact k-fastest order, no ghosts;
// neighbours outside a level read as 0).  Level lt's r comes from and its x
// goes to global memory.  Level descriptors are read from a device table.
template <class T>
__global__ __launch_bounds__(kTailThreads) void k_mg_tail(MgCommon<T> K, const MgLvl<T>* __restrict__ lv, int lt,
                                                          int nl, const T* __restrict__ cinv,
                                                          const int* __restrict__ flags, int m) {
  const int skip = flags[m];   // tested once level lt is staged
  constexpr int kTailPool = TailCfg<T>::pool;
  __shared__ T pr[kTailPool];
  __shared__ T px[kTailPool];
  __shared__ T pt[kTailPool];
  __shared__ T tab_d[kMgMaxLevels * 64];
  __shared__ T tab_omd[kMgMaxLevels * 64];
  const int tid = threadIdx.x;
  auto offset = [&](int l) {
    int o = 0;
    for (int q = lt; q < l; ++q) o += (int)ncells(lv[q].L);
    return o;
  };
  auto cid = [](const Layout& L, int i, int j, int k) { return (i * L.ny + j) * L.nz + k; };
  // value of a compact level array at (i, j, k); 0 outside the level
  auto at = [&](const T* a, const Layout& L, int i, int j, int k) {
    return inside(L, i, j, k) ? a[cid(L, i, j, k)] : T(0);
  };
  for (int e = tid; e < (nl - lt) * 64; e += blockDim.x) {
    const MgLvl<T> F = lv[lt + e / 64];
    const T D = class_diag(K, F, e % 64);
    tab_d[e] = D;
    tab_omd[e] = D > T(0) ? K.om / D : T(0);
  }
  {
    const MgLvl<T> F = lv[lt];
    const int nf = (int)ncells(F.L);
    for (int idx = tid; idx < nf; idx += blockDim.x) {
      int i, j, k;
      decode(idx, F.L, i, j, k);
      pr[idx] = F.r[F.L.at(i, j, k)];
    }
  }
  if (skip) return;
  __syncthreads();
  for (int l = lt; l < nl - 1; ++l) {
    const MgLvl<T> F = lv[l];
    const MgLvl<T> C = lv[l + 1];
    const T* om_l = tab_omd + (l - lt) * 64;
    const int of = offset(l), oc = of + (int)ncells(F.L);
    const int nf = (int)ncells(F.L), nc = (int)ncells(C.L);
    const T* r = pr + of;
    T* t = pt + of;
    for (int idx = tid; idx < nf; idx += blockDim.x) {
      int i, j, k;
      decode(idx, F.L, i, j, k);
      // e = om D^-1 r, 0 outside the level
      auto e = [&](int a, int b, int q) { return om_l[cls3(F.L, a, b, q)] * at(r, F.L, a, b, q); };
      t[idx] = (T(1) - K.om) * r[idx] + F.w[0] * (e(i + 1, j, k) + e(i - 1, j, k)) +
               F.w[1] * (e(i, j + 1, k) + e(i, j - 1, k)) + F.w[2] * (e(i, j, k + 1) + e(i, j, k - 1));
    }
    __syncthreads();
    for (int idx = tid; idx < nc; idx += blockDim.x) {
      int I, J, Kc;
      decode(idx, C.L, I, J, Kc);
      pr[oc + idx] = restrict_at(K, F, C, I, J, Kc, [&](int i, int j, int k) { return t[cid(F.L, i, j, k)]; });
    }
    __syncthreads();
  }
  {
    const MgLvl<T> B = lv[nl - 1];
    const T* d_b = tab_d + (nl - 1 - lt) * 64;
    const T* om_b = tab_omd + (nl - 1 - lt) * 64;
    const int ob = offset(nl - 1);
    const int nb = (int)ncells(B.L);
    const T* r = pr + ob;
    if (cinv) {
      // x = Ainv r: tpr lanes per row (power of two <= 64), partial sums
      // combined with lane shuffles
      int tpr = 1;
      while (tpr < 64 && tpr * 2 * nb <= (int)blockDim.x) tpr *= 2;
      for (int base = 0; base < nb * tpr; base += blockDim.x) {
        const int row = (base + tid) / tpr, lane = (base + tid) % tpr;
        T s = T(0);
        if (row < nb)
          for (int col = lane; col < nb; col += tpr) s += cinv[(size_t)row * nb + col] * r[col];
        for (int w = 1; w < tpr; w *= 2) s += __shfl_xor(s, w, 64);
        if (row < nb && lane == 0) px[ob + row] = s;
      }
      __syncthreads();
    } else {
      // fixed Jacobi sweeps from zero (symmetric, positive definite for om <= 1)
      T* xa = px + ob;
      T* xb = pt + ob;
      for (int idx = tid; idx < nb; idx += blockDim.x) xa[idx] = T(0);
      __syncthreads();
      for (int sw = 0; sw < kCoarseSweeps; ++sw) {
        for (int idx = tid; idx < nb; idx += blockDim.x) {
          int i, j, k;
          decode(idx, B.L, i, j, k);
          const int cl = cls3(B.L, i, j, k);
          const T Ax = d_b[cl] * xa[idx] - B.w[0] * (at(xa, B.L, i + 1, j, k) + at(xa, B.L, i - 1, j, k)) -
                       B.w[1] * (at(xa, B.L, i, j + 1, k) + at(xa, B.L, i, j - 1, k)) -
                       B.w[2] * (at(xa, B.L, i, j, k + 1) + at(xa, B.L, i, j, k - 1));
          xb[idx] = xa[idx] + om_b[cl] * (r[idx] - Ax);
        }
        __syncthreads();
        T* tmp = xa;
        xa = xb;
        xb = tmp;
      }
      if (xa != px + ob) {
        for (int idx = tid; idx < nb; idx += blockDim.x) px[ob + idx] = xa[idx];
        __syncthreads();
      }
    }
  }
  for (int l = nl - 2; l >= lt; --l) {
    const MgLvl<T> F = lv[l];
    const MgLvl<T> C = lv[l + 1];
    const T* d_l = tab_d + (l - lt) * 64;
    const T* om_l = tab_omd + (l - lt) * 64;
    const int of = offset(l), oc = of + (int)ncells(F.L);
    const int nf = (int)ncells(F.L);
    const T* r = pr + of;
    const T* xc = px + oc;
    T* t = pt + of;
    for (int idx = tid; idx < nf; idx += blockDim.x) {
      int i, j, k;
      decode(idx, F.L, i, j, k);
      const Tap2<T> a = ptap(i, F.c[0], C.L.nx, K.sgn[0], K.sgn[1]);
      const Tap2<T> b = ptap(j, F.c[1], C.L.ny, K.sgn[2], K.sgn[3]);
      const Tap2<T> e = ptap(k, F.c[2], C.L.nz, K.sgn[4], K.sgn[5]);
      auto row = [&](int I, int J) { return e.w0 * xc[cid(C.L, I, J, e.i0)] + e.w1 * xc[cid(C.L, I, J, e.i1)]; };
      t[idx] = om_l[cls3(F.L, i, j, k)] * r[idx] + a.w0 * (b.w0 * row(a.i0, b.i0) + b.w1 * row(a.i0, b.i1)) +
               a.w1 * (b.w0 * row(a.i1, b.i0) + b.w1 * row(a.i1, b.i1));
    }
    __syncthreads();
    for (int idx = tid; idx < nf; idx += blockDim.x) {
      int i, j, k;
      decode(idx, F.L, i, j, k);
      const int cl = cls3(F.L, i, j, k);
      const T At = d_l[cl] * t[idx] - F.w[0] * (at(t, F.L, i + 1, j, k) + at(t, F.L, i - 1, j, k)) -
                   F.w[1] * (at(t, F.L, i, j + 1, k) + at(t, F.L, i, j - 1, k)) -
                   F.w[2] * (at(t, F.L, i, j, k + 1) + at(t, F.L, i, j, k - 1));
      px[of + idx] = t[idx] + om_l[cl] * (r[idx] - At);
    }
    __syncthreads();
  }
  {
    const MgLvl<T> F = lv[lt];
    const int nf = (int)ncells(F.L);
    for (int idx = tid; idx < nf; idx += blockDim.x) {
      int i, j, k;
      decode(idx, F.L, i, j, k);
      F.x[F.L.at(i, j, k)] = px[idx];
    }
  }
}

// The same in global memory (arrays that stay in the L2), for hierarchies
// whose small levels do not fit the LDS pool (e.g. a large coarsest level
// left where no axis can be halved).
template <class T>
__global__ __launch_bounds__(kTailThreads) void k_mg_tail_global(MgCommon<T> K, const MgLvl<T>* __restrict__ lv, int lt,
                                                          int nl, const T* __restrict__ cinv,
                                                          const int* __restrict__ flags, int m) {
  if (flags[m]) return;
  __shared__ T rs[kDenseMax];
  for (int l = lt; l < nl - 1; ++l) {
    const MgLvl<T> F = lv[l];
    const MgLvl<T> C = lv[l + 1];
    const int nf = (int)ncells(F.L), nc = (int)ncells(C.L);
    for (int idx = threadIdx.x; idx < nf; idx += blockDim.x) {
      int i, j, k;
      decode(idx, F.L, i, j, k);
      F.t[F.L.at(i, j, k)] = smoothed_residual(K, F, F.r, i, j, k);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nc; idx += blockDim.x) {
      int I, J, Kc;
      decode(idx, C.L, I, J, Kc);
      const T* __restrict__ res = F.t;
      C.r[C.L.at(I, J, Kc)] =
          restrict_at(K, F, C, I, J, Kc, [&](int i, int j, int k) { return res[F.L.at(i, j, k)]; });
    }
    __syncthreads();
  }
  {
    const MgLvl<T> B = lv[nl - 1];
    const int nb = (int)ncells(B.L);
    if (cinv) {
      for (int idx = threadIdx.x; idx < nb; idx += blockDim.x) {
        int i, j, k;
        decode(idx, B.L, i, j, k);
        rs[idx] = B.r[B.L.at(i, j, k)];
      }
      __syncthreads();
      for (int row = threadIdx.x; row < nb; row += blockDim.x) {
        T s = T(0);
        const T* a = cinv + (size_t)row * nb;
        for (int col = 0; col < nb; ++col) s += a[col] * rs[col];
        int i, j, k;
        decode(row, B.L, i, j, k);
        B.x[B.L.at(i, j, k)] = s;
      }
      __syncthreads();
    } else {
      // fixed Jacobi sweeps from zero (symmetric, positive definite for om <= 1)
      T* xa = B.x;
      T* xb = B.t;
      for (int idx = threadIdx.x; idx < nb; idx += blockDim.x) {
        int i, j, k;
        decode(idx, B.L, i, j, k);
        xa[B.L.at(i, j, k)] = T(0);
      }
      __syncthreads();
      for (int sw = 0; sw < kCoarseSweeps; ++sw) {
        for (int idx = threadIdx.x; idx < nb; idx += blockDim.x) {
          int i, j, k;
          decode(idx, B.L, i, j, k);
          const long long o = B.L.at(i, j, k);
          xb[o] = xa[o] + omd(K, B, i, j, k) * (B.r[o] - apply_w(K.bc, B.L, B.w, xa, i, j, k, o));
        }
        __syncthreads();
        T* tmp = xa;
        xa = xb;
        xb = tmp;
      }
      if (xa != B.x) {
        for (int idx = threadIdx.x; idx < nb; idx += blockDim.x) {
          int i, j, k;
          decode(idx, B.L, i, j, k);
          const long long o = B.L.at(i, j, k);
          B.x[o] = xa[o];
        }
        __syncthreads();
      }
    }
  }
  for (int l = nl - 2; l >= lt; --l) {
    const MgLvl<T> F = lv[l];
    const MgLvl<T> C = lv[l + 1];
    const int nf = (int)ncells(F.L);
    for (int idx = threadIdx.x; idx < nf; idx += blockDim.x) {
      int i, j, k;
      decode(idx, F.L, i, j, k);
      F.t[F.L.at(i, j, k)] = pre_plus_coarse<true>(K, F, C, i, j, k);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nf; idx += blockDim.x) {
      int i, j, k;
      decode(idx, F.L, i, j, k);
      const long long o = F.L.at(i, j, k);
      // t has zero ghosts: apply_w gives A t directly
      F.x[o] = F.t[o] + omd(K, F, i, j, k) * (F.r[o] - apply_w(K.bc, F.L, F.w, F.t, i, j, k, o));
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------- host
template <class T>
static MgCommon<T> mg_common(const Grid& g) {
  MgCommon<T> K{};
  for (int q = 0; q < 6; ++q) {
    K.bc[q] = g.bc[q];
    K.sgn[q] = g.bc[q] == OUTLET ? T(-1) : T(1);
  }
  K.om = T(g.mg_omega);
  return K;
}

template <class T>
static MgLvl<T> mg_level(const Grid& g, int l) {
  const MgLevel& S = g.mg[l];
  MgLvl<T> D{};
  D.L = S.L;
  for (int a = 0; a < 3; ++a) {
    D.w[a] = T(S.w[a]);
    D.c[a] = S.coarsen[a];
  }
  D.omd_in = T(g.mg_omega / (2.0 * (S.w[0] + S.w[1] + S.w[2])));
  D.r = (T*)S.r;
  D.x = (T*)S.x;
  D.t = (T*)S.t;
  return D;
}

void mg_free(Grid& g) {
  for (size_t l = 1; l < g.mg.size(); ++l) {
    gfree(g, g.mg[l].r);
    gfree(g, g.mg[l].x);
    gfree(g, g.mg[l].t);
  }
  g.mg.clear();
  gfree(g, g.mg_cinv);
  g.mg_cinv = nullptr;
  gfree(g, g.mg_table);
  g.mg_table = nullptr;
}

static Layout level_layout(int nx, int ny, int nz) {
  Layout L;
  L.nx = nx;
  L.ny = ny;
  L.nz = nz;
  L.PZ = nz + 3;
  L.SX = (long long)(ny + 3) * L.PZ;
  return L;
}

// Dense inverse of the coarsest operator (Gauss-Jordan in double on the
// host; the operator is symmetric positive definite).
static bool dense_inverse(const MgLevel& B, const int bc[6], std::vector<double>& inv) {
  const int nx = B.L.nx, ny = B.L.ny, nz = B.L.nz, n = nx * ny * nz;
  if (n > kDenseMax) return false;
  std::vector<double> A((size_t)n * n, 0.0);
  auto id = [&](int i, int j, int k) { return (i * ny + j) * nz + k; };
  const int nn[3] = {nx, ny, nz};
  for (int i = 0; i < nx; ++i)
    for (int j = 0; j < ny; ++j)
      for (int k = 0; k < nz; ++k) {
        const int c = id(i, j, k);
        const int idx[3] = {i, j, k};
        double d = 0;
        for (int a = 0; a < 3; ++a)
          for (int s = -1; s <= 1; s += 2) {
            int q[3] = {i, j, k};
            q[a] += s;
            const bool inside = q[a] >= 0 && q[a] < nn[a];
            if (inside) {
              d += B.w[a];
              A[(size_t)c * n + id(q[0], q[1], q[2])] -= B.w[a];
            } else if (bc[2 * a + (s > 0)] == OUTLET) {
              d += B.w[a];
            }
            (void)idx;
          }
        A[(size_t)c * n + c] = d;
      }
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + col]) > std::fabs(A[(size_t)piv * n + col])) piv = r;
    if (A[(size_t)piv * n + col] == 0.0) return false;
    if (piv != col)
      for (int q = 0; q < n; ++q) {
        std::swap(A[(size_t)piv * n + q], A[(size_t)col * n + q]);
        std::swap(inv[(size_t)piv * n + q], inv[(size_t)col * n + q]);
      }
    const double p = 1.0 / A[(size_t)col * n + col];
    for (int q = 0; q < n; ++q) {
      A[(size_t)col * n + q] *= p;
      inv[(size_t)col * n + q] *= p;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = A[(size_t)r * n + col];
      if (f == 0.0) continue;
      for (int q = 0; q < n; ++q) {
        A[(size_t)r * n + q] -= f * A[(size_t)col * n + q];
        inv[(size_t)r * n + q] -= f * inv[(size_t)col * n + q];
      }
    }
  }
  return true;
}

template <class T>
void mg_setup(Grid& g) {
  mg_free(g);
  const size_t es = sizeof(T);
  MgLevel l0;
  l0.L = g.L;
  l0.w[0] = 1.0 / (g.cfg.dx * g.cfg.dx);
  l0.w[1] = 1.0 / (g.cfg.dy * g.cfg.dy);
  l0.w[2] = 1.0 / (g.cfg.dz * g.cfg.dz);
  g.mg.push_back(l0);
  while ((int)g.mg.size() < kMgMaxLevels) {
    MgLevel& F = g.mg.back();
    const int n[3] = {F.L.nx, F.L.ny, F.L.nz};
    if (ncells(F.L) <= kCoarsestCells) break;
    // every axis of at least 4 cells is halved; an odd one gets ceil(n/2)
    // coarse cells, the last of which has a single child
    int c[3], any = 0;
    for (int a = 0; a < 3; ++a) {
      c[a] = n[a] >= 4 ? 1 : 0;
      any |= c[a];
    }
    if (!any) break;
    MgLevel C;
    C.L = level_layout((n[0] + c[0]) >> c[0], (n[1] + c[1]) >> c[1], (n[2] + c[2]) >> c[2]);
    for (int a = 0; a < 3; ++a) {
      F.coarsen[a] = c[a];
      C.w[a] = F.w[a] / (c[a] ? 4.0 : 1.0);   // re-discretised with the doubled spacing
    }
    const size_t bytes = (size_t)(C.L.nx + 3) * C.L.SX * es;
    for (void** q : {&C.r, &C.x, &C.t}) {
      *q = galloc(g, bytes);
      UF_HIP_CHECK(hipMemsetAsync(*q, 0, bytes, g.stream));
    }
    g.mg.push_back(C);
  }
  MgLevel& last = g.mg.back();
  for (int a = 0; a < 3; ++a) last.coarsen[a] = 0;
  const int nl = (int)g.mg.size();
  // first small level (>= 1) for the single-workgroup kernel
  g.mg_lt = nl;
  for (int l = 1; l < nl; ++l)
    if (ncells(g.mg[l].L) <= TailCfg<T>::cells) {
      g.mg_lt = l;
      break;
    }
  // the coarsest level is always solved by the single-workgroup kernel
  if (nl > 1 && g.mg_lt > nl - 1) g.mg_lt = nl - 1;
  {
    long long pool = 0;
    for (int l = std::min(g.mg_lt, nl - 1); l < nl; ++l) pool += ncells(g.mg[l].L);
    g.mg_tail_lds = pool <= TailCfg<T>::pool;
  }
  g.mg_cinv = nullptr;
  g.mg_nc = (int)ncells(last.L);
  g.mg_omega = kJacobiOmega;
  {
    std::vector<MgLvl<T>> tab(nl);
    for (int l = 0; l < nl; ++l) tab[l] = mg_level<T>(g, l);
    g.mg_table = galloc(g, tab.size() * sizeof(MgLvl<T>));
    upload(g, g.mg_table, tab.data(), tab.size() * sizeof(MgLvl<T>));
  }
  if (nl > 1) {
    std::vector<double> inv;
    if (dense_inverse(last, g.bc, inv)) {
      std::vector<T> tv(inv.begin(), inv.end());
      g.mg_cinv = galloc(g, tv.size() * es);
      upload(g, g.mg_cinv, tv.data(), tv.size() * es);
    }
  }
}

static bool big_tile(const Layout& L) { return ncells(L) >= kUpBigCells; }

template <class Tile>
static int3 up_tiles(const Layout& F) {
  return make_int3((F.nz + Tile::TK - 1) / Tile::TK, (F.ny + Tile::TJ - 1) / Tile::TJ, (F.nx + Tile::TI - 1) / Tile::TI);
}

// Blocks of a persistent level kernel over nt tiles.
static int level_blocks(long long nt) {
  const long long cap = (long long)kCUs * kLevelBlocksPerCU;
  return (int)std::max(1LL, std::min(nt, cap));
}

// Blocks of the fine up/smoothing kernel (one r.z partial each).
size_t mg_fine_blocks(const Layout& L) {
  if (up_march(L)) return (size_t)(8 * ((up_geom(L).ntot + 7) / 8));
  const int3 t = big_tile(L) ? up_tiles<UpBig>(L) : up_tiles<UpSmall>(L);
  return (size_t)level_blocks((long long)t.x * t.y * t.z);
}

template <class T>
static int3 restrict_tiles(const Layout& C) {
  using Rt = RTile<T>;
  return make_int3((C.nz + Rt::CK - 1) / Rt::CK, (C.ny + Rt::CJ - 1) / Rt::CJ, (C.nx + Rt::CI - 1) / Rt::CI);
}

template <class T>
static void launch_restrict(Grid& g, const MgCommon<T>& K, const MgLvl<T>& F, const MgLvl<T>& C, int has_coarse,
                            const CgCtl& c, int m, int mode, const CgUpd<T>* upd = nullptr) {
  const int3 nt3 = has_coarse ? restrict_tiles<T>(C.L) : make_int3(1, 1, 1);
  // mode 1 adds the deciding block after the tile walkers
  const int G = has_coarse ? level_blocks((long long)nt3.x * nt3.y * nt3.z) + (!upd && mode == 1 ? 1 : 0) : 1;
  if (upd)
    launch_k(g, k_mg_restrict<true, T>, dim3(G), dim3(256), K, F, C, has_coarse, c, m, mode, nt3, *upd);
  else
    launch_k(g, k_mg_restrict<false, T>, dim3(G), dim3(256), K, F, C, has_coarse, c, m, mode, nt3, CgUpd<T>{});
}

// Launch geometry of the marching update + restriction: coarse column
// tiles of 8 x 32, x-chunks of nci coarse planes, about 1024 blocks.  It
// is taken when every axis of level 0 is halved and the coarse level is at
// least 32 cells deep (narrower tiles would leave most threads idle).
struct MarchGeom {
  int nci = 0, nkt = 0, nchunk = 0, ntot = 0;
  bool use = false;
};

static MarchGeom march_geom(const MgLevel& F, const MgLevel& C) {
  MarchGeom m;
  if (!(F.coarsen[0] && F.coarsen[1] && F.coarsen[2]) || C.L.nz < 32) return m;
  const int njt = (C.L.ny + 7) / 8, nkt = (C.L.nz + 31) / 32;
  const int tiles = njt * nkt;
  const int want = std::max(1, std::min(C.L.nx, (1024 + tiles - 1) / tiles));
  m.nci = (C.L.nx + want - 1) / want;
  m.nchunk = (C.L.nx + m.nci - 1) / m.nci;
  m.nkt = nkt;
  m.ntot = tiles * m.nchunk;
  // a chunk re-reads four fine planes around its own: below 8 coarse planes
  // per chunk (256x256x64: 2) the tiled kernel moves fewer bytes
  m.use = m.nci >= 8;
  return m;
}

bool mg_splits_update(const Grid& g) {
  return g.mg_fused && g.mg.size() > 1 && march_geom(g.mg[0], g.mg[1]).use;
}

// Launch size of a marching restriction: 8 * ceil(n / 8) blocks for the
// ntot walkers and, in mode 1, the deciding block (logical block ntot).
static int march_blocks(const MarchGeom& m, int mode) {
  const int n = m.ntot + (mode == 1 ? 1 : 0);
  return 8 * ((n + 7) / 8);
}

template <class T>
static void launch_march_restrict(Grid& g, const MgCommon<T>& K, const MgLvl<T>& F, const MgLvl<T>& C,
                                  const MarchGeom& mgeo, const CgCtl& c, int m, int mode) {
  launch_k(g, k_mg_update_march<false, T>, dim3(march_blocks(mgeo, mode)), dim3(256), K, F, C, c, CgUpd<T>{},
           mgeo.nci, mgeo.nkt, mgeo.nchunk, mgeo.ntot, m, mode);
}

// Blocks of the level-0 restriction when it carries the CG update (the
// writer of the r.r partials besides the CG kernels), or 0 when the update
// stays separate: it needs a coarse restriction kernel after it to decide
// whether the solve has finished.
size_t mg_fused_blocks(const Grid& g) {
  const int nl = (int)g.mg.size();
  if (g.cfg.precond != UF_PC_MG || nl < 3 || std::min(g.mg_lt, nl - 1) < 2) return 0;
  const MarchGeom mg = march_geom(g.mg[0], g.mg[1]);
  if (mg.use) return (size_t)march_blocks(mg, 0);
  const Layout& C = g.mg[1].L;
  const int3 nt3 = g.esize == 4 ? restrict_tiles<float>(C) : restrict_tiles<double>(C);
  return (size_t)level_blocks((long long)nt3.x * nt3.y * nt3.z);
}

template <bool FINE, bool COARSE, class Tile, class T>
static void launch_up_t(Grid& g, const MgCommon<T>& K, const MgLvl<T>& F, const MgLvl<T>& C, const CgCtl& c, int m) {
  const int3 nt3 = up_tiles<Tile>(F.L);
  const int G = level_blocks((long long)nt3.x * nt3.y * nt3.z);
  if (COARSE && F.c[0] && F.c[1] && F.c[2])
    launch_k(g, k_mg_upsmooth<FINE, COARSE, true, Tile, T>, dim3(G), dim3(256), K, F, C, c, m, nt3);
  else
    launch_k(g, k_mg_upsmooth<FINE, COARSE, false, Tile, T>, dim3(G), dim3(256), K, F, C, c, m, nt3);
}

template <bool FINE, bool COARSE, class T>
static void launch_up(Grid& g, const MgCommon<T>& K, const MgLvl<T>& F, const MgLvl<T>& C, const CgCtl& c, int m) {
  if (big_tile(F.L))
    launch_up_t<FINE, COARSE, UpBig, T>(g, K, F, C, c, m);
  else
    launch_up_t<FINE, COARSE, UpSmall, T>(g, K, F, C, c, m);
}

template <class T>
void mg_launch(Grid& g, const Params<T>& P, int m, const void* r, void* z, int decide,
               const CgUpd<T>* upd = nullptr) {
  (void)P;
  const MgCommon<T> K = mg_common<T>(g);
  const CgCtl c = make_ctl(g);
  const int nl = (int)g.mg.size();
  MgLvl<T> L0 = mg_level<T>(g, 0);
  L0.r = (T*)r;
  L0.x = (T*)z;
  const MgLvl<T> L1 = nl > 1 ? mg_level<T>(g, 1) : L0;
  bool xfork = false;   // x += alpha d runs on the second stream
  hipEvent_t fork = nullptr;   // completed by the restriction's dispatch
  const MarchGeom mgeo = nl > 1 ? march_geom(g.mg[0], g.mg[1]) : MarchGeom{};
  {
    TimedLaunch tl(g, upd ? (mgeo.use ? UF_TK_MG_RUPD0 : UF_TK_MG_UPDATE0) : UF_TK_MG_DOWN0);
    if (mgeo.use && upd)
      fork = launch_k_done(g, g.ev_xfork, k_mg_update_march<true, T>, dim3(march_blocks(mgeo, 0)), dim3(256), K,
                           L0, L1, c, *upd, mgeo.nci, mgeo.nkt, mgeo.nchunk, mgeo.ntot, m, 0);
    else if (mgeo.use)
      launch_march_restrict<T>(g, K, L0, L1, mgeo, c, m, decide ? 1 : 2);
    else
      launch_restrict<T>(g, K, L0, L1, nl > 1 ? 1 : 0, c, m, decide ? 1 : 2, upd);
  }
  if (mgeo.use && upd) {
    if (!g.xstream) throw HipError("the second solve stream is missing");   // made with the grid (mg_splits_update)
    // x += alpha d of the iteration on the second stream, beside the
    // coarse levels; joined before the next iteration (at 256x256x64,
    // where the tiled kernel keeps the update, a separate pass and the
    // stream switch cost more than they save: 1.34 -> 1.43 ms per step)
    UF_HIP_CHECK(hipStreamWaitEvent(g.xstream, fork, 0));
    hipLaunchKernelGGL(k_cg_xupd<T>, dim3(1024), dim3(256), 0, g.xstream, L0.L, upd->X, upd->D, c, upd->t);
    UF_HIP_CHECK(hipEventRecord(g.ev_xjoin, g.xstream));
    xfork = true;
  }
  const int lt = std::min(g.mg_lt, nl - 1);
  for (int l = 1; l < lt; ++l) {
    const MgLvl<T> F = mg_level<T>(g, l), C = mg_level<T>(g, l + 1);
    TimedLaunch tl(g, UF_TK_MG_COARSE);
    // after a fused update the first coarse restriction takes the decision
    // (the coarse levels keep the tiled kernel: their x-chunks of a few
    // planes would re-read as much as they restrict)
    launch_restrict<T>(g, K, F, C, 1, c, m, (upd && l == 1) ? 1 : 0);
  }
  if (nl > 1) {
    {
      TimedLaunch tl(g, UF_TK_MG_COARSE);
      if (g.mg_tail_lds)
        launch_k(g, k_mg_tail<T>, dim3(1), dim3(kTailThreads), K, (const MgLvl<T>*)g.mg_table, lt, nl,
                 (const T*)g.mg_cinv, (const int*)c.flags, m);
      else
        launch_k(g, k_mg_tail_global<T>, dim3(1), dim3(kTailThreads), K, (const MgLvl<T>*)g.mg_table, lt, nl,
                 (const T*)g.mg_cinv, (const int*)c.flags, m);
    }
    for (int l = lt - 1; l >= 1; --l) {
      const MgLvl<T> F = mg_level<T>(g, l), C = mg_level<T>(g, l + 1);
      TimedLaunch tl(g, UF_TK_MG_COARSE);
      launch_up<false, true, T>(g, K, F, C, c, m);
    }
  }
  {
    TimedLaunch tl(g, UF_TK_MG_UP0);
    if (nl > 1 && up_march(L0.L)) {
      const UpGeom u = up_geom(L0.L);
      launch_k(g, k_mg_upsmooth_march<T>, dim3(8 * ((u.ntot + 7) / 8)), dim3(UTile::NTH), K, L0, L1, c, m, u.nfi,
               u.nkt, u.nchunk, u.ntot);
    } else if (nl > 1)
      launch_up<true, true, T>(g, K, L0, L1, c, m);
    else
      launch_up<true, false, T>(g, K, L0, L1, c, m);
  }
  if (xfork) g.xpending = true;   // joined by the next d/q kernel or the solve's end
}

template <class T>
void mg_precond(Grid& g, const Params<T>& P, int m) {
  mg_launch<T>(g, P, m, resid(g, m), g.Z, 1);
}

// CG update of iteration t and the preconditioner application that follows
// (m = t + 1), the update inside the level-0 restriction.
template <class T>
void mg_iteration_update(Grid& g, const Params<T>& P, int t, const void* Dnew) {
  const CgUpd<T> upd{(T*)g.X, (const T*)resid(g, t), (const T*)Dnew, (const T*)g.Qv, t};
  mg_launch<T>(g, P, t + 1, resid(g, t + 1), g.Z, 1, &upd);
}

// Stand-alone application z = M^-1 r: uses the spare flag slot past the
// iteration range and applies the cycle unconditionally.  The r.z partials
// it writes are not used.
template <class T>
void mg_apply(Grid& g, const Params<T>& P, const void* r, void* z) {
  mg_launch<T>(g, P, g.cfg.cg_maxit + 1, r, z, 0);
}

template void mg_setup<float>(Grid&);
template void mg_setup<double>(Grid&);
template void mg_precond<float>(Grid&, const Params<float>&, int);
template void mg_precond<double>(Grid&, const Params<double>&, int);
template void mg_iteration_update<float>(Grid&, const Params<float>&, int, const void*);
template void mg_iteration_update<double>(Grid&, const Params<double>&, int, const void*);
template void mg_apply<float>(Grid&, const Params<float>&, const void*, void*);
template void mg_apply<double>(Grid&, const Params<double>&, const void*, void*);

}  // namespace uf
