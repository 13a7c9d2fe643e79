// Geometric multigrid V-cycle used as the CG preconditioner.
//
// Cell-centred hierarchy: an axis is halved while its cell count is even
// and at least 4; levels stop at <= 256 cells (or when no axis halves).
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
// Kernels of one application (the fine-level residual of the pre-smoothed
// problem comes from the CG update kernel, see k_mg_axpy): restrict level
// 0 -> 1 (block 0 also decides whether the solve has finished), restrict
// down to the first small level, one single-workgroup kernel for all small
// levels, prolongate + smooth back up, and the fine-level prolongation +
// smoothing that writes z and the partials of r.z.
#include <cmath>
#include <cstdlib>
#include <vector>

#include "pressure_common.h"

namespace uf {

constexpr int kMgMaxLevels = 16;
constexpr int kTailThreads = 1024;
constexpr int kMgFineBlock = 512;        // must match the CG kernels' block (cg_launch)
constexpr long long kTailCells = 1024;   // levels this small run in the single-workgroup kernel
constexpr int kDenseMax = 512;           // largest coarsest level with an exact inverse
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
// level get weight 0 and a clamped index), or f = I alone.  Fixed tap
// positions keep the arrays in registers.
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
  f[2] = 2 * I + 1;
  w[2] = T(0.5) * (T(0.75) + (I == nc - 1 ? T(0.25) * shi : T(0)));
  f[3] = 2 * I + 2 < nf ? 2 * I + 2 : 2 * I + 1;
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
#pragma unroll
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

// CG update with the multigrid's first step fused in: x += alpha d,
// r -= alpha q, partials of ||r||^2, and the residual of the pre-smoothed
// problem (1 - om) r + sum_a w_a om/D r_neighbours from the updated r
// (neighbours' updated r recomputed from r and q).  Marches along x.
template <class T>
__global__ __launch_bounds__(kMgFineBlock) void k_mg_axpy(MgCommon<T> K, MgLvl<T> F, T* __restrict__ X,
                                                          const T* __restrict__ Rin, T* __restrict__ R,
                                                          const T* __restrict__ Dv, const T* __restrict__ Qv,
                                                          T* __restrict__ RES, CgCtl c, int t, int ilen) {
  const Layout& L = F.L;
  double rz = 0.0, dq = 0.0;
  bool run = iteration_runs(c, t, &rz);
  if (run) {
    dq = slot_sum(c.part + (size_t)S_DQ * c.stride, c.nb);
    run = dq > 0.0 && isfinite(dq);
  }
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    c.exec[t] = run;
    if (run) c.st->iter = t + 1;
  }
  if (!run) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = p < L.ny * L.nz;
  const int j = active ? p / L.nz : 0;
  const int k = active ? p - j * L.nz : 0;
  const int i0 = blockIdx.y * ilen;
  const int i1 = active ? min(L.nx, i0 + ilen) : i0;
  const T alpha = (T)(rz / dq);
  double v[1] = {0.0};
  if (i0 < i1) {
    const long long SX = L.SX, PZ = L.PZ;
    // updated residual at any cell, from the untouched input buffer
    auto rn = [&](long long q) { return Rin[q] - alpha * Qv[q]; };
    long long o = L.at(i0, j, k);
    T rm = rn(o - SX), rc = rn(o);
    for (int i = i0; i < i1; ++i, o += SX) {
      const T rp = rn(o + SX);
      X[o] += alpha * Dv[o];
      R[o] = rc;
      v[0] += (double)rc * (double)rc;
      T s;
      if (deep_inside(L, i, j, k)) {
        s = F.omd_in * (F.w[0] * (rp + rm) + F.w[1] * (rn(o + PZ) + rn(o - PZ)) + F.w[2] * (rn(o + 1) + rn(o - 1)));
      } else {
        // zero ghosts of r and q make out-of-range neighbours vanish; omd is 0 there
        s = F.w[0] * (omd(K, F, i + 1, j, k) * rp + omd(K, F, i - 1, j, k) * rm) +
            F.w[1] * (omd(K, F, i, j + 1, k) * rn(o + PZ) + omd(K, F, i, j - 1, k) * rn(o - PZ)) +
            F.w[2] * (omd(K, F, i, j, k + 1) * rn(o + 1) + omd(K, F, i, j, k - 1) * rn(o - 1));
      }
      RES[o] = (T(1) - K.om) * rc + s;
      rm = rc;
      rc = rp;
    }
  }
  const int slots[1] = {S_RR};
  write_partials<1>(v, c.part, c.stride, slots);
}

// Tiles of the level kernels.  Restriction: a block owns RT_I x RT_J x RT_K
// next-level cells (one per thread); up/smoothing: a block owns
// UT_I x UT_J x UT_K cells of its level.
template <class T>
struct MgTiles {
  static constexpr int RT_I = 4, RT_J = 4, RT_K = sizeof(T) == 4 ? 16 : 8;
  static constexpr int RES_N = (2 * RT_I + 2) * (2 * RT_J + 2) * (2 * RT_K + 2);  // fine residual region
  static constexpr int R_N = (2 * RT_I + 4) * (2 * RT_J + 4) * (2 * RT_K + 4);    // r region (+1 halo)
  static constexpr int UT_I = 8, UT_J = 8, UT_K = 32;
  static constexpr int T_N = (UT_I + 2) * (UT_J + 2) * (UT_K + 2);
};

__device__ __forceinline__ bool inside(const Layout& L, int i, int j, int k) {
  return (unsigned)i < (unsigned)L.nx && (unsigned)j < (unsigned)L.ny && (unsigned)k < (unsigned)L.nz;
}

// Restriction of one tile of next-level cells.  The fine residual of the
// pre-smoothed problem over the tile's footprint comes either from a stored
// array (HAS_RES: level 0, written by the CG update) or is computed here from
// r staged in LDS.  mode 0: skip when flags[m] is set; 1: block 0 decides
// whether the solve has finished and publishes flags[m] (first kernel of a
// preconditioner application; after convergence the work here is wasted,
// not wrong); 2: unconditional.
template <bool HAS_RES, class T>
__global__ __launch_bounds__(256) void k_mg_restrict(MgCommon<T> K, MgLvl<T> F, MgLvl<T> C, int has_coarse, CgCtl c,
                                                     int m, int mode) {
  using Tl = MgTiles<T>;
  __shared__ T sres[Tl::RES_N];
  __shared__ T sr[HAS_RES ? 1 : Tl::R_N];
  if (mode == 1) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0) {
      const bool skip = precond_skip(c, m);
      if (threadIdx.x == 0) c.flags[m] = skip;
    }
  } else if (mode == 0) {
    if (c.flags[m]) return;
  }
  if (!has_coarse) return;
  const int X0[3] = {(int)blockIdx.z * Tl::RT_I, (int)blockIdx.y * Tl::RT_J, (int)blockIdx.x * Tl::RT_K};
  const int TT[3] = {Tl::RT_I, Tl::RT_J, Tl::RT_K};
  int lo[3], len[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = F.c[a] ? 2 * X0[a] - 1 : X0[a];
    len[a] = F.c[a] ? 2 * TT[a] + 2 : TT[a];
  }
  const Layout& L = F.L;
  const int nres = len[0] * len[1] * len[2];
  if (HAS_RES) {
    for (int idx = threadIdx.x; idx < nres; idx += blockDim.x) {
      const int kk = idx % len[2], jj = (idx / len[2]) % len[1], ii = idx / (len[2] * len[1]);
      const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
      sres[idx] = inside(L, i, j, k) ? F.t[L.at(i, j, k)] : T(0);
    }
  } else {
    const int q1 = len[1] + 2, q2 = len[2] + 2;
    const int nq = (len[0] + 2) * q1 * q2;
    for (int idx = threadIdx.x; idx < nq; idx += blockDim.x) {
      const int kk = idx % q2, jj = (idx / q2) % q1, ii = idx / (q2 * q1);
      const int i = lo[0] - 1 + ii, j = lo[1] - 1 + jj, k = lo[2] - 1 + kk;
      sr[idx] = inside(L, i, j, k) ? F.r[L.at(i, j, k)] : T(0);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nres; idx += blockDim.x) {
      const int kk = idx % len[2], jj = (idx / len[2]) % len[1], ii = idx / (len[2] * len[1]);
      const int i = lo[0] + ii, j = lo[1] + jj, k = lo[2] + kk;
      T res = T(0);
      if (inside(L, i, j, k)) {
        const int q = ((ii + 1) * q1 + (jj + 1)) * q2 + (kk + 1);
        const int sI = q1 * q2;
        if (deep_inside(L, i, j, k)) {
          res = (T(1) - K.om) * sr[q] + F.omd_in * (F.w[0] * (sr[q + sI] + sr[q - sI]) + F.w[1] * (sr[q + q2] + sr[q - q2]) +
                                                    F.w[2] * (sr[q + 1] + sr[q - 1]));
        } else {
          res = (T(1) - K.om) * sr[q] +
                F.w[0] * (omd(K, F, i + 1, j, k) * sr[q + sI] + omd(K, F, i - 1, j, k) * sr[q - sI]) +
                F.w[1] * (omd(K, F, i, j + 1, k) * sr[q + q2] + omd(K, F, i, j - 1, k) * sr[q - q2]) +
                F.w[2] * (omd(K, F, i, j, k + 1) * sr[q + 1] + omd(K, F, i, j, k - 1) * sr[q - 1]);
        }
      }
      sres[idx] = res;
    }
  }
  __syncthreads();
  const int tk = threadIdx.x % Tl::RT_K, tj = (threadIdx.x / Tl::RT_K) % Tl::RT_J, ti = threadIdx.x / (Tl::RT_K * Tl::RT_J);
  if (ti >= Tl::RT_I) return;
  const int I = X0[0] + ti, J = X0[1] + tj, Kc = X0[2] + tk;
  if (!inside(C.L, I, J, Kc)) return;
  C.r[C.L.at(I, J, Kc)] = restrict_at(K, F, C, I, J, Kc, [&](int i, int j, int k) {
    return sres[((i - lo[0]) * len[1] + (j - lo[1])) * len[2] + (k - lo[2])];
  });
}

// Prolongation + post-smoothing of one tile of level F: t = om D^-1 r + P x_c
// over the tile and a one-cell halo (LDS), then x = t + om D^-1 (r - A t).
// FINE: level 0, also writes the partials of r.z for the CG.
template <bool FINE, bool COARSE, class T>
__global__ __launch_bounds__(256) void k_mg_upsmooth(MgCommon<T> K, MgLvl<T> F, MgLvl<T> C, CgCtl c, int m) {
  using Tl = MgTiles<T>;
  __shared__ T st[Tl::T_N];
  if (c.flags[m]) return;
  const Layout& L = F.L;
  const int i0 = blockIdx.z * Tl::UT_I, j0 = blockIdx.y * Tl::UT_J, k0 = blockIdx.x * Tl::UT_K;
  constexpr int HI = Tl::UT_I + 2, HJ = Tl::UT_J + 2, HK = Tl::UT_K + 2;
  for (int idx = threadIdx.x; idx < HI * HJ * HK; idx += blockDim.x) {
    const int kk = idx % HK, jj = (idx / HK) % HJ, ii = idx / (HK * HJ);
    st[idx] = pre_plus_coarse<COARSE>(K, F, C, i0 - 1 + ii, j0 - 1 + jj, k0 - 1 + kk);
  }
  __syncthreads();
  double v[1] = {0.0};
  for (int idx = threadIdx.x; idx < Tl::UT_I * Tl::UT_J * Tl::UT_K; idx += blockDim.x) {
    const int kk = idx % Tl::UT_K, jj = (idx / Tl::UT_K) % Tl::UT_J, ii = idx / (Tl::UT_K * Tl::UT_J);
    const int i = i0 + ii, j = j0 + jj, k = k0 + kk;
    if (!inside(L, i, j, k)) continue;
    const int q = ((ii + 1) * HJ + (jj + 1)) * HK + (kk + 1);
    const T tc = st[q];
    const T D = diag_w(K.bc, L, F.w, i, j, k);
    const T At = D * tc - F.w[0] * (st[q + HJ * HK] + st[q - HJ * HK]) - F.w[1] * (st[q + HK] + st[q - HK]) -
                 F.w[2] * (st[q + 1] + st[q - 1]);
    const long long o = L.at(i, j, k);
    const T rr = F.r[o];
    const T z = tc + omd(K, F, i, j, k) * (rr - At);
    F.x[o] = z;
    if (FINE) v[0] += (double)rr * (double)z;
  }
  if (FINE) {
    const int slots[1] = {S_RZ0 + (m & 1)};
    write_partials<1>(v, c.part, c.stride, slots);
  }
}

// All levels from lt down to the coarsest and back, in one workgroup, as
// phases separated by barriers over arrays that stay in the L2.  The level
// descriptors are read from a device table.
template <class T>
__global__ __launch_bounds__(kTailThreads) void k_mg_tail(MgCommon<T> K, const MgLvl<T>* __restrict__ lv, int lt,
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
    if (g.mg[l].r) (void)hipFree(g.mg[l].r);
    if (g.mg[l].x) (void)hipFree(g.mg[l].x);
    if (g.mg[l].t) (void)hipFree(g.mg[l].t);
  }
  g.mg.clear();
  if (g.mg_cinv) (void)hipFree(g.mg_cinv);
  g.mg_cinv = nullptr;
  if (g.mg_table) (void)hipFree(g.mg_table);
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
    if (ncells(F.L) <= 256) break;
    int c[3], any = 0;
    for (int a = 0; a < 3; ++a) {
      c[a] = (n[a] % 2 == 0 && n[a] >= 4) ? 1 : 0;
      any |= c[a];
    }
    if (!any) break;
    MgLevel C;
    C.L = level_layout(n[0] >> c[0], n[1] >> c[1], n[2] >> c[2]);
    for (int a = 0; a < 3; ++a) {
      F.coarsen[a] = c[a];
      C.w[a] = F.w[a] / (c[a] ? 4.0 : 1.0);   // re-discretised with the doubled spacing
    }
    const size_t bytes = (size_t)(C.L.nx + 3) * C.L.SX * es;
    for (void** q : {&C.r, &C.x, &C.t}) {
      if (hipMalloc(q, bytes) != hipSuccess) throw HipError("hipMalloc failed (multigrid level)");
      UF_HIP_CHECK(hipMemset(*q, 0, bytes));
    }
    g.mg.push_back(C);
  }
  MgLevel& last = g.mg.back();
  for (int a = 0; a < 3; ++a) last.coarsen[a] = 0;
  const int nl = (int)g.mg.size();
  // first small level (>= 1) for the single-workgroup kernel
  g.mg_lt = nl;
  for (int l = 1; l < nl; ++l)
    if (ncells(g.mg[l].L) <= kTailCells) {
      g.mg_lt = l;
      break;
    }
  // the coarsest level is always solved by the single-workgroup kernel
  if (nl > 1 && g.mg_lt > nl - 1) g.mg_lt = nl - 1;
  g.mg_cinv = nullptr;
  g.mg_nc = (int)ncells(last.L);
  g.mg_omega = kJacobiOmega;
  {
    std::vector<MgLvl<T>> tab(nl);
    for (int l = 0; l < nl; ++l) tab[l] = mg_level<T>(g, l);
    UF_HIP_CHECK(hipMalloc(&g.mg_table, tab.size() * sizeof(MgLvl<T>)));
    UF_HIP_CHECK(hipMemcpy(g.mg_table, tab.data(), tab.size() * sizeof(MgLvl<T>), hipMemcpyHostToDevice));
  }
  if (nl > 1) {
    std::vector<double> inv;
    if (dense_inverse(last, g.bc, inv)) {
      std::vector<T> tv(inv.begin(), inv.end());
      UF_HIP_CHECK(hipMalloc(&g.mg_cinv, tv.size() * es));
      UF_HIP_CHECK(hipMemcpy(g.mg_cinv, tv.data(), tv.size() * es, hipMemcpyHostToDevice));
    }
  }
}

size_t mg_fine_blocks(const Layout& L) {
  using Tl = MgTiles<float>;   // the up/smoothing tile does not depend on the dtype
  return (size_t)((L.nz + Tl::UT_K - 1) / Tl::UT_K) * ((L.ny + Tl::UT_J - 1) / Tl::UT_J) *
         ((L.nx + Tl::UT_I - 1) / Tl::UT_I);
}

template <class T>
static dim3 restrict_grid(const Layout& C) {
  using Tl = MgTiles<T>;
  return dim3((C.nz + Tl::RT_K - 1) / Tl::RT_K, (C.ny + Tl::RT_J - 1) / Tl::RT_J, (C.nx + Tl::RT_I - 1) / Tl::RT_I);
}

template <class T>
static dim3 up_grid(const Layout& F) {
  using Tl = MgTiles<T>;
  return dim3((F.nz + Tl::UT_K - 1) / Tl::UT_K, (F.ny + Tl::UT_J - 1) / Tl::UT_J, (F.nx + Tl::UT_I - 1) / Tl::UT_I);
}

template <class T>
void mg_launch(Grid& g, const Params<T>& P, int m, const void* r, void* z, int decide) {
  (void)P;
  const MgCommon<T> K = mg_common<T>(g);
  const CgCtl c = make_ctl(g);
  const int nl = (int)g.mg.size();
  MgLvl<T> L0 = mg_level<T>(g, 0);
  L0.r = (T*)r;
  L0.x = (T*)z;
  L0.t = (T*)z;   // the fine residual from the CG update lives in z until z is written
  const MgLvl<T> L1 = nl > 1 ? mg_level<T>(g, 1) : L0;
  // level 0 -> 1: the stored residual exists only after a CG update
  const bool stored = decide && m > 0;
  const int mode0 = decide ? 1 : 2;
  {
    TimedLaunch tl(g, UF_TK_MG_DOWN0);
    const dim3 grid = nl > 1 ? restrict_grid<T>(L1.L) : dim3(1);
    if (stored)
      hipLaunchKernelGGL((k_mg_restrict<true, T>), grid, dim3(256), 0, g.stream, K, L0, L1, nl > 1 ? 1 : 0, c, m, mode0);
    else
      hipLaunchKernelGGL((k_mg_restrict<false, T>), grid, dim3(256), 0, g.stream, K, L0, L1, nl > 1 ? 1 : 0, c, m, mode0);
  }
  const int lt = std::min(g.mg_lt, nl - 1);
  for (int l = 1; l < lt; ++l) {
    const MgLvl<T> F = mg_level<T>(g, l), C = mg_level<T>(g, l + 1);
    TimedLaunch tl(g, UF_TK_MG_COARSE);
    hipLaunchKernelGGL((k_mg_restrict<false, T>), restrict_grid<T>(C.L), dim3(256), 0, g.stream, K, F, C, 1, c, m, 0);
  }
  if (nl > 1) {
    {
      TimedLaunch tl(g, UF_TK_MG_COARSE);
      hipLaunchKernelGGL(k_mg_tail<T>, dim3(1), dim3(kTailThreads), 0, g.stream, K, (const MgLvl<T>*)g.mg_table, lt,
                         nl, (const T*)g.mg_cinv, (const int*)c.flags, m);
    }
    for (int l = lt - 1; l >= 1; --l) {
      const MgLvl<T> F = mg_level<T>(g, l), C = mg_level<T>(g, l + 1);
      TimedLaunch tl(g, UF_TK_MG_COARSE);
      hipLaunchKernelGGL((k_mg_upsmooth<false, true, T>), up_grid<T>(F.L), dim3(256), 0, g.stream, K, F, C, c, m);
    }
  }
  TimedLaunch tl(g, UF_TK_MG_UP0);
  if (nl > 1)
    hipLaunchKernelGGL((k_mg_upsmooth<true, true, T>), up_grid<T>(L0.L), dim3(256), 0, g.stream, K, L0, L1, c, m);
  else
    hipLaunchKernelGGL((k_mg_upsmooth<true, false, T>), up_grid<T>(L0.L), dim3(256), 0, g.stream, K, L0, L1, c, m);
}

template <class T>
void mg_precond(Grid& g, const Params<T>& P, int m) {
  mg_launch<T>(g, P, m, resid(g, m), g.Z, 1);
}

// CG update fused with the fine residual of the next preconditioner
// application (written into Z, which the application overwrites last).
template <class T>
void mg_axpy(Grid& g, const Params<T>& P, int t) {
  (void)P;
  const MgCommon<T> K = mg_common<T>(g);
  MgLvl<T> L0 = mg_level<T>(g, 0);
  const CgLaunch cl = cg_launch(g.L);
  TimedLaunch tl(g, UF_TK_CG_AXPY);
  hipLaunchKernelGGL(k_mg_axpy<T>, cl.grid, dim3(kMgFineBlock), 0, g.stream, K, L0, (T*)g.X,
                     (const T*)resid(g, t), (T*)resid(g, t + 1), (const T*)g.D[(t + 1) & 1], (const T*)g.Qv,
                     (T*)g.Z, make_ctl(g), t, cl.ilen);
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
template void mg_apply<float>(Grid&, const Params<float>&, const void*, void*);
template void mg_apply<double>(Grid&, const Params<double>&, const void*, void*);
template void mg_axpy<float>(Grid&, const Params<float>&, int);
template void mg_axpy<double>(Grid&, const Params<double>&, int);

}  // namespace uf
