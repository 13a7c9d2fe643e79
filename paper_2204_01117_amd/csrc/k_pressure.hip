// Pressure projection solve (Sec. 3): A p = b with A = -L_h, the 7-point
// negative Laplacian on cell centres (Neumann rows at inlet/wall/slip sides,
// zero ghost pressure at outlets), b = -(rho/dt) div u*.  A never changes
// because obstacles act through the porosity drag, so it is applied
// matrix-free and every CG vector keeps zero ghosts.
//
// Preconditioned CG (Saad, Alg. 9.1) with vectors in the grid's dtype and
// every dot product and norm accumulated in FP64.  Each reducing kernel
// writes one FP64 partial per block; the next kernel in stream order adds
// the partials in block order inside every block, so alpha, beta and the
// stopping test are identical in all blocks, deterministic, and never need
// a device-wide fence.  flags[m] records that the solve has finished before
// iteration m, so iterations enqueued past convergence return at once.
#include "pressure_common.h"

namespace uf {

constexpr int kCgBlock = 512;

#define UF_CG_RANGE(L, ilen)                                                 \
  const int cg_gx = ((L).ny * (L).nz + kCgBlock - 1) / kCgBlock;             \
  int cg_bx, cg_by;                                                          \
  if (!xcd_block(cg_gx, ((L).nx + (ilen) - 1) / (ilen), cg_bx, cg_by)) return; \
  const int cg_bid = cg_by * cg_gx + cg_bx;                                  \
  const int p = cg_bx * kCgBlock + threadIdx.x;                              \
  const bool active = p < (L).ny * (L).nz;                                   \
  const int j = active ? p / (L).nz : 0;                                     \
  const int k = active ? p - j * (L).nz : 0;                                 \
  const int i0 = cg_by * (ilen);                                             \
  const int i1 = active ? min((L).nx, i0 + (ilen)) : i0;

// First-order approximate inverse (Sec. 3): M^-1 = K^T K with
// K = sqrt(2-w) Dbar^-1/2 (I - L Dbar^-1), Dbar = D/w.  Written out,
//   u_c = (w/D_c) (r_c + sum_{lower n} (w/D_n) r_n / h_n^2)
//   z_c = (2-w) (u_c + (w/D_c) sum_{upper m} u_m / h_m^2)
// where lower/upper are the -x,-y,-z / +x,+y,+z neighbours inside the grid
// (z-fastest lexicographic order).
template <class T>
__device__ __forceinline__ T ai1_u(const Params<T>& P, const T* __restrict__ r, int i, int j, int k, T om) {
  const Layout& L = P.L;
  const long long o = L.at(i, j, k);
  T s = r[o];
  if (i > 0) s += om / poisson_diag(P, i - 1, j, k) * r[o - L.SX] * P.ih2[0];
  if (j > 0) s += om / poisson_diag(P, i, j - 1, k) * r[o - L.PZ] * P.ih2[1];
  if (k > 0) s += om / poisson_diag(P, i, j, k - 1) * r[o - 1] * P.ih2[2];
  return om / poisson_diag(P, i, j, k) * s;
}

template <class T>
__device__ __forceinline__ T precond_apply(const Params<T>& P, int pc, T om, const T* __restrict__ r, int i, int j,
                                           int k, long long o) {
  if (pc == UF_PC_JACOBI) return r[o] / poisson_diag(P, i, j, k);
  if (pc == UF_PC_AI1) {
    const Layout& L = P.L;
    T up = T(0);
    if (i + 1 < L.nx) up += ai1_u(P, r, i + 1, j, k, om) * P.ih2[0];
    if (j + 1 < L.ny) up += ai1_u(P, r, i, j + 1, k, om) * P.ih2[1];
    if (k + 1 < L.nz) up += ai1_u(P, r, i, j, k + 1, om) * P.ih2[2];
    return (T(2) - om) * (ai1_u(P, r, i, j, k, om) + om / poisson_diag(P, i, j, k) * up);
  }
  return r[o];
}

// Second-order approximate inverse (Sec. 3): M^-1 = K^T K with
// K = sqrt(2-w) Dbar^-1/2 (I - L Dbar^-1 + (L Dbar^-1)^2), applied in two
// passes through a scratch vector v:
//   v_c = (w/D_c) (r_c + sum_{lower n} (w/D_n) (r_n + sum_{lower m of n} (w/D_m) r_m / h_m^2) / h_n^2)
//   z_c = (2-w) (v_c + (w/D_c) sum_{upper m} (v_m + (w/D_m) sum_{upper p of m} v_p / h_p^2) / h_m^2)
// (the off-diagonal entries of A are -1/h^2; every hop stays inside the grid).
template <class T>
__device__ __forceinline__ T ai2_lower(const Params<T>& P, const T* __restrict__ r, int i, int j, int k, T om) {
  // r_n + sum over the in-grid lower neighbours m of n of (w/D_m) r_m / h^2
  const Layout& L = P.L;
  const long long o = L.at(i, j, k);
  T s = r[o];
  if (i > 0) s += om / poisson_diag(P, i - 1, j, k) * r[o - L.SX] * P.ih2[0];
  if (j > 0) s += om / poisson_diag(P, i, j - 1, k) * r[o - L.PZ] * P.ih2[1];
  if (k > 0) s += om / poisson_diag(P, i, j, k - 1) * r[o - 1] * P.ih2[2];
  return s;
}

template <class T>
__device__ __forceinline__ T ai2_v(const Params<T>& P, const T* __restrict__ r, int i, int j, int k, T om) {
  T s = r[P.L.at(i, j, k)];
  if (i > 0) s += om / poisson_diag(P, i - 1, j, k) * ai2_lower(P, r, i - 1, j, k, om) * P.ih2[0];
  if (j > 0) s += om / poisson_diag(P, i, j - 1, k) * ai2_lower(P, r, i, j - 1, k, om) * P.ih2[1];
  if (k > 0) s += om / poisson_diag(P, i, j, k - 1) * ai2_lower(P, r, i, j, k - 1, om) * P.ih2[2];
  return om / poisson_diag(P, i, j, k) * s;
}

template <class T>
__device__ __forceinline__ T ai2_upper(const Params<T>& P, const T* __restrict__ v, int i, int j, int k, T om) {
  // v_m + (w/D_m) sum over the in-grid upper neighbours p of m of v_p / h^2
  const Layout& L = P.L;
  const long long o = L.at(i, j, k);
  T s = T(0);
  if (i + 1 < L.nx) s += v[o + L.SX] * P.ih2[0];
  if (j + 1 < L.ny) s += v[o + L.PZ] * P.ih2[1];
  if (k + 1 < L.nz) s += v[o + 1] * P.ih2[2];
  return v[o] + om / poisson_diag(P, i, j, k) * s;
}

template <class T>
__device__ __forceinline__ T ai2_z(const Params<T>& P, const T* __restrict__ v, int i, int j, int k, T om) {
  const Layout& L = P.L;
  T s = T(0);
  if (i + 1 < L.nx) s += ai2_upper(P, v, i + 1, j, k, om) * P.ih2[0];
  if (j + 1 < L.ny) s += ai2_upper(P, v, i, j + 1, k, om) * P.ih2[1];
  if (k + 1 < L.nz) s += ai2_upper(P, v, i, j, k + 1, om) * P.ih2[2];
  return (T(2) - om) * (v[L.at(i, j, k)] + om / poisson_diag(P, i, j, k) * s);
}

// Diagonal of A split as the part from the y and z axes (fixed along a
// thread's x-march) and the x part at cell i.
template <class T>
__device__ __forceinline__ T diag_yz(const Params<T>& P, int j, int k) {
  const Layout& L = P.L;
  return ((j > 0 || P.bc[2] == OUTLET) ? P.ih2[1] : T(0)) + ((j < L.ny - 1 || P.bc[3] == OUTLET) ? P.ih2[1] : T(0)) +
         ((k > 0 || P.bc[4] == OUTLET) ? P.ih2[2] : T(0)) + ((k < L.nz - 1 || P.bc[5] == OUTLET) ? P.ih2[2] : T(0));
}

template <class T>
__device__ __forceinline__ T diag_x(const Params<T>& P, int i) {
  return ((i > 0 || P.bc[0] == OUTLET) ? P.ih2[0] : T(0)) + ((i < P.L.nx - 1 || P.bc[1] == OUTLET) ? P.ih2[0] : T(0));
}

// r = b - A x with b = -(rho/dt) div u* (or a given b); partials of ||b||^2
// and ||r||^2.
template <class T>
__global__ __launch_bounds__(kCgBlock) void k_cg_init(Params<T> P, const T* __restrict__ U, const T* __restrict__ V,
                                                      const T* __restrict__ W, const T* __restrict__ bin,
                                                      const T* __restrict__ X, T* __restrict__ R, CgCtl c, int ilen) {
  const Layout& L = P.L;
  UF_CG_RANGE(L, ilen);
  double v[2] = {0.0, 0.0};
  if (i0 < i1) {
    const T dyz = diag_yz(P, j, k);
    long long o = L.at(i0, j, k);
    T xm = X[o - L.SX], xc = X[o];
    for (int i = i0; i < i1; ++i, o += L.SX) {
      const T xp = X[o + L.SX];
      T b;
      if (bin) {
        b = bin[o];
      } else {
        const T div = (U[o + L.SX] - U[o]) * P.ih[0] + (V[o + L.PZ] - V[o]) * P.ih[1] + (W[o + 1] - W[o]) * P.ih[2];
        b = -P.rho_dt * div;
      }
      const T ax = (dyz + diag_x(P, i)) * xc - (xp + xm) * P.ih2[0] - (X[o + L.PZ] + X[o - L.PZ]) * P.ih2[1] -
                   (X[o + 1] + X[o - 1]) * P.ih2[2];
      const T r = b - ax;
      R[o] = r;
      v[0] += (double)b * (double)b;
      v[1] += (double)r * (double)r;
      xm = xc;
      xc = xp;
    }
  }
  const int slots[2] = {S_BB, S_RR};
  write_partials<2>(v, c.part, c.stride, slots, cg_bid);
  pad_partials(c, S_RR, cg_bid, c.nb);
}

// One block: ||b||, the stopping threshold and whether x0 already solves.
// An initial guess whose residual is larger than b itself (the warm start
// of a step after a sudden change of the flow) is dropped for x0 = 0: the
// iterate is then accumulated from zero, so its rounding is relative to
// the new solution rather than to the larger old one; k_cg_restart resets
// x and r.
__global__ __launch_bounds__(256) void k_cg_start(CgCtl c, double tol) {
  const double bb = slot_sum(c.part + (size_t)S_BB * c.stride, c.nb);
  double rr = slot_sum(c.part + (size_t)S_RR * c.stride, c.nb_rr);
  if (threadIdx.x != 0) return;
  CgState* st = c.st;
  const bool restart = isfinite(bb) && isfinite(rr) && rr > bb;
  if (restart) rr = bb;
  st->restart = restart;
  st->bb = bb;
  st->rr = rr;
  st->iter = 0;
  st->noconv = 0;
  st->maxit = c.maxit;
  st->criterion = c.criterion;
  st->nonfinite = !(isfinite(bb) && isfinite(rr));
  st->zero_rhs = (bb == 0.0);
  st->tol2_bb = c.criterion == 0 ? tol * tol * bb : tol * bb;
  st->done = st->nonfinite || st->zero_rhs || (c.criterion == 0 && rr <= st->tol2_bb);
  c.flags[0] = st->done;
}

// x = 0 and r = b when k_cg_start dropped the initial guess (b formed as
// k_cg_init forms it); nothing otherwise.
template <class T>
__global__ __launch_bounds__(kCgBlock) void k_cg_restart(Params<T> P, const T* __restrict__ U,
                                                         const T* __restrict__ V, const T* __restrict__ W,
                                                         const T* __restrict__ bin, T* __restrict__ X,
                                                         T* __restrict__ R, CgCtl c, int ilen) {
  if (!c.st->restart) return;
  const Layout& L = P.L;
  UF_CG_RANGE(L, ilen);
  for (int i = i0; i < i1; ++i) {
    const long long o = L.at(i, j, k);
    T b;
    if (bin) {
      b = bin[o];
    } else {
      const T div = (U[o + L.SX] - U[o]) * P.ih[0] + (V[o + L.PZ] - V[o]) * P.ih[1] + (W[o + 1] - W[o]) * P.ih[2];
      b = -P.rho_dt * div;
    }
    R[o] = b;
    X[o] = T(0);
  }
}

// Preconditioner application m (m = 0 after init, m = t+1 after iteration
// t): z = M^-1 r and the partials of r.z.
template <class T>
__global__ __launch_bounds__(kCgBlock) void k_cg_precond(Params<T> P, const T* __restrict__ R, T* __restrict__ Z,
                                                         CgCtl c, int m, int pc, T om, int ilen) {
  const Layout& L = P.L;
  const bool skip = precond_skip(c, m);
  if (blockIdx.x == 0 && threadIdx.x == 0) c.flags[m] = skip;
  if (skip) return;
  UF_CG_RANGE(L, ilen);
  double v[1] = {0.0};
  for (int i = i0; i < i1; ++i) {
    const long long o = L.at(i, j, k);
    const T z = precond_apply(P, pc, om, R, i, j, k, o);
    Z[o] = z;
    v[0] += (double)R[o] * (double)z;
  }
  const int slots[1] = {S_RZ0 + (m & 1)};
  write_partials<1>(v, c.part, c.stride, slots, cg_bid);
}

// First pass of the second-order approximate inverse: v from r (all cells).
template <class T>
__global__ __launch_bounds__(kCgBlock) void k_ai2_v(Params<T> P, const T* __restrict__ R, T* __restrict__ V, T om,
                                                   int ilen) {
  const Layout& L = P.L;
  UF_CG_RANGE(L, ilen);
  for (int i = i0; i < i1; ++i) V[L.at(i, j, k)] = ai2_v(P, R, i, j, k, om);
}

// Second pass: z from v.  In a solve (cg != 0) it is preconditioner
// application m: it decides whether the solve has finished (as
// k_cg_precond) and writes the partials of r.z.
template <class T>
__global__ __launch_bounds__(kCgBlock) void k_ai2_z(Params<T> P, const T* __restrict__ R, const T* __restrict__ V,
                                                   T* __restrict__ Z, CgCtl c, int m, T om, int ilen, int cg) {
  const Layout& L = P.L;
  if (cg) {
    const bool skip = precond_skip(c, m);
    if (blockIdx.x == 0 && threadIdx.x == 0) c.flags[m] = skip;
    if (skip) return;
  }
  UF_CG_RANGE(L, ilen);
  double v[1] = {0.0};
  for (int i = i0; i < i1; ++i) {
    const long long o = L.at(i, j, k);
    const T z = ai2_z(P, V, i, j, k, om);
    Z[o] = z;
    v[0] += (double)R[o] * (double)z;
  }
  if (cg) {
    const int slots[1] = {S_RZ0 + (m & 1)};
    write_partials<1>(v, c.part, c.stride, slots, cg_bid);
  }
}

// d = z + beta d_old; q = A d; partials of d.q.
//
// A block owns a JT x KT tile of (j, k) columns (KT = z extent of the tile,
// JT = 512 / KT) and marches its x-range in passes of four planes.  Each
// thread loads z and d_old of its own column and, at the tile's edge, of the
// halo cell beside it; d of the pass's four planes is staged in LDS, so the
// y and z neighbours come from LDS (about 2.5 global loads per cell instead
// of 10) and the x neighbours stay in registers.  The next pass's loads are
// issued before the current pass is computed, and the first pass's before
// the flags and beta are known.
template <int KT, class T>
__global__ __launch_bounds__(512) void k_cg_Ad(Params<T> P, const T* __restrict__ Z, const T* __restrict__ Dold,
                                              T* __restrict__ Dnew, T* __restrict__ Qv, T* __restrict__ X, CgCtl c,
                                              int t, int ilen, int njt, int nkt) {
  constexpr int JT = 512 / KT, PW = KT + 2, PN = (JT + 2) * PW;
  __shared__ T sd[4 * PN];
  const Layout& L = P.L;
  const int ntile = njt * nkt;
  int bx, by;
  if (!xcd_block(ntile, (L.nx + ilen - 1) / ilen, bx, by)) return;
  const int bid = by * ntile + bx;
  const int jtile = bx / nkt, ktile = bx - jtile * nkt;
  const int tk = threadIdx.x % KT, tj = threadIdx.x / KT;
  const int j = jtile * JT + tj, k = ktile * KT + tk;
  const bool act = j < L.ny && k < L.nz;
  const int i0 = by * ilen, i1 = min(L.nx, i0 + ilen);
  const bool first = t == 0;
  const int sx = (int)L.SX, pz = (int)L.PZ;   // a plane of the padded layout is far below 2^31 elements
  // halo roles at the tile's edge: the neighbouring row (y) and column (z)
  const int rrole = tj == 0 ? -1 : (tj == JT - 1 ? 1 : 0);
  const int crole = tk == 0 ? -1 : (tk == KT - 1 ? 1 : 0);
  const T* __restrict__ zc = Z + (act ? L.at(0, j, k) : 0);
  const T* __restrict__ dc0 = Dold + (act ? L.at(0, j, k) : 0);
  // raw values of a pass starting at plane p0: own planes p0-1 .. p0+4 and
  // the halo cells of planes p0 .. p0+3
  T zo[6], dz[6], zr[4], dr[4], zcol[4], dcol[4];
  auto load_pass = [&](int p0, bool with_prev) {
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int pl = p0 - 1 + u;
      const bool ok = act && (u >= 2 || with_prev) && pl <= i1;
      zo[u] = ok ? zc[pl * sx] : T(0);
      dz[u] = ok && !first ? dc0[pl * sx] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int pl = p0 + u;
      const bool ok = act && pl < i1;
      zr[u] = ok && rrole ? zc[pl * sx + rrole * pz] : T(0);
      dr[u] = ok && rrole && !first ? dc0[pl * sx + rrole * pz] : T(0);
      zcol[u] = ok && crole ? zc[pl * sx + crole] : T(0);
      dcol[u] = ok && crole && !first ? dc0[pl * sx + crole] : T(0);
    }
  };
  load_pass(i0, true);
  if (first && c.flags[0] && c.st->zero_rhs) {
    // b = 0: the solution is x = 0
    if (act)
      for (int i = i0; i < i1; ++i) X[L.at(i, j, k)] = T(0);
    return;
  }
  if (!iteration_open(c, t)) return;
  const double rz = rz_of(c, t);
  if (blockIdx.x == 0 && threadIdx.x == 0) c.st->rzh[t & 1] = rz;
  if (!rz_allows(c, rz)) return;
  // r.z of iteration t - 1 was published by this kernel's previous launch
  const T beta = first ? T(0) : (T)(rz / c.st->rzh[(t + 1) & 1]);
  auto dv = [&](T z, T d) { return first ? z : z + beta * d; };
  const T dyz = act ? diag_yz(P, j, k) : T(0);
  const int own = (tj + 1) * PW + tk + 1;
  double acc[1] = {0.0};
  T dm = dv(zo[0], dz[0]), dcur = dv(zo[1], dz[1]);
  for (int p0 = i0; p0 < i1; p0 += 4) {
    T d[6];
    d[0] = dm;
    d[1] = dcur;
#pragma unroll
    for (int u = 2; u < 6; ++u) d[u] = dv(zo[u], dz[u]);
    __syncthreads();   // the previous pass is done with the LDS
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      T* s = sd + u * PN;
      s[own] = d[u + 1];
      if (rrole) s[own + rrole * PW] = dv(zr[u], dr[u]);
      if (crole) s[own + crole] = dv(zcol[u], dcol[u]);
    }
    if (p0 + 4 < i1) load_pass(p0 + 4, false);
    __syncthreads();
    if (act) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = p0 + u;
        if (i >= i1) break;
        const T* s = sd + u * PN;
        const T q = (dyz + diag_x(P, i)) * d[u + 1] - (d[u] + d[u + 2]) * P.ih2[0] -
                    (s[own - PW] + s[own + PW]) * P.ih2[1] - (s[own - 1] + s[own + 1]) * P.ih2[2];
        const long long o = L.at(i, j, k);
        Dnew[o] = d[u + 1];
        Qv[o] = q;
        acc[0] += (double)d[u + 1] * (double)q;
      }
    }
    dm = d[4];
    dcur = d[5];
  }
  const int slots[1] = {S_DQ};
  write_partials<1>(acc, c.part, c.stride, slots, bid);
}

// x += alpha d; r -= alpha q; partials of ||r||^2.  The first four
// x-planes of the thread's column are loaded before the scalars are known.
template <class T>
__global__ __launch_bounds__(kCgBlock) void k_cg_axpy(Params<T> P, T* __restrict__ X, const T* __restrict__ Rin,
                                                      T* __restrict__ R, const T* __restrict__ D,
                                                      const T* __restrict__ Qv, CgCtl c, int t, int ilen) {
  const Layout& L = P.L;
  UF_CG_RANGE(L, ilen);
  const bool pass0 = i0 + 4 <= i1;
  const long long SX = L.SX;
  const long long o0 = pass0 ? L.at(i0, j, k) : 0;
  T x4[4], r4[4], d4[4], q4[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    x4[u] = r4[u] = d4[u] = q4[u] = T(0);
    if (pass0) {
      const long long o = o0 + u * SX;
      x4[u] = X[o];
      r4[u] = Rin[o];
      d4[u] = D[o];
      q4[u] = Qv[o];
    }
  }
  double rz = 0.0, dq = 0.0;
  bool run = iteration_open(c, t);
  if (run) {
    rz = c.st->rzh[t & 1];
    run = rz_allows(c, rz);
  }
  if (run) {
    dq = slot_sum(c.part + (size_t)S_DQ * c.stride, c.nb_dq);
    run = dq > 0.0 && isfinite(dq);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c.exec[t] = run;
    if (run) c.st->iter = t + 1;
  }
  if (!run) return;
  const T alpha = (T)(rz / dq);
  double v[1] = {0.0};
  int i = i0;
  if (pass0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long o = o0 + u * SX;
      X[o] = x4[u] + alpha * d4[u];
      const T r = r4[u] - alpha * q4[u];
      R[o] = r;
      v[0] += (double)r * (double)r;
    }
    i += 4;
  }
#pragma unroll 4
  for (; i < i1; ++i) {
    const long long o = L.at(i, j, k);
    X[o] += alpha * D[o];
    const T r = Rin[o] - alpha * Qv[o];
    R[o] = r;
    v[0] += (double)r * (double)r;
  }
  const int slots[1] = {S_RR};
  write_partials<1>(v, c.part, c.stride, slots, cg_bid);
  pad_partials(c, S_RR, cg_bid, c.nb);
}

// One block, after a chunk of iterations ending at t_end: publish the
// status for the host.
__global__ __launch_bounds__(256) void k_cg_status(CgCtl c, int t_end) {
  const double rr = slot_sum(c.part + (size_t)S_RR * c.stride, c.nb_rr);
  CgState* st = c.st;
  const int it = st->iter;
  const double rz = slot_sum(c.part + (size_t)(S_RZ0 + (it & 1)) * c.stride, c.nb_rz);
  if (threadIdx.x != 0) return;
  st->rr = rr;
  st->nonfinite = st->nonfinite || !isfinite(rr);
  const bool conv = st->zero_rhs || (c.criterion == 0 ? rr <= st->tol2_bb : rz < st->tol2_bb);
  st->done = c.flags[t_end] || t_end >= c.maxit || st->nonfinite;
  st->noconv = st->done && !conv && !st->nonfinite;
}

// y = A x or y = M^-1 x on all cells (x with zero ghosts).
template <class T>
__global__ __launch_bounds__(kCgBlock) void k_apply(Params<T> P, int op, int pc, T om, const T* __restrict__ x,
                                                    T* __restrict__ y, int ilen) {
  const Layout& L = P.L;
  UF_CG_RANGE(L, ilen);
  for (int i = i0; i < i1; ++i) {
    const long long o = L.at(i, j, k);
    y[o] = op == UF_OP_POISSON ? apply_w(P.bc, L, P.ih2, x, i, j, k, o) : precond_apply(P, pc, om, x, i, j, k, o);
  }
}

// ------------------------------------------------------------------ launch
CgLaunch cg_launch(const Layout& L) {
  const int bp = (L.ny * L.nz + kCgBlock - 1) / kCgBlock;
  // about 512 blocks of 8 waves (16 waves per CU): enough to stream,
  // few partial sums for the next kernel to add
  int nchunk = (512 + bp - 1) / bp;
  if (nchunk > L.nx) nchunk = L.nx;
  if (nchunk < 1) nchunk = 1;
  const int ilen = (L.nx + nchunk - 1) / nchunk;
  const int gy = (L.nx + ilen - 1) / ilen;
  return CgLaunch{xcd_grid(bp, gy), ilen, bp, gy};
}

AdLaunch ad_launch(const Layout& L) {
  AdLaunch a;
  a.kt = L.nz >= 64 ? 64 : (L.nz > 16 ? 32 : 16);
  a.njt = (L.ny + 512 / a.kt - 1) / (512 / a.kt);
  a.nkt = (L.nz + a.kt - 1) / a.kt;
  const int tiles = a.njt * a.nkt;
  // about 512 blocks, as the other CG kernels
  int nchunk = (512 + tiles - 1) / tiles;
  if (nchunk > L.nx) nchunk = L.nx;
  if (nchunk < 1) nchunk = 1;
  a.ilen = (L.nx + nchunk - 1) / nchunk;
  a.gy = (L.nx + a.ilen - 1) / a.ilen;
  a.blocks = tiles * a.gy;
  a.grid = xcd_grid(tiles, a.gy);
  return a;
}

CgCtl make_ctl(Grid& g) {
  CgCtl c;
  c.part = g.partials;
  c.stride = (int)g.part_stride;
  c.nb = (int)g.cg_nb;
  c.nb_rz = (int)g.cg_nb_rz;
  c.nb_dq = (int)g.cg_nb_dq;
  c.nb_rr = (int)g.cg_nb_rr;
  c.flags = g.flags;
  c.exec = g.exec;
  c.st = g.st;
  c.criterion = g.cfg.cg_criterion;
  c.maxit = g.cfg.cg_maxit;
  return c;
}

template <class T>
void launch_cg_start(Grid& g, const Params<T>& P, void* const Qs[3], const void* b) {
  const CgLaunch cl = cg_launch(P.L);
  const CgCtl c = make_ctl(g);
  {
    TimedLaunch tl(g, UF_TK_CG_INIT);
    launch_k(g, k_cg_init<T>, cl.grid, dim3(kCgBlock), P, (const T*)Qs[0], (const T*)Qs[1],
                     (const T*)Qs[2], (const T*)b, (const T*)g.X, (T*)resid(g, 0), c, cl.ilen);
  }
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(256), 0, g.stream, c, g.cfg.cg_tol);
  hipLaunchKernelGGL(k_cg_restart<T>, cl.grid, dim3(kCgBlock), 0, g.stream, P, (const T*)Qs[0], (const T*)Qs[1],
                     (const T*)Qs[2], (const T*)b, (T*)g.X, (T*)resid(g, 0), c, cl.ilen);
}

template <class T>
void launch_cg_precond(Grid& g, const Params<T>& P, int m) {
  if (g.cfg.precond == UF_PC_MG) {
    mg_precond<T>(g, P, m);
    return;
  }
  const CgLaunch cl = cg_launch(P.L);
  if (g.cfg.precond == UF_PC_AI2) {
    // Qv holds q only between the d/q kernel and the update: free here
    hipLaunchKernelGGL(k_ai2_v<T>, cl.grid, dim3(kCgBlock), 0, g.stream, P, (const T*)resid(g, m), (T*)g.Qv,
                       T(g.cfg.ai_omega), cl.ilen);
    TimedLaunch tl(g, UF_TK_CG_PRECOND);
    launch_k(g, k_ai2_z<T>, cl.grid, dim3(kCgBlock), P, (const T*)resid(g, m), (const T*)g.Qv, (T*)g.Z, make_ctl(g),
             m, T(g.cfg.ai_omega), cl.ilen, 1);
    return;
  }
  TimedLaunch tl(g, UF_TK_CG_PRECOND);
  launch_k(g, k_cg_precond<T>, cl.grid, dim3(kCgBlock), P, (const T*)resid(g, m), (T*)g.Z,
                     make_ctl(g), m, g.cfg.precond, T(g.cfg.ai_omega), cl.ilen);
}

template <class T>
void launch_cg_iteration(Grid& g, const Params<T>& P, int t) {
  const CgLaunch cl = cg_launch(P.L);
  const CgCtl c = make_ctl(g);
  void* Dold = g.D[t & 1];
  void* Dnew = g.D[(t + 1) & 1];
  join_x(g);
  {
    TimedLaunch tl(g, UF_TK_CG_AD);
    const AdLaunch al = ad_launch(P.L);
    if (al.kt == 64)
      launch_k(g, k_cg_Ad<64, T>, al.grid, dim3(512), P, (const T*)g.Z, (const T*)Dold, (T*)Dnew, (T*)g.Qv, (T*)g.X,
               c, t, al.ilen, al.njt, al.nkt);
    else if (al.kt == 32)
      launch_k(g, k_cg_Ad<32, T>, al.grid, dim3(512), P, (const T*)g.Z, (const T*)Dold, (T*)Dnew, (T*)g.Qv, (T*)g.X,
               c, t, al.ilen, al.njt, al.nkt);
    else
      launch_k(g, k_cg_Ad<16, T>, al.grid, dim3(512), P, (const T*)g.Z, (const T*)Dold, (T*)Dnew, (T*)g.Qv, (T*)g.X,
               c, t, al.ilen, al.njt, al.nkt);
  }
  if (g.mg_fused) {
    // r -= alpha q runs inside the multigrid's first restriction, x +=
    // alpha d beside its coarse levels
    mg_iteration_update<T>(g, P, t, Dnew);
    return;
  }
  {
    TimedLaunch tl(g, UF_TK_CG_AXPY);
    launch_k(g, k_cg_axpy<T>, cl.grid, dim3(kCgBlock), P, (T*)g.X, (const T*)resid(g, t),
                       (T*)resid(g, t + 1), (const T*)Dnew, (const T*)g.Qv, c, t, cl.ilen);
  }
  launch_cg_precond<T>(g, P, t + 1);
}

void launch_cg_status(Grid& g, int t_end) {
  hipLaunchKernelGGL(k_cg_status, dim3(1), dim3(256), 0, g.stream, make_ctl(g), t_end);
}

template <class T>
void launch_apply(Grid& g, const Params<T>& P, int op, const void* x, void* y) {
  const CgLaunch cl = cg_launch(P.L);
  if (op == UF_OP_PRECOND && g.cfg.precond == UF_PC_AI2) {
    hipLaunchKernelGGL(k_ai2_v<T>, cl.grid, dim3(kCgBlock), 0, g.stream, P, (const T*)x, (T*)g.Qv,
                       T(g.cfg.ai_omega), cl.ilen);
    hipLaunchKernelGGL(k_ai2_z<T>, cl.grid, dim3(kCgBlock), 0, g.stream, P, (const T*)x, (const T*)g.Qv, (T*)y,
                       make_ctl(g), 0, T(g.cfg.ai_omega), cl.ilen, 0);
    return;
  }
  hipLaunchKernelGGL(k_apply<T>, cl.grid, dim3(kCgBlock), 0, g.stream, P, op, g.cfg.precond, T(g.cfg.ai_omega),
                     (const T*)x, (T*)y, cl.ilen);
}

#define UF_INST(T)                                                                          \
  template void launch_cg_start<T>(Grid&, const Params<T>&, void* const[3], const void*);   \
  template void launch_cg_precond<T>(Grid&, const Params<T>&, int);                         \
  template void launch_cg_iteration<T>(Grid&, const Params<T>&, int);                       \
  template void launch_apply<T>(Grid&, const Params<T>&, int, const void*, void*);
UF_INST(float)
UF_INST(double)
#undef UF_INST

}  // namespace uf
