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
}

// One block: ||b||, the stopping threshold and whether x0 already solves.
__global__ __launch_bounds__(256) void k_cg_start(CgCtl c, double tol) {
  const double bb = slot_sum(c.part + (size_t)S_BB * c.stride, c.nb);
  const double rr = slot_sum(c.part + (size_t)S_RR * c.stride, c.nb);
  if (threadIdx.x != 0) return;
  CgState* st = c.st;
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

// d = z + beta d_old; q = A d; partials of d.q.  Marches along x with the
// x-neighbours of d in registers.
template <class T>
__global__ __launch_bounds__(kCgBlock) void k_cg_Ad(Params<T> P, const T* __restrict__ Z, const T* __restrict__ Dold,
                                                    T* __restrict__ Dnew, T* __restrict__ Qv, T* __restrict__ X,
                                                    CgCtl c, int t, int ilen) {
  const Layout& L = P.L;
  UF_CG_RANGE(L, ilen);
  if (t == 0 && c.flags[0] && c.st->zero_rhs) {
    // b = 0: the solution is x = 0
    for (int i = i0; i < i1; ++i) X[L.at(i, j, k)] = T(0);
    return;
  }
  if (!iteration_open(c, t)) return;
  const bool first = t == 0;
  const long long SX = L.SX, PZ = L.PZ;
  const bool work = i0 < i1;
  const bool pass0 = i0 + 4 <= i1;
  long long o = work ? L.at(i0, j, k) : 0;
  // Raw z and d_old of the first pass (cells i0 .. i0+3, their x-neighbours
  // and their y/z-neighbours) are loaded before beta is known, so that the
  // sum of the r.z partials overlaps those loads.  Entry p: 0 = i0-1,
  // 1..5 = i0..i0+4, then four groups of four (+y, -y, +z, -z).
  const int sx = (int)SX, pz = (int)PZ;   // a plane of the padded layout is far below 2^31 elements
  auto off = [&](int p) -> int {
    if (p == 0) return -sx;
    if (p < 6) return (p - 1) * sx;
    const int u = (p - 6) & 3, g = (p - 6) >> 2;
    return u * sx + (g == 0 ? pz : (g == 1 ? -pz : (g == 2 ? 1 : -1)));
  };
  T zr[22], dr[22];
  const T* __restrict__ zo = Z + o;
  const T* __restrict__ d0 = Dold + o;
#pragma unroll
  for (int p = 0; p < 22; ++p) {
    zr[p] = T(0);
    dr[p] = T(0);
    if (work && (p < 2 || pass0)) {
      zr[p] = zo[off(p)];
      if (!first) dr[p] = d0[off(p)];
    }
  }
  const double rz = rz_of(c, t);
  if (blockIdx.x == 0 && threadIdx.x == 0) c.st->rzh[t & 1] = rz;
  if (!rz_allows(c, rz)) return;
  // r.z of iteration t - 1 was published by this kernel's previous launch
  const T beta = first ? T(0) : (T)(rz / c.st->rzh[(t + 1) & 1]);
  double v[1] = {0.0};
  if (work) {
    auto dn = [&](long long q) { return first ? Z[q] : Z[q] + beta * Dold[q]; };
    auto dv = [&](int p) { return first ? zr[p] : zr[p] + beta * dr[p]; };
    const T dyz = diag_yz(P, j, k);
    T dm = dv(0), dc = dv(1);
    int i = i0;
    // four cells per pass so that each wave keeps four cells' loads in flight
    auto pass = [&](const T (&d)[5], const T (&lat_y)[4], const T (&lat_z)[4]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const T prev = u == 0 ? dm : d[u - 1];
        const T qv = (dyz + diag_x(P, i + u)) * d[u] - (d[u + 1] + prev) * P.ih2[0] - lat_y[u] * P.ih2[1] -
                     lat_z[u] * P.ih2[2];
        Dnew[o + u * SX] = d[u];
        Qv[o + u * SX] = qv;
        v[0] += (double)d[u] * (double)qv;
      }
      dm = d[3];
      dc = d[4];
      i += 4;
      o += 4 * SX;
    };
    if (pass0) {
      T d[5], lat_y[4], lat_z[4];
#pragma unroll
      for (int u = 0; u < 5; ++u) d[u] = dv(1 + u);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        lat_y[u] = dv(6 + u) + dv(10 + u);
        lat_z[u] = dv(14 + u) + dv(18 + u);
      }
      pass(d, lat_y, lat_z);
    }
    while (i + 4 <= i1) {
      T d[5], lat_y[4], lat_z[4];
      d[0] = dc;
#pragma unroll
      for (int u = 1; u <= 4; ++u) d[u] = dn(o + u * SX);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const long long q = o + u * SX;
        lat_y[u] = dn(q + PZ) + dn(q - PZ);
        lat_z[u] = dn(q + 1) + dn(q - 1);
      }
      pass(d, lat_y, lat_z);
    }
    for (; i < i1; ++i, o += SX) {
      const T dp = dn(o + SX);
      const T q = (dyz + diag_x(P, i)) * dc - (dp + dm) * P.ih2[0] - (dn(o + PZ) + dn(o - PZ)) * P.ih2[1] -
                  (dn(o + 1) + dn(o - 1)) * P.ih2[2];
      Dnew[o] = dc;
      Qv[o] = q;
      v[0] += (double)dc * (double)q;
      dm = dc;
      dc = dp;
    }
  }
  const int slots[1] = {S_DQ};
  write_partials<1>(v, c.part, c.stride, slots, cg_bid);
}

// x += alpha d; r -= alpha q; partials of ||r||^2.
template <class T>
__global__ __launch_bounds__(kCgBlock) void k_cg_axpy(Params<T> P, T* __restrict__ X, const T* __restrict__ Rin,
                                                      T* __restrict__ R, const T* __restrict__ D,
                                                      const T* __restrict__ Qv, CgCtl c, int t, int ilen) {
  const Layout& L = P.L;
  double rz = 0.0, dq = 0.0;
  bool run = iteration_open(c, t);
  if (run) {
    rz = c.st->rzh[t & 1];
    run = rz_allows(c, rz);
  }
  if (run) {
    dq = slot_sum(c.part + (size_t)S_DQ * c.stride, c.nb);
    run = dq > 0.0 && isfinite(dq);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c.exec[t] = run;
    if (run) c.st->iter = t + 1;
  }
  if (!run) return;
  UF_CG_RANGE(L, ilen);
  const T alpha = (T)(rz / dq);
  double v[1] = {0.0};
#pragma unroll 4
  for (int i = i0; i < i1; ++i) {
    const long long o = L.at(i, j, k);
    X[o] += alpha * D[o];
    const T r = Rin[o] - alpha * Qv[o];
    R[o] = r;
    v[0] += (double)r * (double)r;
  }
  const int slots[1] = {S_RR};
  write_partials<1>(v, c.part, c.stride, slots, cg_bid);
}

// One block, after a chunk of iterations ending at t_end: publish the
// status for the host.
__global__ __launch_bounds__(256) void k_cg_status(CgCtl c, int t_end) {
  const double rr = slot_sum(c.part + (size_t)S_RR * c.stride, c.nb);
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

CgCtl make_ctl(Grid& g) {
  CgCtl c;
  c.part = g.partials;
  c.stride = (int)g.part_stride;
  c.nb = (int)g.cg_nb;
  c.nb_rz = (int)g.cg_nb_rz;
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
}

template <class T>
void launch_cg_precond(Grid& g, const Params<T>& P, int m) {
  if (g.cfg.precond == UF_PC_MG) {
    mg_precond<T>(g, P, m);
    return;
  }
  const CgLaunch cl = cg_launch(P.L);
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
  {
    TimedLaunch tl(g, UF_TK_CG_AD);
    launch_k(g, k_cg_Ad<T>, cl.grid, dim3(kCgBlock), P, (const T*)g.Z, (const T*)Dold, (T*)Dnew,
                       (T*)g.Qv, (T*)g.X, c, t, cl.ilen);
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
