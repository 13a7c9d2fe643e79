// Geometric multigrid V-cycle used as the CG preconditioner.
//
// Cell-centred hierarchy: an axis is halved while its cell count is even
// and at least 4; levels stop at <= 256 cells (or when no axis halves).
// Restriction averages the children (R = P^T / m, m children per coarse
// cell) and prolongation copies the parent (piecewise constant P).  The
// coarse operator is the Galerkin product R A P, which for this pair is
// again a 7-point stencil with the same boundary rows and per-axis weights
// halved on every halved axis.  Smoothing: one damped-Jacobi sweep before
// (from zero) and one after the coarse correction, so the V-cycle is a
// fixed symmetric positive-definite operator as PCG requires.  The coarsest
// level is solved with its exact dense inverse (<= 512 cells) or, failing
// that, with a fixed number of Jacobi sweeps.
//
// Kernels per application: restrict level 0 -> 1 (and decide whether the
// solve has already finished), restrict down to the first small level, one
// single-workgroup kernel for all small levels, prolongate + smooth back up,
// and the fine-level prolongation + smoothing that writes z and r.z.
#include <cmath>
#include <cstdlib>
#include <vector>

#include "pressure_common.h"

namespace uf {

constexpr int kMgMaxLevels = 16;
constexpr int kTailThreads = 1024;
constexpr int kMgFineBlock = 512;   // must match the CG kernels' block (cg_launch)
constexpr long long kTailCells = 1024;   // levels this small run in the single-workgroup kernel
constexpr int kDenseMax = 512;           // largest coarsest level with an exact inverse
constexpr int kCoarseSweeps = 10;        // Jacobi sweeps when there is no exact inverse
// Smoother weight and coarse-correction scaling, chosen by measured PCG
// iteration counts on the 256x256x64 and 512x512x128 workloads (alpha in
// [1.4, 1.7] and omega 0.9 are within a few percent of each other; alpha = 1
// needs 40-75% more iterations).  A scaled coarse correction keeps the
// V-cycle symmetric; it compensates the low accuracy of piecewise-constant
// prolongation for smooth error.
constexpr double kJacobiOmega = 0.9;
constexpr double kCoarseAlpha = 1.5;

template <class T>
struct MgLvl {
  Layout L;
  T w[3];
  T omd_in;   // om / D of an interior cell
  int c[3];   // axis halved towards the next level
  int m;      // children per next-level cell
  T* r;
  T* x;
  T* t;       // scratch (coarsest-level Jacobi)
};

// Scalars shared by every level.  Kernels get these and the descriptors of
// the one or two levels they touch as separate by-value arguments (a
// dynamically indexed table in the arguments would live in scratch memory).
template <class T>
struct MgCommon {
  int bc[6];
  T om;       // Jacobi weight
  T alpha;    // scaling of the coarse-grid correction
};

__device__ __forceinline__ void decode(int idx, const Layout& L, int& i, int& j, int& k) {
  k = idx % L.nz;
  const int r = idx / L.nz;
  j = r % L.ny;
  i = r / L.ny;
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

// Residual of the pre-smoothed level-F problem averaged over the children
// of next-level cell (I, J, K): mean over children f of r_f - (A e)_f with
// e = om D^-1 r (one Jacobi sweep from zero), i.e.
//   r_f - om r_f + sum_a w_a (e_{f+a} + e_{f-a}).
template <class T>
__device__ __forceinline__ T down_body(const MgCommon<T>& K, const MgLvl<T>& F, int I, int J, int Kc) {
  const Layout& L = F.L;
  const T* __restrict__ r = F.r;
  auto e_at = [&](int i, int j, int k) -> T { return omd(K, F, i, j, k) * r[L.at(i, j, k)]; };
  T acc = T(0);
  for (int a0 = 0; a0 <= F.c[0]; ++a0)
    for (int a1 = 0; a1 <= F.c[1]; ++a1)
      for (int a2 = 0; a2 <= F.c[2]; ++a2) {
        const int i = (I << F.c[0]) + a0, j = (J << F.c[1]) + a1, k = (Kc << F.c[2]) + a2;
        const T rf = r[L.at(i, j, k)];
        const T s = F.w[0] * (e_at(i + 1, j, k) + e_at(i - 1, j, k)) + F.w[1] * (e_at(i, j + 1, k) + e_at(i, j - 1, k)) +
                    F.w[2] * (e_at(i, j, k + 1) + e_at(i, j, k - 1));
        acc += (T(1) - K.om) * rf + s;
      }
  return acc / T(F.m);
}

// Value before post-smoothing at a cell of level F: the pre-smoothed
// om D^-1 r plus the prolongated, scaled coarse correction.  Zero outside
// the level (r and the coarse correction have zero ghosts).
template <bool COARSE, class T>
__device__ __forceinline__ T pre_plus_coarse(const MgCommon<T>& K, const MgLvl<T>& F, const MgLvl<T>& C, int i, int j,
                                             int k) {
  T v = omd(K, F, i, j, k) * F.r[F.L.at(i, j, k)];
  if (COARSE) v += K.alpha * C.x[C.L.at(i >> F.c[0], j >> F.c[1], k >> F.c[2])];
  return v;
}

// t = om D^-1 r + alpha P x_c; one Jacobi sweep: x = t + om D^-1 (r - A t).
template <bool COARSE, class T>
__device__ __forceinline__ T up_body(const MgCommon<T>& K, const MgLvl<T>& F, const MgLvl<T>& C, int i, int j, int k) {
  const Layout& L = F.L;
  const T D = diag_w(K.bc, L, F.w, i, j, k);
  const T tc = pre_plus_coarse<COARSE>(K, F, C, i, j, k);
  const T At = D * tc -
               F.w[0] * (pre_plus_coarse<COARSE>(K, F, C, i + 1, j, k) + pre_plus_coarse<COARSE>(K, F, C, i - 1, j, k)) -
               F.w[1] * (pre_plus_coarse<COARSE>(K, F, C, i, j + 1, k) + pre_plus_coarse<COARSE>(K, F, C, i, j - 1, k)) -
               F.w[2] * (pre_plus_coarse<COARSE>(K, F, C, i, j, k + 1) + pre_plus_coarse<COARSE>(K, F, C, i, j, k - 1));
  return tc + omd(K, F, i, j, k) * (F.r[L.at(i, j, k)] - At);
}

__host__ __device__ static inline long long ncells(const Layout& L) { return (long long)L.nx * L.ny * L.nz; }

// Restrict level 0 -> 1; also decides whether the solve finished before
// this preconditioner application (block 0 publishes it in flags[m]).
template <class T>
__global__ __launch_bounds__(256) void k_mg_down0(MgCommon<T> K, MgLvl<T> F, MgLvl<T> C, int has_coarse, CgCtl c,
                                                  int m, int decide) {
  const bool skip = decide ? precond_skip(c, m) : false;
  if (blockIdx.x == 0 && threadIdx.x == 0) c.flags[m] = skip;
  if (skip || !has_coarse) return;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ncells(C.L)) return;
  int I, J, Kc;
  decode(idx, C.L, I, J, Kc);
  C.r[C.L.at(I, J, Kc)] = down_body(K, F, I, J, Kc);
}

template <class T>
__global__ __launch_bounds__(256) void k_mg_down(MgCommon<T> K, MgLvl<T> F, MgLvl<T> C, const int* __restrict__ flags,
                                                 int m) {
  if (flags[m]) return;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ncells(C.L)) return;
  int I, J, Kc;
  decode(idx, C.L, I, J, Kc);
  C.r[C.L.at(I, J, Kc)] = down_body(K, F, I, J, Kc);
}

template <class T>
__global__ __launch_bounds__(256) void k_mg_up(MgCommon<T> K, MgLvl<T> F, MgLvl<T> C, const int* __restrict__ flags,
                                               int m) {
  if (flags[m]) return;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ncells(F.L)) return;
  int i, j, k;
  decode(idx, F.L, i, j, k);
  F.x[F.L.at(i, j, k)] = up_body<true>(K, F, C, i, j, k);
}

// All levels from lt down to the coarsest and back, in one workgroup.  The
// level descriptors are read from a device table.
template <class T>
__global__ __launch_bounds__(kTailThreads) void k_mg_tail(MgCommon<T> K, const MgLvl<T>* __restrict__ lv, int lt,
                                                          int nl, const T* __restrict__ cinv,
                                                          const int* __restrict__ flags, int m) {
  if (flags[m]) return;
  __shared__ T rs[kDenseMax];
  for (int l = lt; l < nl - 1; ++l) {
    const MgLvl<T> F = lv[l];
    const MgLvl<T> C = lv[l + 1];
    const int n = (int)ncells(C.L);
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
      int I, J, Kc;
      decode(idx, C.L, I, J, Kc);
      C.r[C.L.at(I, J, Kc)] = down_body(K, F, I, J, Kc);
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
    const int n = (int)ncells(F.L);
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
      int i, j, k;
      decode(idx, F.L, i, j, k);
      F.x[F.L.at(i, j, k)] = up_body<true>(K, F, C, i, j, k);
    }
    __syncthreads();
  }
}

// Fine level: z = (prolongation + post-smoothing) and partials of r.z.
// Marches along x keeping the x-neighbours' values in registers.
template <bool COARSE, class T>
__global__ __launch_bounds__(kMgFineBlock) void k_mg_up0(MgCommon<T> K, MgLvl<T> F, MgLvl<T> C, CgCtl c, int m,
                                                         int ilen) {
  if (c.flags[m]) return;
  const Layout& L = F.L;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = p < L.ny * L.nz;
  const int j = active ? p / L.nz : 0;
  const int k = active ? p - j * L.nz : 0;
  const int i0 = blockIdx.y * ilen;
  const int i1 = active ? min(L.nx, i0 + ilen) : i0;
  double v[1] = {0.0};
  if (i0 < i1) {
    T tm = pre_plus_coarse<COARSE>(K, F, C, i0 - 1, j, k);
    T tc = pre_plus_coarse<COARSE>(K, F, C, i0, j, k);
    for (int i = i0; i < i1; ++i) {
      const T tp = pre_plus_coarse<COARSE>(K, F, C, i + 1, j, k);
      const T D = diag_w(K.bc, L, F.w, i, j, k);
      const T At = D * tc - F.w[0] * (tp + tm) -
                   F.w[1] * (pre_plus_coarse<COARSE>(K, F, C, i, j + 1, k) + pre_plus_coarse<COARSE>(K, F, C, i, j - 1, k)) -
                   F.w[2] * (pre_plus_coarse<COARSE>(K, F, C, i, j, k + 1) + pre_plus_coarse<COARSE>(K, F, C, i, j, k - 1));
      const long long o = L.at(i, j, k);
      const T rr = F.r[o];
      const T z = tc + omd(K, F, i, j, k) * (rr - At);
      F.x[o] = z;
      v[0] += (double)rr * (double)z;
      tm = tc;
      tc = tp;
    }
  }
  const int slots[1] = {S_RZ0 + (m & 1)};
  write_partials<1>(v, c.part, c.nb, slots);
}

// ------------------------------------------------------------------- host
template <class T>
static MgCommon<T> mg_common(const Grid& g) {
  MgCommon<T> K{};
  for (int q = 0; q < 6; ++q) K.bc[q] = g.bc[q];
  K.om = T(g.mg_omega);
  K.alpha = T(g.mg_alpha);
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
  D.m = 1 << (S.coarsen[0] + S.coarsen[1] + S.coarsen[2]);
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
      C.w[a] = F.w[a] / (c[a] ? 2.0 : 1.0);   // Galerkin weight of R A P
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
  g.mg_alpha = kCoarseAlpha;
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

template <class T>
void mg_launch(Grid& g, const Params<T>& P, int m, const void* r, void* z, int decide) {
  (void)P;
  const MgCommon<T> K = mg_common<T>(g);
  const CgCtl c = make_ctl(g);
  const int nl = (int)g.mg.size();
  MgLvl<T> L0 = mg_level<T>(g, 0);
  L0.r = (T*)r;
  L0.x = (T*)z;
  const MgLvl<T> L1 = nl > 1 ? mg_level<T>(g, 1) : L0;
  const int nb1 = nl > 1 ? (int)((ncells(L1.L) + 255) / 256) : 1;
  hipLaunchKernelGGL(k_mg_down0<T>, dim3(nb1), dim3(256), 0, g.stream, K, L0, L1, nl > 1 ? 1 : 0, c, m, decide);
  const int lt = std::min(g.mg_lt, nl - 1);
  for (int l = 1; l < lt; ++l) {
    const MgLvl<T> F = mg_level<T>(g, l), C = mg_level<T>(g, l + 1);
    const int nb = (int)((ncells(C.L) + 255) / 256);
    hipLaunchKernelGGL(k_mg_down<T>, dim3(nb), dim3(256), 0, g.stream, K, F, C, (const int*)c.flags, m);
  }
  if (nl > 1) {
    hipLaunchKernelGGL(k_mg_tail<T>, dim3(1), dim3(kTailThreads), 0, g.stream, K, (const MgLvl<T>*)g.mg_table, lt, nl,
                       (const T*)g.mg_cinv, (const int*)c.flags, m);
    for (int l = lt - 1; l >= 1; --l) {
      const MgLvl<T> F = mg_level<T>(g, l), C = mg_level<T>(g, l + 1);
      const int nb = (int)((ncells(F.L) + 255) / 256);
      hipLaunchKernelGGL(k_mg_up<T>, dim3(nb), dim3(256), 0, g.stream, K, F, C, (const int*)c.flags, m);
    }
  }
  const CgLaunch cl = cg_launch(g.L);
  if (nl > 1)
    hipLaunchKernelGGL((k_mg_up0<true, T>), cl.grid, dim3(kMgFineBlock), 0, g.stream, K, L0, L1, c, m, cl.ilen);
  else
    hipLaunchKernelGGL((k_mg_up0<false, T>), cl.grid, dim3(kMgFineBlock), 0, g.stream, K, L0, L1, c, m, cl.ilen);
}

template <class T>
void mg_precond(Grid& g, const Params<T>& P, int m) {
  mg_launch<T>(g, P, m, g.R, g.Z, 1);
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

}  // namespace uf
