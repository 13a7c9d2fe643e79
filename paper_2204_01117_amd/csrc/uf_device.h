// Device-side data layout, boundary rules and reductions shared by the
// kernels of the RANS step.
//
// Storage: every field (cell scalars and the three face components) lives in
// an array of identical padded shape (nx+3) x (ny+3) x (nz+3), z fastest,
// holding one ghost layer around the interior extent of that field.  A
// common shape lets cell (i, j, k) and the faces u(i,j,k), v(i,j,k),
// w(i,j,k) share one linear offset, so stencils over several fields use the
// same neighbour strides.  Element (i, j, k), i in [-1, nx+1], is at
// (i+1)*SX + (j+1)*PZ + (k+1).
//
// Ghost values are written by the kernel that produces the interior value
// next to them (no separate fill pass): a face element on the edge of its
// interior range also writes each ghost whose nearest interior element it
// is, composing the side rules axis by axis, x first, then y, then z.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace uf {

enum SideKind { INLET = 0, OUTLET = 1, WALL = 2, SLIP = 3 };

struct Layout {
  int nx, ny, nz;
  int PZ;            // stride of j
  long long SX;      // stride of i
  __host__ __device__ __forceinline__ long long at(int i, int j, int k) const {
    return (long long)(i + 1) * SX + (long long)(j + 1) * PZ + (k + 1);
  }
};

// Everything a step kernel needs, passed by value.
template <class T>
struct Params {
  Layout L;
  int bc[6];
  T h[3];           // dx, dy, dz
  T ih[3];          // 1/h
  T ih2[3];         // 1/h^2
  T dth[3];         // dt/h (trace length per unit velocity, in cells)
  T dt, nu, rho;
  T dt_rho;         // dt / rho
  T rho_dt;         // rho / dt
  T cap;            // nu_max - nu: upper bound of the eddy viscosity
  T k_in, w_in, k_min, w_min;
  T lim_coef;       // C_lim / sqrt(C_mu / 2): omega limiter per unit |S|
  const T* inflow;  // [2][nz+2]: inflow u and v at vertical index k in [-1, nz]
};

// max/min that propagate NaN (like numpy.maximum/minimum), so that a
// non-finite value is never silently replaced by a clamp bound.
template <class T>
__device__ __forceinline__ T nmax(T a, T b) {
  return (a != a || a > b) ? a : b;
}
template <class T>
__device__ __forceinline__ T nmin(T a, T b) {
  return (a != a || a < b) ? a : b;
}

// ---------------------------------------------------------------- ghosts --
template <class T>
__device__ __forceinline__ T inflow_comp(const Params<T>& P, int c, int k) {
  if (c == 2) return T(0);
  return P.inflow[c * (P.L.nz + 2) + (k + 1)];
}

// Value of the ghost across side (a, hi) of component c, given the value v of
// its neighbour: the face beyond a normal face copies it; a tangential ghost
// takes the inflow at an inlet, -v at a no-slip wall, v otherwise.
template <class T>
__device__ __forceinline__ T face_rule(const Params<T>& P, int c, int a, int hi, T v, int k) {
  if (a == c) return v;
  const int kind = P.bc[2 * a + hi];
  if (kind == INLET) return inflow_comp(P, c, k);
  if (kind == WALL) return -v;
  return v;
}

template <int C>
__device__ __forceinline__ void face_ext(const Layout& L, int ext[3]) {
  ext[0] = L.nx + (C == 0);
  ext[1] = L.ny + (C == 1);
  ext[2] = L.nz + (C == 2);
}

// Is face (i,j,k) of component C a fixed (Dirichlet) boundary normal face?
// If so, return its value in *val.
template <int C, class T>
__device__ __forceinline__ bool face_dirichlet(const Params<T>& P, int i, int j, int k, T* val) {
  int ext[3];
  face_ext<C>(P.L, ext);
  const int idx = (C == 0) ? i : (C == 1) ? j : k;
  int side = -1;
  if (idx == 0) side = 2 * C;
  else if (idx == ext[C] - 1) side = 2 * C + 1;
  if (side < 0 || P.bc[side] == OUTLET) return false;
  *val = (P.bc[side] == INLET) ? inflow_comp(P, C, k) : T(0);
  return true;
}

// Store the value of interior face (i,j,k) of component C and every ghost
// derived from it.  Ghosts across one side are written straight-line (the
// common case: faces next to one domain side); ghosts across an edge or a
// corner compose the side rules x, then y, then z.
template <int C, class T>
__device__ __forceinline__ void store_face(T* __restrict__ q, const Params<T>& P, int i, int j, int k, T v) {
  const Layout& L = P.L;
  const long long o = L.at(i, j, k);
  q[o] = v;
  int ext[3];
  face_ext<C>(L, ext);
  const bool lo0 = i == 0, hi0 = i == ext[0] - 1;
  const bool lo1 = j == 0, hi1 = j == ext[1] - 1;
  const bool lo2 = k == 0, hi2 = k == ext[2] - 1;
  if (lo2) q[o - 1] = face_rule(P, C, 2, 0, v, k - 1);
  if (hi2) q[o + 1] = face_rule(P, C, 2, 1, v, k + 1);
  if (lo1) q[o - L.PZ] = face_rule(P, C, 1, 0, v, k);
  if (hi1) q[o + L.PZ] = face_rule(P, C, 1, 1, v, k);
  if (lo0) q[o - L.SX] = face_rule(P, C, 0, 0, v, k);
  if (hi0) q[o + L.SX] = face_rule(P, C, 0, 1, v, k);
  if (int(lo0 | hi0) + int(lo1 | hi1) + int(lo2 | hi2) < 2) return;
  for (int ox = -1; ox <= 1; ++ox) {
    if ((ox == -1 && !lo0) || (ox == 1 && !hi0)) continue;
    for (int oy = -1; oy <= 1; ++oy) {
      if ((oy == -1 && !lo1) || (oy == 1 && !hi1)) continue;
      for (int oz = -1; oz <= 1; ++oz) {
        if ((oz == -1 && !lo2) || (oz == 1 && !hi2)) continue;
        if (int(ox != 0) + int(oy != 0) + int(oz != 0) < 2) continue;
        T g = v;
        if (ox) g = face_rule(P, C, 0, ox > 0, g, k);
        if (oy) g = face_rule(P, C, 1, oy > 0, g, k);
        if (oz) g = face_rule(P, C, 2, oz > 0, g, k + oz);
        q[L.at(i + ox, j + oy, k + oz)] = g;
      }
    }
  }
}

// Store a cell value and its face-adjacent ghosts.  inlet_value is used on
// INLET sides when use_inlet is set; otherwise ghosts copy (zero gradient).
template <class T>
__device__ __forceinline__ void store_cell(T* __restrict__ q, const Params<T>& P, int i, int j, int k, T v,
                                           bool use_inlet, T inlet_value) {
  const Layout& L = P.L;
  q[L.at(i, j, k)] = v;
  const int n[3] = {L.nx, L.ny, L.nz};
  const int idx[3] = {i, j, k};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int hi = 0; hi < 2; ++hi) {
      if (idx[a] != (hi ? n[a] - 1 : 0)) continue;
      const T g = (use_inlet && P.bc[2 * a + hi] == INLET) ? inlet_value : v;
      const int o = hi ? 1 : -1;
      q[L.at(i + (a == 0) * o, j + (a == 1) * o, k + (a == 2) * o)] = g;
    }
  }
}

// Diagonal of the Poisson matrix at cell (i,j,k): 1/h^2 for every neighbour
// that is a cell or an outlet ghost (zero pressure); Neumann sides drop out.
template <class T>
__device__ __forceinline__ T poisson_diag(const Params<T>& P, int i, int j, int k) {
  const Layout& L = P.L;
  T d = T(0);
  d += ((i > 0 || P.bc[0] == OUTLET) ? P.ih2[0] : T(0)) + ((i < L.nx - 1 || P.bc[1] == OUTLET) ? P.ih2[0] : T(0));
  d += ((j > 0 || P.bc[2] == OUTLET) ? P.ih2[1] : T(0)) + ((j < L.ny - 1 || P.bc[3] == OUTLET) ? P.ih2[1] : T(0));
  d += ((k > 0 || P.bc[4] == OUTLET) ? P.ih2[2] : T(0)) + ((k < L.nz - 1 || P.bc[5] == OUTLET) ? P.ih2[2] : T(0));
  return d;
}

// ------------------------------------------------------------ reductions --
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum NV values over the block (blockDim.x a multiple of 64, <= 1024);
// the totals are valid in thread 0.  Fixed order: deterministic.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double sh[NV][16];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
  for (int m = 0; m < NV; ++m) v[m] = wave_sum(v[m]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < NV; ++m) sh[m][w] = v[m];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      double s = 0.0;
      for (int q = 0; q < nw; ++q) s += sh[m][q];
      v[m] = s;
    }
  }
}

// Launch shape of the stencil kernels: a logical gx x gy grid of blocks (bx
// fastest) launched as a 1-D grid of 8 * ceil(gx gy / 8) blocks.  Workgroups
// are dealt to the 8 XCDs round-robin; remapped this way each XCD takes one
// contiguous range of the logical order, so blocks whose halos overlap (the
// neighbouring x-planes) share that XCD's L2.  False for padding blocks.
__device__ __forceinline__ bool xcd_block(int gx, int gy, int& bx, int& by) {
  const int per = (int)(gridDim.x >> 3);
  const int b = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  if (b >= gx * gy) return false;
  by = b / gx;
  bx = b - by * gx;
  return true;
}

// Logical block b of a gx x gy grid of blocks (gy planes of gx blocks) in
// band-major order: the planes of one band of `band` consecutive blocks (the
// last band narrower) before the next band.
__device__ __forceinline__ void band_map(int gx, int gy, int band, int b, int& bx, int& by) {
  const int bw = min(band, gx);
  const int nfull = gx / bw;                 // bands of bw blocks
  const int full = nfull * bw * gy;          // logical blocks in them
  if (b < full) {
    const int bd = b / (bw * gy), rem = b - bd * bw * gy;
    by = rem / bw;
    bx = bd * bw + (rem - by * bw);
  } else {
    const int wl = gx - nfull * bw, rem = b - full;   // the last, narrower band
    by = rem / wl;
    bx = nfull * bw + (rem - by * wl);
  }
}

inline dim3 xcd_grid(int gx, int gy) {
  const long long n = (long long)gx * gy;
  return dim3((unsigned)(8 * ((n + 7) / 8)));
}

}  // namespace uf
