// Helpers shared by the pressure-solve kernels (CG and multigrid).
//
// Cell vectors of the solve keep zero ghosts; the operator at a cell is
//   (A x)_c = D_c x_c - sum_a w_a (x_{c+a} + x_{c-a})
// with per-axis weights w_a (1/h_a^2 on the fine grid) and D_c = sum of w_a
// over the neighbours that are cells or outlet ghosts (zero pressure);
// Neumann sides drop out.
#pragma once
#include "uf_internal.h"

namespace uf {

// Partial-sum slots of the solve: every block of a reducing kernel writes
// its FP64 partial into part[slot * stride + block]; later kernels add the
// block partials in block order (no atomics, no intra-kernel cross-block
// traffic).
enum CgSlot { S_BB = 0, S_RR = 1, S_DQ = 2, S_RZ0 = 3, S_RZ1 = 4, S_NSLOT = 5 };

template <class T>
__device__ __forceinline__ T diag_w(const int bc[6], const Layout& L, const T w[3], int i, int j, int k) {
  T d = T(0);
  d += ((i > 0 || bc[0] == OUTLET) ? w[0] : T(0)) + ((i < L.nx - 1 || bc[1] == OUTLET) ? w[0] : T(0));
  d += ((j > 0 || bc[2] == OUTLET) ? w[1] : T(0)) + ((j < L.ny - 1 || bc[3] == OUTLET) ? w[1] : T(0));
  d += ((k > 0 || bc[4] == OUTLET) ? w[2] : T(0)) + ((k < L.nz - 1 || bc[5] == OUTLET) ? w[2] : T(0));
  return d;
}

template <class T>
__device__ __forceinline__ T apply_w(const int bc[6], const Layout& L, const T w[3], const T* __restrict__ x, int i,
                                     int j, int k, long long o) {
  return diag_w(bc, L, w, i, j, k) * x[o] - (x[o + L.SX] + x[o - L.SX]) * w[0] - (x[o + L.PZ] + x[o - L.PZ]) * w[1] -
         (x[o + 1] + x[o - 1]) * w[2];
}

// Sum of one partial-sum slot, identical in every thread of the block.
__device__ __forceinline__ double slot_sum(const double* __restrict__ part, int nb) {
  __shared__ double sh[16];
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) v += part[b];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < nw; ++q) s += sh[q];
  __syncthreads();
  return s;
}

// Write the block's partial sums of NV values into their slots (slot s
// starts at part + s * stride; bid = the block's logical index).
template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], double* __restrict__ part, int stride,
                                               const int slot[NV], int bid) {
  block_sum<NV>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < NV; ++m) part[(size_t)slot[m] * stride + bid] = v[m];
  }
}

// State of the solve shared by the kernels (passed by value).
struct CgCtl {
  double* part;    // S_NSLOT slots of partial sums, slot s at part + s * stride
  int stride;
  int nb;          // blocks of the CG kernels (slots BB, RR, DQ)
  int nb_rz;       // blocks of the kernel writing r.z (slots RZ0, RZ1)
  int nb_dq;       // blocks of the d/q kernel (slot DQ)
  int nb_rr;       // partials of slot RR (its writers zero the ones past their blocks)
  int* flags;      // flags[m]: the solve finished before iteration m
  int* exec;       // exec[t]: iteration t performed its update
  CgState* st;
  int criterion;
  int maxit;
};

struct Grid;
CgCtl make_ctl(Grid& g);

// Has the solve finished before the preconditioner application that
// follows iteration t (m = t + 1)?  Evaluated by the first kernel of that
// application; its block 0 publishes the answer in flags[m].
// Kernels with different block counts write the r.r partials: each writer
// zeroes the slots past its own blocks (block b the slots b + n, b + 2n, ...
// below the total), so that the sum over nb_rr entries is the full sum.
__device__ __forceinline__ void pad_partials(const CgCtl& c, int slot, int bid, int nwriters) {
  if (threadIdx.x == 0)
    for (int q = bid + nwriters; q < c.nb_rr; q += nwriters) c.part[(size_t)slot * c.stride + q] = 0.0;
}

__device__ __forceinline__ bool precond_skip(const CgCtl& c, int m) {
  if (m == 0) return c.flags[0] != 0;
  if (!c.exec[m - 1]) return true;
  const double rr = slot_sum(c.part + (size_t)S_RR * c.stride, c.nb_rr);
  if (!isfinite(rr)) return true;
  return c.criterion == 0 && rr <= c.st->tol2_bb;
}

// Does iteration t run?  The d/q kernel of iteration t adds the r.z
// partials (rz_of) and block 0 publishes the sum in st->rzh[t & 1]; the
// update kernel reads it back (rz_published), so both take the same
// decision from the same value.
__device__ __forceinline__ bool iteration_open(const CgCtl& c, int t) { return !c.flags[t] && t < c.maxit; }

__device__ __forceinline__ double rz_of(const CgCtl& c, int t) {
  return slot_sum(c.part + (size_t)(S_RZ0 + (t & 1)) * c.stride, c.nb_rz);
}

__device__ __forceinline__ bool rz_allows(const CgCtl& c, double rz) {
  if (!isfinite(rz)) return false;
  if (c.criterion == 1 && rz < c.st->tol2_bb) return false;
  return true;
}

}  // namespace uf
