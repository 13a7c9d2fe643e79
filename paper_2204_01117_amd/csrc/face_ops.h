// Face-centred helpers shared by the momentum stages and their reverse
// (adjoint) kernels: face ownership, the velocity vector at a face, the
// trilinear sample of a face array, and the thread mapping of the face
// kernels (one thread per cell corner, three faces each).
#pragma once
#include "uf_internal.h"

namespace uf {

constexpr int kFaceBlock = 256;

template <int C, class T>
__device__ __forceinline__ bool owns_face(const Layout& L, int i, int j, int k) {
  if (C == 0) return j < L.ny && k < L.nz;
  if (C == 1) return i < L.nx && k < L.nz;
  return i < L.nx && j < L.ny;
}

template <int C>
__device__ __forceinline__ long long stride(const Layout& L) {
  return C == 0 ? L.SX : (C == 1 ? (long long)L.PZ : 1LL);
}

// Velocity vector at face (i,j,k) of component C: the stored component, and
// for each other component the mean of its four nearest faces (offsets
// {-1, 0} along C and {0, +1} along that component's own axis).
template <int C, class T>
__device__ __forceinline__ void face_velocity(const Layout& L, const T* __restrict__ U, const T* __restrict__ V,
                                              const T* __restrict__ W, long long o, T vel[3]) {
  const T* Qs[3] = {U, V, W};
  const long long st[3] = {L.SX, (long long)L.PZ, 1LL};
  const long long sc = st[C];
#pragma unroll
  for (int cp = 0; cp < 3; ++cp) {
    if (cp == C) {
      vel[cp] = Qs[cp][o];
    } else {
      const T* q = Qs[cp];
      const long long s2 = st[cp];
      vel[cp] = T(0.25) * (q[o - sc] + q[o - sc + s2] + q[o] + q[o + s2]);
    }
  }
}

// A trace position along one axis, n + s: n the face's integer index, s the
// signed displacement in cells (-V dt / h for the forward trace).  The
// position is clamped to [-1, ext] and its cell and fraction taken in the
// displacement's frame, where the bounds -1 - n and ext - n are exact
// integers: c = n + floor(s'), t = s' - floor(s') for the clamped s'.  They
// are then exact in the kernel's precision -- forming n + s first would
// round s to the spacing of floats near n (2^-24 n, about 3e-5 cells at
// n = 512 in FP32), and a position within that distance of a cell boundary
// could land in either cell: with the MacCormack clamp, whose range is the
// eight samples of that cell, a different value.  As for the position: a
// clamped top end gives (ext - 1, t = 1), a NaN displacement (-1, 0); live
// is false when the clamp moved the position.
template <class T>
struct AxisPos {
  int c;
  T t;
  bool live;
};

template <class T>
__device__ __forceinline__ AxisPos<T> trace_axis(int n, T s, int ext) {
  const T lo = T(-1 - n), hi = T(ext - n);
  const T sc = fmin(fmax(s, lo), hi);
  const T fl = fmin(floor(sc), hi - T(1));
  AxisPos<T> a;
  a.c = n + (int)fl;
  a.t = sc - fl;
  a.live = s >= lo && s <= hi;
  return a;
}

template <int C, class T>
__device__ __forceinline__ void trace_pos(const Layout& L, int i, int j, int k, T si, T sj, T sk, AxisPos<T> a[3]) {
  int ext[3];
  face_ext<C>(L, ext);
  a[0] = trace_axis(i, si, ext[0]);
  a[1] = trace_axis(j, sj, ext[1]);
  a[2] = trace_axis(k, sk, ext[2]);
}

// Trilinear interpolation of component C's padded array at the trace
// position (i + si, j + sj, k + sk) (unpadded indices), clamped to the
// padded extent.  Optionally returns the min and max of the eight samples.
template <int C, bool MINMAX, class T>
__device__ __forceinline__ T sample(const Layout& L, const T* __restrict__ q, int i, int j, int k, T si, T sj, T sk,
                                    T* mn, T* mx) {
  AxisPos<T> a[3];
  trace_pos<C>(L, i, j, k, si, sj, sk, a);
  const T ti = a[0].t, tj = a[1].t, tk = a[2].t;
  const long long o = L.at(a[0].c, a[1].c, a[2].c);
  const long long SX = L.SX, PZ = L.PZ;
  const T s000 = q[o], s100 = q[o + SX], s010 = q[o + PZ], s110 = q[o + SX + PZ];
  const T s001 = q[o + 1], s101 = q[o + SX + 1], s011 = q[o + PZ + 1], s111 = q[o + SX + PZ + 1];
  const T c00 = s000 + ti * (s100 - s000);
  const T c10 = s010 + ti * (s110 - s010);
  const T c01 = s001 + ti * (s101 - s001);
  const T c11 = s011 + ti * (s111 - s011);
  const T c0 = c00 + tj * (c10 - c00);
  const T c1 = c01 + tj * (c11 - c01);
  if (MINMAX) {
    *mn = fmin(fmin(fmin(s000, s100), fmin(s010, s110)), fmin(fmin(s001, s101), fmin(s011, s111)));
    *mx = fmax(fmax(fmax(s000, s100), fmax(s010, s110)), fmax(fmax(s001, s101), fmax(s011, s111)));
  }
  return c0 + tk * (c1 - c0);
}

// ------------------------------------------- 32-bit trilinear sampling ---
// The advection kernels address the padded arrays with 32-bit unsigned
// element offsets when an array's bytes stay below 4 GiB (the launchers
// check; larger grids take the 64-bit kernels).  A sample is split in three
// so that a kernel can issue loads before it evaluates anything:
// tri_corner() clamps the trace position and gives the corner offset and
// weights (no memory access), tri_load() issues the eight loads, tri_eval()
// interpolates (the arithmetic of sample()).  A NaN position is clamped
// like any other, so the loads stay inside the array; the kernels replace
// such a value by NaN afterwards.
template <class T>
struct Tri {
  unsigned o;
  T ti, tj, tk;
};

template <int C, class T>
__device__ __forceinline__ Tri<T> tri_corner(const Layout& L, int i, int j, int k, T si, T sj, T sk) {
  AxisPos<T> a[3];
  trace_pos<C>(L, i, j, k, si, sj, sk, a);
  Tri<T> t;
  t.o = (unsigned)(a[0].c + 1) * (unsigned)L.SX + (unsigned)(a[1].c + 1) * (unsigned)L.PZ + (unsigned)(a[2].c + 1);
  t.ti = a[0].t;
  t.tj = a[1].t;
  t.tk = a[2].t;
  return t;
}

// s: the samples 000, 100, 010, 110, 001, 101, 011, 111 (digits i, j, k).
template <class T>
__device__ __forceinline__ void tri_load(const T* __restrict__ q, const Layout& L, unsigned o, T s[8]) {
  const unsigned SX = (unsigned)L.SX, PZ = (unsigned)L.PZ;
  s[0] = q[o];
  s[1] = q[o + SX];
  s[2] = q[o + PZ];
  s[3] = q[o + SX + PZ];
  s[4] = q[o + 1];
  s[5] = q[o + SX + 1];
  s[6] = q[o + PZ + 1];
  s[7] = q[o + SX + PZ + 1];
}

template <class T>
__device__ __forceinline__ T tri_eval(const Tri<T>& t, const T s[8]) {
  const T c00 = s[0] + t.ti * (s[1] - s[0]);
  const T c10 = s[2] + t.ti * (s[3] - s[2]);
  const T c01 = s[4] + t.ti * (s[5] - s[4]);
  const T c11 = s[6] + t.ti * (s[7] - s[6]);
  const T c0 = c00 + t.tj * (c10 - c00);
  const T c1 = c01 + t.tj * (c11 - c01);
  return c0 + t.tk * (c1 - c0);
}

template <class T>
__device__ __forceinline__ void tri_range(const T s[8], T& mn, T& mx) {
  mn = fmin(fmin(fmin(s[0], s[1]), fmin(s[2], s[3])), fmin(fmin(s[4], s[5]), fmin(s[6], s[7])));
  mx = fmax(fmax(fmax(s[0], s[1]), fmax(s[2], s[3])), fmax(fmax(s[4], s[5]), fmax(s[6], s[7])));
}

// face_velocity() with 32-bit offsets.
template <int C, class T>
__device__ __forceinline__ void face_velocity32(const Layout& L, const T* __restrict__ U, const T* __restrict__ V,
                                                const T* __restrict__ W, unsigned o, T vel[3]) {
  const T* Qs[3] = {U, V, W};
  const unsigned st[3] = {(unsigned)L.SX, (unsigned)L.PZ, 1u};
  const unsigned sc = st[C];
#pragma unroll
  for (int cp = 0; cp < 3; ++cp) {
    if (cp == C) {
      vel[cp] = Qs[cp][o];
    } else {
      const T* q = Qs[cp];
      const unsigned s2 = st[cp];
      vel[cp] = T(0.25) * (q[o - sc] + q[o - sc + s2] + q[o] + q[o + s2]);
    }
  }
}

template <class T>
__device__ __forceinline__ bool any_nan3(const T v[3]) {
  return v[0] != v[0] || v[1] != v[1] || v[2] != v[2];
}

// NaN when b holds, else +0 (x + nan_if(b) is x for every x but -0).
template <class T>
__device__ __forceinline__ T nan_if(bool b) {
  return b ? T(NAN) : T(0);
}

// Largest element offset (exclusive) of a padded array, and whether 32-bit
// byte offsets reach all of it.
inline bool offsets_fit_32(const Layout& L, size_t esize) {
  const unsigned long long n = (unsigned long long)(L.nx + 3) * (unsigned long long)L.SX;
  return n * esize < (1ULL << 32);
}

__host__ __device__ inline int face_gx(const Layout& L) { return ((L.ny + 1) * (L.nz + 1) + kFaceBlock - 1) / kFaceBlock; }

// Blocks of a plane taken together along x (bands of (j, k) points).
constexpr int kFaceBand = 8;

// Logical block (bx, i) of a face kernel launched on xcd_grid(face_gx, nx
// + 1): every XCD takes a contiguous range of the logical order, as
// xcd_block(), and that order is band-major (band_map), so the blocks in
// flight on an XCD cover a few dozen planes of one band and the
// neighbouring planes a trace or stencil reads stay in that XCD's L2
// (plane by plane over the whole (j, k) range, the six arrays of three
// neighbouring planes of a 512x128 cross-section are 4.8 MB, more than the
// 4 MB L2).  False for padding blocks.
__device__ __forceinline__ bool face_block(const Layout& L, int& bx, int& i) {
  const int gx = face_gx(L), gy = L.nx + 1;
  const int per = (int)(gridDim.x >> 3);
  const int b = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  if (b >= gx * gy) return false;
  band_map(gx, gy, kFaceBand, b, bx, i);
  return true;
}

// A thread owns the three faces at corner (i, j, k) of logical block (bx,
// iplane); threads past the plane's corners return.
#define UF_FACE_POINT(L, bx, iplane)                                 \
  const int i = (iplane);                                            \
  const int p = (bx) * kFaceBlock + threadIdx.x;                     \
  if (p >= ((L).ny + 1) * ((L).nz + 1)) return;                      \
  const int j = p / ((L).nz + 1);                                    \
  const int k = p - j * ((L).nz + 1);

// The same for a kernel of one grid (the logical block from face_block).
#define UF_FACE_THREAD(L)                                            \
  int f_bx, f_by;                                                    \
  if (!face_block((L), f_bx, f_by)) return;                          \
  UF_FACE_POINT(L, f_bx, f_by)

// Each kernel computes the values of the thread's three faces first, with
// every load unconditional (all positions read lie in the padded arrays,
// ghosts included), and only then stores the faces the thread owns; fixed
// boundary normal faces get their Dirichlet value.  Independent loads of
// the three components are then in flight together.
template <int C, class T>
__device__ __forceinline__ void finish_face(const Params<T>& P, T* __restrict__ out, int i, int j, int k, T v) {
  if (!owns_face<C, T>(P.L, i, j, k)) return;
  T val;
  if (face_dirichlet<C>(P, i, j, k, &val)) v = val;
  store_face<C>(out, P, i, j, k, v);
}

}  // namespace uf
