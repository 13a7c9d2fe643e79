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

// Trilinear interpolation of component C's padded array at continuous
// (unpadded) index (fi, fj, fk), positions clamped to the padded extent.
// Optionally returns the min and max of the eight samples.
template <int C, bool MINMAX, class T>
__device__ __forceinline__ T sample(const Layout& L, const T* __restrict__ q, T fi, T fj, T fk, T* mn, T* mx) {
  int ext[3];
  face_ext<C>(L, ext);
  // a NaN position (NaN velocity) yields NaN; the index clamp below keeps
  // every access inside the padded array in any case
  const bool nan_pos = fi != fi || fj != fj || fk != fk;
  fi = fmin(fmax(fi, T(-1)), T(ext[0]));
  fj = fmin(fmax(fj, T(-1)), T(ext[1]));
  fk = fmin(fmax(fk, T(-1)), T(ext[2]));
  const T i0f = fmin(floor(fi), T(ext[0] - 1));
  const T j0f = fmin(floor(fj), T(ext[1] - 1));
  const T k0f = fmin(floor(fk), T(ext[2] - 1));
  const T ti = fi - i0f, tj = fj - j0f, tk = fk - k0f;
  const long long o = L.at((int)i0f, (int)j0f, (int)k0f);
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
  const T val = c0 + tk * (c1 - c0);
  return nan_pos ? fi + fj + fk : val;
}

__host__ __device__ inline int face_gx(const Layout& L) { return ((L.ny + 1) * (L.nz + 1) + kFaceBlock - 1) / kFaceBlock; }

// A thread owns the three faces at corner (i, j, k); logical block (bx, i).
#define UF_FACE_THREAD(L)                                            \
  int f_bx, f_by;                                                    \
  if (!xcd_block(face_gx(L), (L).nx + 1, f_bx, f_by)) return;        \
  const int i = f_by;                                                \
  const int p = f_bx * kFaceBlock + threadIdx.x;                     \
  if (p >= ((L).ny + 1) * ((L).nz + 1)) return;                      \
  const int j = p / ((L).nz + 1);                                    \
  const int k = p - j * ((L).nz + 1);

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
