// Momentum stages of the RANS step on the staggered grid (Sec. 3): MacCormack
// semi-Lagrangian advection, explicit (nu + nu_t) diffusion, the porosity drag
// and the pressure-gradient correction of the projection.
//
// Each kernel handles the three face components: a thread owns the faces
// u(i,j,k), v(i,j,k), w(i,j,k) of the cell corner (i,j,k), i in [0, nx],
// (j, k) in [0, ny] x [0, nz], flattened z fastest so that a wavefront
// reads consecutive memory.  Fixed boundary normal faces get their
// Dirichlet value; ghosts are written by store_face.
#include "face_ops.h"

namespace uf {

// ------------------------------------------------------------- advection --
template <int C, class T>
__device__ __forceinline__ T advect_fwd_value(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V,
                                              const T* __restrict__ W, long long o, int i, int j, int k) {
  T vel[3];
  face_velocity<C>(P.L, U, V, W, o, vel);
  const T* q = C == 0 ? U : (C == 1 ? V : W);
  T mn, mx;
  return sample<C, false>(P.L, q, i, j, k, -(vel[0] * P.dth[0]), -(vel[1] * P.dth[1]), -(vel[2] * P.dth[2]), &mn,
                          &mx);
}

template <int C, class T>
__device__ __forceinline__ T advect_corr_value(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V,
                                               const T* __restrict__ W, const T* __restrict__ qhat, long long o, int i,
                                               int j, int k) {
  T vel[3];
  face_velocity<C>(P.L, U, V, W, o, vel);
  const T* q = C == 0 ? U : (C == 1 ? V : W);
  const T di = vel[0] * P.dth[0], dj = vel[1] * P.dth[1], dk = vel[2] * P.dth[2];
  T mn, mx;
  // forward trace again: same value as stored in qhat, plus the sample range
  const T qh = sample<C, true>(P.L, q, i, j, k, -di, -dj, -dk, &mn, &mx);
  T d0, d1;
  const T qc = sample<C, false>(P.L, qhat, i, j, k, di, dj, dk, &d0, &d1);
  const T qt = qh + T(0.5) * (q[o] - qc);
  return nmin(nmax(qt, mn), mx);
}

template <class T>
__global__ __launch_bounds__(kFaceBlock) void k_advect_fwd(Params<T> P, const T* __restrict__ U, const T* __restrict__ V,
                                                           const T* __restrict__ W, T* __restrict__ Uh,
                                                           T* __restrict__ Vh, T* __restrict__ Wh) {
  UF_FACE_THREAD(P.L);
  const long long o = P.L.at(i, j, k);
  const T a0 = advect_fwd_value<0>(P, U, V, W, o, i, j, k);
  const T a1 = advect_fwd_value<1>(P, U, V, W, o, i, j, k);
  const T a2 = advect_fwd_value<2>(P, U, V, W, o, i, j, k);
  finish_face<0>(P, Uh, i, j, k, a0);
  finish_face<1>(P, Vh, i, j, k, a1);
  finish_face<2>(P, Wh, i, j, k, a2);
}

template <class T>
__global__ __launch_bounds__(kFaceBlock) void k_advect_corr(Params<T> P, const T* __restrict__ U, const T* __restrict__ V,
                                                            const T* __restrict__ W, const T* __restrict__ Uh,
                                                            const T* __restrict__ Vh, const T* __restrict__ Wh,
                                                            T* __restrict__ Uo, T* __restrict__ Vo, T* __restrict__ Wo) {
  UF_FACE_THREAD(P.L);
  const long long o = P.L.at(i, j, k);
  const T a0 = advect_corr_value<0>(P, U, V, W, Uh, o, i, j, k);
  const T a1 = advect_corr_value<1>(P, U, V, W, Vh, o, i, j, k);
  const T a2 = advect_corr_value<2>(P, U, V, W, Wh, o, i, j, k);
  finish_face<0>(P, Uo, i, j, k, a0);
  finish_face<1>(P, Vo, i, j, k, a1);
  finish_face<2>(P, Wo, i, j, k, a2);
}

// The advection kernels with 32-bit offsets (arrays below 4 GiB).  The
// predictor gathers the face velocities of the thread's three faces, then
// issues the trilinear loads of all three components at once, then
// evaluates: two memory round trips instead of one per component.
template <class T>
__device__ __forceinline__ void advect_fwd32_faces(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ W, T* __restrict__ Uh, T* __restrict__ Vh, T* __restrict__ Wh, int bx, int ib) {
  UF_FACE_POINT(P.L, bx, ib);
  const Layout& L = P.L;
  const unsigned o = (unsigned)L.at(i, j, k);
  T v0[3], v1[3], v2[3];
  face_velocity32<0>(L, U, V, W, o, v0);
  face_velocity32<1>(L, U, V, W, o, v1);
  face_velocity32<2>(L, U, V, W, o, v2);
  const Tri<T> t0 = tri_corner<0>(L, i, j, k, -(v0[0] * P.dth[0]), -(v0[1] * P.dth[1]), -(v0[2] * P.dth[2]));
  const Tri<T> t1 = tri_corner<1>(L, i, j, k, -(v1[0] * P.dth[0]), -(v1[1] * P.dth[1]), -(v1[2] * P.dth[2]));
  const Tri<T> t2 = tri_corner<2>(L, i, j, k, -(v2[0] * P.dth[0]), -(v2[1] * P.dth[1]), -(v2[2] * P.dth[2]));
  T s0[8], s1[8], s2[8];
  tri_load(U, L, t0.o, s0);
  tri_load(V, L, t1.o, s1);
  tri_load(W, L, t2.o, s2);
  // NaN for a NaN velocity, added rather than selected: a select would let
  // the compiler move the loads under a branch
  const T a0 = tri_eval(t0, s0) + nan_if<T>(any_nan3(v0));
  const T a1 = tri_eval(t1, s1) + nan_if<T>(any_nan3(v1));
  const T a2 = tri_eval(t2, s2) + nan_if<T>(any_nan3(v2));
  finish_face<0>(P, Uh, i, j, k, a0);
  finish_face<1>(P, Vh, i, j, k, a1);
  finish_face<2>(P, Wh, i, j, k, a2);
}

template <class T>
__global__ __launch_bounds__(kFaceBlock) void k_advect_fwd32(Params<T> P, const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ W, T* __restrict__ Uh, T* __restrict__ Vh, T* __restrict__ Wh) {
  int bx, ib;
  if (!face_block(P.L, bx, ib)) return;
  advect_fwd32_faces(P, U, V, W, Uh, Vh, Wh, bx, ib);
}

// The corrector with 32-bit offsets, one component: the forward trace
// again (its value and the range of its eight samples), the reverse trace
// through the traced field, the correction and the clamp.
template <int C, class T>
__device__ __forceinline__ T advect_corr32_value(const Params<T>& P, const T* __restrict__ U,
                                                 const T* __restrict__ V, const T* __restrict__ W,
                                                 const T* __restrict__ qhat, unsigned o, int i, int j, int k) {
  T vel[3];
  face_velocity32<C>(P.L, U, V, W, o, vel);
  const T* q = C == 0 ? U : (C == 1 ? V : W);
  const T di = vel[0] * P.dth[0], dj = vel[1] * P.dth[1], dk = vel[2] * P.dth[2];
  const Tri<T> fw = tri_corner<C>(P.L, i, j, k, -di, -dj, -dk);
  const Tri<T> bw = tri_corner<C>(P.L, i, j, k, di, dj, dk);
  T sf[8], sb[8];
  tri_load(q, P.L, fw.o, sf);
  tri_load(qhat, P.L, bw.o, sb);
  T mn, mx;
  tri_range(sf, mn, mx);
  const T qh = tri_eval(fw, sf);
  const T qc = tri_eval(bw, sb);
  const T qt = qh + T(0.5) * (vel[C] - qc);
  return nmin(nmax(qt, mn), mx) + nan_if<T>(any_nan3(vel));
}

// The corrector of one component comp of the faces of logical block (bx,
// ib).  The kernels give each component blocks of its own: a thread then
// holds one component's samples (57 registers instead of 110 for all three)
// and twice as many wavefronts hide the gathers' latency (879 -> 781 us per
// launch at 512x512x128).
template <class T>
__device__ __forceinline__ void advect_corr32_component(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ W, const T* __restrict__ Uh, const T* __restrict__ Vh, const T* __restrict__ Wh, T* __restrict__ Uo, T* __restrict__ Vo, T* __restrict__ Wo, int comp, int bx, int ib) {
  UF_FACE_POINT(P.L, bx, ib);
  const unsigned o = (unsigned)P.L.at(i, j, k);
  if (comp == 0) {
    const T a = advect_corr32_value<0>(P, U, V, W, Uh, o, i, j, k);
    finish_face<0>(P, Uo, i, j, k, a);
  } else if (comp == 1) {
    const T a = advect_corr32_value<1>(P, U, V, W, Vh, o, i, j, k);
    finish_face<1>(P, Vo, i, j, k, a);
  } else {
    const T a = advect_corr32_value<2>(P, U, V, W, Wh, o, i, j, k);
    finish_face<2>(P, Wo, i, j, k, a);
  }
}

// Single grid, launched on xcd_grid(3 face_gx, nx + 1): the three
// components of a face block are neighbours in the logical order, so they
// run together on one XCD and share the velocity and sample loads in its
// L2 (with the component as a grid dimension of its own each array was
// fetched from HBM three times).
template <class T>
__global__ __launch_bounds__(kFaceBlock) void k_advect_corr32(Params<T> P, const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ W, const T* __restrict__ Uh, const T* __restrict__ Vh, const T* __restrict__ Wh, T* __restrict__ Uo, T* __restrict__ Vo, T* __restrict__ Wo) {
  const int gx = face_gx(P.L), gy = P.L.nx + 1;
  const int per = (int)(gridDim.x >> 3);
  const int e = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  if (e >= 3 * gx * gy) return;
  int bx, ib;
  band_map(gx, gy, kFaceBand, e / 3, bx, ib);
  advect_corr32_component(P, U, V, W, Uh, Vh, Wh, Uo, Vo, Wo, e % 3, bx, ib);
}

// ------------------------------------------------------------- diffusion --
template <int C, class T>
__device__ __forceinline__ T diffuse_value(const Params<T>& P, const T* __restrict__ q, const T* __restrict__ nut,
                                           long long o) {
  const Layout& L = P.L;
  const T qc = q[o];
  const T lap = (q[o + L.SX] - T(2) * qc + q[o - L.SX]) * P.ih2[0] +
                (q[o + L.PZ] - T(2) * qc + q[o - L.PZ]) * P.ih2[1] +
                (q[o + 1] - T(2) * qc + q[o - 1]) * P.ih2[2];
  const T nuf = P.nu + T(0.5) * (nut[o - stride<C>(L)] + nut[o]);
  return qc + P.dt * nuf * lap;
}

template <class T>
__device__ __forceinline__ void diffuse_faces(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ W, const T* __restrict__ NUT, T* __restrict__ Uo, T* __restrict__ Vo, T* __restrict__ Wo, int bx, int ib) {
  UF_FACE_POINT(P.L, bx, ib);
  const long long o = P.L.at(i, j, k);
  const T a0 = diffuse_value<0>(P, U, NUT, o);
  const T a1 = diffuse_value<1>(P, V, NUT, o);
  const T a2 = diffuse_value<2>(P, W, NUT, o);
  finish_face<0>(P, Uo, i, j, k, a0);
  finish_face<1>(P, Vo, i, j, k, a1);
  finish_face<2>(P, Wo, i, j, k, a2);
}

template <class T>
__global__ __launch_bounds__(kFaceBlock) void k_diffuse(Params<T> P, const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ W, const T* __restrict__ NUT, T* __restrict__ Uo, T* __restrict__ Vo, T* __restrict__ Wo) {
  int bx, ib;
  if (!face_block(P.L, bx, ib)) return;
  diffuse_faces(P, U, V, W, NUT, Uo, Vo, Wo, bx, ib);
}

// ------------------------------------------------------------ porosity drag
template <int C, class T>
__device__ __forceinline__ T drag_value(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V,
                                        const T* __restrict__ W, const T* __restrict__ Cc, long long o) {
  T vel[3];
  face_velocity<C>(P.L, U, V, W, o, vel);
  const T speed = sqrt(vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]);
  const T cf = T(0.5) * (Cc[o - stride<C>(P.L)] + Cc[o]);
  const T fac = nmax(T(0), T(1) - P.dt * cf * speed);
  return fac * vel[C];
}

template <class T>
__device__ __forceinline__ void drag_faces(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ W, const T* __restrict__ Cc, T* __restrict__ Uo, T* __restrict__ Vo, T* __restrict__ Wo, int* nf, int bx, int ib) {
  UF_FACE_POINT(P.L, bx, ib);
  const long long o = P.L.at(i, j, k);
  const T a0 = drag_value<0>(P, U, V, W, Cc, o);
  const T a1 = drag_value<1>(P, U, V, W, Cc, o);
  const T a2 = drag_value<2>(P, U, V, W, Cc, o);
  // a NaN/Inf in an owned face raises the state's non-finite flag (every
  // writer stores 1, so the race is benign)
  if ((owns_face<0, T>(P.L, i, j, k) && !isfinite(a0)) || (owns_face<1, T>(P.L, i, j, k) && !isfinite(a1)) ||
      (owns_face<2, T>(P.L, i, j, k) && !isfinite(a2)))
    *nf = 1;
  finish_face<0>(P, Uo, i, j, k, a0);
  finish_face<1>(P, Vo, i, j, k, a1);
  finish_face<2>(P, Wo, i, j, k, a2);
}

template <class T>
__global__ __launch_bounds__(kFaceBlock) void k_drag(Params<T> P, const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ W, const T* __restrict__ Cc, T* __restrict__ Uo, T* __restrict__ Vo, T* __restrict__ Wo, int* nf) {
  int bx, ib;
  if (!face_block(P.L, bx, ib)) return;
  drag_faces(P, U, V, W, Cc, Uo, Vo, Wo, nf, bx, ib);
}

// ------------------------------------------------ projection (velocity part)
template <int C, class T>
__device__ __forceinline__ T project_value(const Params<T>& P, const T* __restrict__ q, const T* __restrict__ p,
                                           long long o) {
  const T grad = (p[o] - p[o - stride<C>(P.L)]) * P.ih[C];
  return q[o] - P.dt_rho * grad;
}

template <class T>
__device__ __forceinline__ void project_faces(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ W, const T* __restrict__ Pp, T* __restrict__ Uo, T* __restrict__ Vo, T* __restrict__ Wo, int bx, int ib) {
  UF_FACE_POINT(P.L, bx, ib);
  const long long o = P.L.at(i, j, k);
  const T a0 = project_value<0>(P, U, Pp, o);
  const T a1 = project_value<1>(P, V, Pp, o);
  const T a2 = project_value<2>(P, W, Pp, o);
  finish_face<0>(P, Uo, i, j, k, a0);
  finish_face<1>(P, Vo, i, j, k, a1);
  finish_face<2>(P, Wo, i, j, k, a2);
}

// gate: when given, the launch does nothing unless *gate is set (a step's
// projection enqueued before the host has read whether the solve ended).
template <class T>
__global__ __launch_bounds__(kFaceBlock) void k_project(Params<T> P, const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ W, const T* __restrict__ Pp, T* __restrict__ Uo, T* __restrict__ Vo, T* __restrict__ Wo, const int* __restrict__ gate) {
  if (gate && !*gate) return;
  int bx, ib;
  if (!face_block(P.L, bx, ib)) return;
  project_faces(P, U, V, W, Pp, Uo, Vo, Wo, bx, ib);
}

// ------------------------------------------------ boundary refresh (in place)
template <int C, class T>
__global__ __launch_bounds__(kFaceBlock) void k_face_bc(Params<T> P, T* __restrict__ q) {
  UF_FACE_THREAD(P.L);
  if (!owns_face<C, T>(P.L, i, j, k)) return;
  T val;
  if (!face_dirichlet<C>(P, i, j, k, &val)) val = q[P.L.at(i, j, k)];
  store_face<C>(q, P, i, j, k, val);
}

// Initial state: the inflow profile on every face (fixed faces keep their
// boundary value).
template <int C, class T>
__global__ __launch_bounds__(kFaceBlock) void k_face_init(Params<T> P, T* __restrict__ q) {
  UF_FACE_THREAD(P.L);
  if (!owns_face<C, T>(P.L, i, j, k)) return;
  T val;
  if (!face_dirichlet<C>(P, i, j, k, &val)) val = inflow_comp(P, C, k);
  store_face<C>(q, P, i, j, k, val);
}

// ------------------------------------------------- several grids at once --
// One launch of a face stage for every case of a batch: the cases' logical
// blocks form one queue (case c owns [start[c], start[c + 1])),
// which a persistent grid walks -- every XCD takes a contiguous share and
// its blocks stride through it -- each block running the stage's per-block
// body with its case's parameters and buffers (read from the case table).
// Sets: sin is read, saux is the predictor's output the corrector reads,
// sout is written.
template <int S, class T>
__global__ __launch_bounds__(kFaceBlock) void k_faces_multi(const MultiCase<T>* __restrict__ mc, CaseStarts cs,
                                                            int band, int sin, int saux, int sout) {
  // the corrector's queue holds three entries (components) per face block
  constexpr int NC = S == MS_ADVECT_CORR ? 3 : 1;
  const int nb = (int)(gridDim.x >> 3);
  const int xcd = (int)(blockIdx.x & 7u), lid = (int)(blockIdx.x >> 3);
  const int total = NC * cs.start[cs.n];
  const int share = (total + 7) >> 3;
  const int lo = xcd * share, hi = min(total, lo + share);
  for (int le = lo + lid; le < hi; le += nb) {
    const int lb = le / NC;
    const int c = find_case(cs, lb);
    const MultiCase<T>& A = mc[c];
    int bx, ib;
    band_map(face_gx(A.P.L), A.P.L.nx + 1, band, lb - cs.start[c], bx, ib);
    T* const* qi = A.q[sin];
    T* const* qo = A.q[sout];
    if (S == MS_ADVECT_FWD) {
      advect_fwd32_faces(A.P, qi[0], qi[1], qi[2], qo[0], qo[1], qo[2], bx, ib);
    } else if (S == MS_ADVECT_CORR) {
      T* const* qa = A.q[saux];
      advect_corr32_component(A.P, qi[0], qi[1], qi[2], qa[0], qa[1], qa[2], qo[0], qo[1], qo[2], le - NC * lb, bx,
                              ib);
    } else if (S == MS_DIFFUSE) {
      diffuse_faces(A.P, qi[0], qi[1], qi[2], A.nut, qo[0], qo[1], qo[2], bx, ib);
    } else if (S == MS_DRAG) {
      drag_faces(A.P, qi[0], qi[1], qi[2], A.cc, qo[0], qo[1], qo[2], A.nf, bx, ib);
    } else {
      project_faces(A.P, qi[0], qi[1], qi[2], A.x, qo[0], qo[1], qo[2], bx, ib);
    }
  }
}

template <class T>
void launch_faces_multi(int stage, const MultiCase<T>* mc, const CaseStarts& cs, int band, int blocks, int sin,
                        int saux, int sout, hipStream_t stream) {
  const dim3 grid((unsigned)blocks), blk(kFaceBlock);
  switch (stage) {
    case MS_ADVECT_FWD:
      hipLaunchKernelGGL((k_faces_multi<MS_ADVECT_FWD, T>), grid, blk, 0, stream, mc, cs, band, sin, saux, sout);
      break;
    case MS_ADVECT_CORR:
      hipLaunchKernelGGL((k_faces_multi<MS_ADVECT_CORR, T>), grid, blk, 0, stream, mc, cs, band, sin, saux, sout);
      break;
    case MS_DIFFUSE:
      hipLaunchKernelGGL((k_faces_multi<MS_DIFFUSE, T>), grid, blk, 0, stream, mc, cs, band, sin, saux, sout);
      break;
    case MS_DRAG:
      hipLaunchKernelGGL((k_faces_multi<MS_DRAG, T>), grid, blk, 0, stream, mc, cs, band, sin, saux, sout);
      break;
    default:
      hipLaunchKernelGGL((k_faces_multi<MS_PROJECT, T>), grid, blk, 0, stream, mc, cs, band, sin, saux, sout);
      break;
  }
}

// ----------------------------------------------------------------- launchers
static inline dim3 face_grid(const Layout& L) { return xcd_grid(face_gx(L), L.nx + 1); }

template <class T>
void launch_advect(Grid& g, const Params<T>& P, void* const Qin[3], void* const Qhat[3], void* const Qout[3]) {
  const dim3 grid = face_grid(P.L);
  if (offsets_fit_32(P.L, sizeof(T))) {
    {
      TimedLaunch tl(g, UF_TK_ADVECT_FWD);
      launch_k(g, k_advect_fwd32<T>, grid, dim3(kFaceBlock), P, (const T*)Qin[0], (const T*)Qin[1],
               (const T*)Qin[2], (T*)Qhat[0], (T*)Qhat[1], (T*)Qhat[2]);
    }
    TimedLaunch tl(g, UF_TK_ADVECT_CORR);
    launch_k(g, k_advect_corr32<T>, xcd_grid(3 * face_gx(P.L), P.L.nx + 1), dim3(kFaceBlock), P, (const T*)Qin[0], (const T*)Qin[1],
             (const T*)Qin[2], (const T*)Qhat[0], (const T*)Qhat[1], (const T*)Qhat[2], (T*)Qout[0], (T*)Qout[1],
             (T*)Qout[2]);
    return;
  }
  {
    TimedLaunch tl(g, UF_TK_ADVECT_FWD);
    launch_k(g, k_advect_fwd<T>, grid, dim3(kFaceBlock), P, (const T*)Qin[0], (const T*)Qin[1],
                       (const T*)Qin[2], (T*)Qhat[0], (T*)Qhat[1], (T*)Qhat[2]);
  }
  TimedLaunch tl(g, UF_TK_ADVECT_CORR);
  launch_k(g, k_advect_corr<T>, grid, dim3(kFaceBlock), P, (const T*)Qin[0], (const T*)Qin[1],
                     (const T*)Qin[2], (const T*)Qhat[0], (const T*)Qhat[1], (const T*)Qhat[2], (T*)Qout[0],
                     (T*)Qout[1], (T*)Qout[2]);
}

template <class T>
void launch_diffuse(Grid& g, const Params<T>& P, void* const Qin[3], void* const Qout[3]) {
  TimedLaunch tl(g, UF_TK_DIFFUSE);
  launch_k(g, k_diffuse<T>, face_grid(P.L), dim3(kFaceBlock), P, (const T*)Qin[0],
                     (const T*)Qin[1], (const T*)Qin[2], (const T*)g.NUT, (T*)Qout[0], (T*)Qout[1], (T*)Qout[2]);
}

template <class T>
void launch_drag(Grid& g, const Params<T>& P, void* const Qin[3], void* const Qout[3]) {
  TimedLaunch tl(g, UF_TK_DRAG);
  launch_k(g, k_drag<T>, face_grid(P.L), dim3(kFaceBlock), P, (const T*)Qin[0], (const T*)Qin[1],
                     (const T*)Qin[2], (const T*)g.C, (T*)Qout[0], (T*)Qout[1], (T*)Qout[2], nf_word(g));
}

template <class T>
void launch_project(Grid& g, const Params<T>& P, void* const Qin[3], void* const Qout[3], const int* gate) {
  TimedLaunch tl(g, UF_TK_PROJECT);
  launch_k(g, k_project<T>, face_grid(P.L), dim3(kFaceBlock), P, (const T*)Qin[0],
                     (const T*)Qin[1], (const T*)Qin[2], (const T*)g.X, (T*)Qout[0], (T*)Qout[1], (T*)Qout[2], gate);
}

template <class T>
void launch_face_bc(Grid& g, const Params<T>& P, void* q, int comp) {
  const dim3 grid = face_grid(P.L);
  if (comp == 0) hipLaunchKernelGGL((k_face_bc<0, T>), grid, dim3(kFaceBlock), 0, g.stream, P, (T*)q);
  if (comp == 1) hipLaunchKernelGGL((k_face_bc<1, T>), grid, dim3(kFaceBlock), 0, g.stream, P, (T*)q);
  if (comp == 2) hipLaunchKernelGGL((k_face_bc<2, T>), grid, dim3(kFaceBlock), 0, g.stream, P, (T*)q);
}

template <class T>
void launch_face_init(Grid& g, const Params<T>& P, void* const Q[3]) {
  const dim3 grid = face_grid(P.L);
  hipLaunchKernelGGL((k_face_init<0, T>), grid, dim3(kFaceBlock), 0, g.stream, P, (T*)Q[0]);
  hipLaunchKernelGGL((k_face_init<1, T>), grid, dim3(kFaceBlock), 0, g.stream, P, (T*)Q[1]);
  hipLaunchKernelGGL((k_face_init<2, T>), grid, dim3(kFaceBlock), 0, g.stream, P, (T*)Q[2]);
}

#define UF_INST(T)                                                                                   \
  template void launch_advect<T>(Grid&, const Params<T>&, void* const[3], void* const[3], void* const[3]); \
  template void launch_diffuse<T>(Grid&, const Params<T>&, void* const[3], void* const[3]);          \
  template void launch_drag<T>(Grid&, const Params<T>&, void* const[3], void* const[3]);             \
  template void launch_project<T>(Grid&, const Params<T>&, void* const[3], void* const[3], const int*); \
  template void launch_face_bc<T>(Grid&, const Params<T>&, void*, int);                             \
  template void launch_face_init<T>(Grid&, const Params<T>&, void* const[3]);                      \
  template void launch_faces_multi<T>(int, const MultiCase<T>*, const CaseStarts&, int, int, int, int, int, hipStream_t);
UF_INST(float)
UF_INST(double)
#undef UF_INST

}  // namespace uf
