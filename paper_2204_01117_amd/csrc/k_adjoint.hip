// Reverse (discrete adjoint) of the momentum stages of one step (Sec. 3),
// for gradients of a design objective (Sec. 4) with respect to the state
// and the porosity.  Each kernel is the transpose of the forward kernel's
// Jacobian at the recomputed forward state, evaluated in the forward's own
// precision:
//
//   * projection: the step's projection is its own transpose (b = -(rho/dt)
//     div u*, A p = b, u = u* - (dt/rho) grad p with A symmetric and div =
//     -grad^T), so its reverse runs the forward solve and projection on the
//     adjoint with homogeneous boundary values (launched by the host);
//   * drag and MacCormack advection: the transpose of the trilinear samples
//     and of the drag coefficient scatters with atomic adds (their order is
//     not fixed, so the FP32 result may differ in the last bits between
//     runs); the velocity-vector part is stored per face and gathered;
//   * diffusion: the transpose is a gather over every padded position;
//   * ghosts: every ghost is written from its nearest interior face by the
//     side rules (copy, negation at a no-slip wall, a constant at an
//     inlet), so its adjoint is folded back into that face with the sign of
//     the rule; fixed boundary faces hold constants and carry no adjoint.
//
// An adjoint array holds the derivative of the objective with respect to
// the interior faces a stage computes; positions outside that set are read
// as zero (adj_in).
#include "face_ops.h"
#include "turb_model.h"

namespace uf {

static inline dim3 adj_face_grid(const Layout& L) { return xcd_grid(face_gx(L), L.nx + 1); }

template <class T>
__device__ __forceinline__ void add_to(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

// Adjoint of face (i,j,k) of component C: zero unless it is an interior
// face whose value the stage computes (inside the face range, not fixed).
template <int C, class T>
__device__ __forceinline__ T adj_in(const Params<T>& P, const T* __restrict__ a, int i, int j, int k) {
  int ext[3];
  face_ext<C>(P.L, ext);
  if (i < 0 || j < 0 || k < 0 || i >= ext[0] || j >= ext[1] || k >= ext[2]) return T(0);
  T v;
  if (face_dirichlet<C>(P, i, j, k, &v)) return T(0);
  return a[P.L.at(i, j, k)];
}

// Reverse of face_velocity in two parts.  A reverse kernel stores, per face
// of component C, the adjoint vb[cp] of each velocity component the face
// saw (VelAdj, nine padded arrays, written at every position of the face
// thread range); k_vel_gather then adds to each face of component cp its own
// entry and a quarter of the entries of the four faces of each other
// component that averaged it.  Plain stores and a gather instead of nine
// atomic adds per face and component.
template <class T>
struct VelAdj {
  T* a[3][3];   // a[C][cp]: adjoint of velocity component cp seen at faces of component C
};

template <int C, class T>
__device__ __forceinline__ void vel_store(const VelAdj<T>& V, long long o, const T vb[3], bool accumulate) {
#pragma unroll
  for (int cp = 0; cp < 3; ++cp) {
    T* q = V.a[C][cp] + o;
    *q = accumulate ? *q + vb[cp] : vb[cp];
  }
}

// Inside the face thread range (where VelAdj entries are written)?
__device__ __forceinline__ bool in_face_range(const Layout& L, int i, int j, int k) {
  return i >= 0 && j >= 0 && k >= 0 && i <= L.nx && j <= L.ny && k <= L.nz;
}

template <int CP, class T>
__device__ __forceinline__ T vel_gather_value(const Layout& L, const VelAdj<T>& V, int i, int j, int k) {
  T s = T(0);
  if (in_face_range(L, i, j, k)) s += V.a[CP][CP][L.at(i, j, k)];
  const int e2[3] = {CP == 0, CP == 1, CP == 2};
#pragma unroll
  for (int C = 0; C < 3; ++C) {
    if (C == CP) continue;
    const int ec[3] = {C == 0, C == 1, C == 2};
    // faces o of component C whose average of component CP reads (i,j,k):
    // o = t + e_C, t + e_C - e_CP, t, t - e_CP
    const int oi[4] = {i + ec[0], i + ec[0] - e2[0], i, i - e2[0]};
    const int oj[4] = {j + ec[1], j + ec[1] - e2[1], j, j - e2[1]};
    const int ok[4] = {k + ec[2], k + ec[2] - e2[2], k, k - e2[2]};
    T q = T(0);
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (in_face_range(L, oi[m], oj[m], ok[m])) q += V.a[C][CP][L.at(oi[m], oj[m], ok[m])];
    s += T(0.25) * q;
  }
  return s;
}

// One thread per padded position: G_cp += the gathered velocity adjoint.
template <class T>
__global__ __launch_bounds__(256) void k_vel_gather(Params<T> P, VelAdj<T> V, T* __restrict__ G0,
                                                    T* __restrict__ G1, T* __restrict__ G2, long long nelem) {
  const Layout& L = P.L;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nelem;
       p += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(p / L.SX) - 1;
    const long long r = p - (long long)(i + 1) * L.SX;
    const int j = (int)(r / L.PZ) - 1;
    const int k = (int)(r - (long long)(j + 1) * L.PZ) - 1;
    if (i > L.nx + 1 || j > L.ny + 1 || k > L.nz + 1) continue;
    G0[p] += vel_gather_value<0>(L, V, i, j, k);
    G1[p] += vel_gather_value<1>(L, V, i, j, k);
    G2[p] += vel_gather_value<2>(L, V, i, j, k);
  }
}

// Cell and fractions of a trace position (i + si, j + sj, k + sk), clamped
// exactly as in sample().
template <int C, class T>
struct SamplePos {
  long long o;      // offset of the lower corner
  T t[3];           // fractions
  bool live[3];     // the position was not clamped along this axis
  __device__ __forceinline__ SamplePos(const Layout& L, int i, int j, int k, T si, T sj, T sk) {
    AxisPos<T> a[3];
    trace_pos<C>(L, i, j, k, si, sj, sk, a);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      t[q] = a[q].t;
      live[q] = a[q].live;
    }
    o = L.at(a[0].c, a[1].c, a[2].c);
  }
};

// Offset of the smallest (want_max false) or largest of the eight samples
// around a position (the first one in corner order on a tie).
template <int C, class T>
__device__ __forceinline__ long long sample_extreme(const Layout& L, const T* __restrict__ q, int i, int j, int k,
                                                    T si, T sj, T sk, bool want_max) {
  const SamplePos<C, T> s(L, i, j, k, si, sj, sk);
  const long long offs[8] = {0, L.SX, L.PZ, L.SX + L.PZ, 1, L.SX + 1, L.PZ + 1, L.SX + L.PZ + 1};
  long long best = s.o;
  T bv = q[s.o];
#pragma unroll
  for (int n = 1; n < 8; ++n) {
    const T v = q[s.o + offs[n]];
    if (want_max ? v > bv : v < bv) {
      bv = v;
      best = s.o + offs[n];
    }
  }
  return best;
}

// ------------------------------------------------------------- advection --
// A trilinear scatter of one lane, made by all lanes of the wavefront
// together.  Lanes are consecutive along z, so lane L's upper layer of
// samples (z index k0 + 1) is usually lane L+1's lower layer: when their
// corners are one apart, L+1 adds L's four upper weights to its own lower
// ones (one shuffle each) and L skips those atomics -- four atomic adds per
// sample instead of eight.  Both lanes decide from the same two corners.
template <class T>
struct Scatter8 {
  long long o;   // lower corner
  T w[8];        // weights times the adjoint, corner order 000 100 010 110 001 101 011 111
  bool on;
};

template <int C, class T>
__device__ __forceinline__ void sample_weights(const Layout& L, const T* __restrict__ q, int i, int j, int k, T si,
                                               T sj, T sk, T wbar, T grad[3], Scatter8<T>& sc) {
  const SamplePos<C, T> s(L, i, j, k, si, sj, sk);
  const long long o = s.o, SX = L.SX, PZ = L.PZ;
  const T ti = s.t[0], tj = s.t[1], tk = s.t[2];
  const T s000 = q[o], s100 = q[o + SX], s010 = q[o + PZ], s110 = q[o + SX + PZ];
  const T s001 = q[o + 1], s101 = q[o + SX + 1], s011 = q[o + PZ + 1], s111 = q[o + SX + PZ + 1];
  const T ui = T(1) - ti, uj = T(1) - tj, uk = T(1) - tk;
  grad[0] = s.live[0] ? uj * uk * (s100 - s000) + tj * uk * (s110 - s010) + uj * tk * (s101 - s001) +
                            tj * tk * (s111 - s011)
                      : T(0);
  grad[1] = s.live[1] ? ui * uk * (s010 - s000) + ti * uk * (s110 - s100) + ui * tk * (s011 - s001) +
                            ti * tk * (s111 - s101)
                      : T(0);
  grad[2] = s.live[2] ? ui * uj * (s001 - s000) + ti * uj * (s101 - s100) + ui * tj * (s011 - s010) +
                            ti * tj * (s111 - s110)
                      : T(0);
  sc.o = o;
  sc.on = wbar != T(0);
  sc.w[0] = wbar * ui * uj * uk;
  sc.w[1] = wbar * ti * uj * uk;
  sc.w[2] = wbar * ui * tj * uk;
  sc.w[3] = wbar * ti * tj * uk;
  sc.w[4] = wbar * ui * uj * tk;
  sc.w[5] = wbar * ti * uj * tk;
  sc.w[6] = wbar * ui * tj * tk;
  sc.w[7] = wbar * ti * tj * tk;
}

// Called by every lane of the wavefront (convergent).
template <class T>
__device__ __forceinline__ void paired_scatter(T* __restrict__ qbar, const Layout& L, const Scatter8<T>& sc) {
  const int lane = (int)(threadIdx.x & 63u);
  const long long mine = sc.on ? sc.o : -2LL;   // corners are >= 0: -2 never matches
  const long long prev = __shfl_up(mine, 1u);
  const long long next = __shfl_down(mine, 1u);
  T r[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = __shfl_up(sc.w[4 + q], 1u);
  if (!sc.on) return;
  const bool take = lane > 0 && prev >= 0 && prev + 1 == sc.o;
  const bool give = lane < 63 && next == sc.o + 1;
  const long long SX = L.SX, PZ = L.PZ;
  const long long lo[4] = {0, SX, PZ, SX + PZ};
#pragma unroll
  for (int q = 0; q < 4; ++q) add_to(qbar + sc.o + lo[q], take ? sc.w[q] + r[q] : sc.w[q]);
  if (!give) {
#pragma unroll
    for (int q = 0; q < 4; ++q) add_to(qbar + sc.o + lo[q] + 1, sc.w[4 + q]);
  }
}

// Reverse of the corrector: out = clamp(qh + (q - qc)/2, min, max) with
// qh sampled from q at the back-traced point and qc from qhat at the
// forward-traced point.  A clamped output is one of the eight samples of q.
// The two trilinear scatters are returned (sb into q's adjoint, sf into
// qhat's); the face's own half goes into vb[C] (gathered back to it).
template <int C, class T>
__device__ __forceinline__ void advect_corr_adj(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V,
                                                const T* __restrict__ W, const T* __restrict__ qhat, T ob,
                                                T* __restrict__ Gq, long long o, int i, int j, int k, T vb[3],
                                                Scatter8<T>& sb, Scatter8<T>& sf) {
  vb[0] = vb[1] = vb[2] = T(0);
  sb = Scatter8<T>();
  sf = Scatter8<T>();
  if (ob == T(0)) return;
  T vel[3];
  face_velocity<C>(P.L, U, V, W, o, vel);
  const T* q = C == 0 ? U : (C == 1 ? V : W);
  const T di = vel[0] * P.dth[0], dj = vel[1] * P.dth[1], dk = vel[2] * P.dth[2];
  T mn, mx, d0, d1;
  const T qh = sample<C, true>(P.L, q, i, j, k, -di, -dj, -dk, &mn, &mx);
  const T qc = sample<C, false>(P.L, qhat, i, j, k, di, dj, dk, &d0, &d1);
  const T qt = qh + T(0.5) * (q[o] - qc);
  if (qt < mn || qt > mx) {
    add_to(Gq + sample_extreme<C>(P.L, q, i, j, k, -di, -dj, -dk, qt > mx), ob);
    return;
  }
  T gb[3], gf[3];
  sample_weights<C>(P.L, q, i, j, k, -di, -dj, -dk, ob, gb, sb);
  sample_weights<C>(P.L, qhat, i, j, k, di, dj, dk, T(-0.5) * ob, gf, sf);
  vb[0] = -ob * P.dth[0] * (gb[0] + T(0.5) * gf[0]);
  vb[1] = -ob * P.dth[1] * (gb[1] + T(0.5) * gf[1]);
  vb[2] = -ob * P.dth[2] * (gb[2] + T(0.5) * gf[2]);
  vb[C] += T(0.5) * ob;
}

// Reverse of the predictor: qhat = q sampled at the back-traced point.
template <int C, class T>
__device__ __forceinline__ void advect_fwd_adj(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V,
                                               const T* __restrict__ W, T ob, long long o, int i, int j, int k,
                                               T vb[3], Scatter8<T>& sb) {
  vb[0] = vb[1] = vb[2] = T(0);
  sb = Scatter8<T>();
  if (ob == T(0)) return;
  T vel[3];
  face_velocity<C>(P.L, U, V, W, o, vel);
  const T* q = C == 0 ? U : (C == 1 ? V : W);
  T g[3];
  sample_weights<C>(P.L, q, i, j, k, -(vel[0] * P.dth[0]), -(vel[1] * P.dth[1]), -(vel[2] * P.dth[2]), ob, g, sb);
  vb[0] = -ob * P.dth[0] * g[0];
  vb[1] = -ob * P.dth[1] * g[1];
  vb[2] = -ob * P.dth[2] * g[2];
}

// The face-thread mapping without the early exit of lanes past the last
// corner (the paired scatter needs every lane of the wavefront): such lanes
// carry no adjoint and write nothing.
#define UF_FACE_THREAD_ALL(L)                                        \
  int f_bx, f_by;                                                    \
  if (!face_block((L), f_bx, f_by)) return;                          \
  const int i = f_by;                                                \
  const int p_raw = f_bx * kFaceBlock + threadIdx.x;                 \
  const bool lane_valid = p_raw < ((L).ny + 1) * ((L).nz + 1);       \
  const int p = lane_valid ? p_raw : 0;                              \
  const int j = p / ((L).nz + 1);                                    \
  const int k = p - j * ((L).nz + 1);

template <class T>
__global__ __launch_bounds__(kFaceBlock) void k_advect_corr_adj(Params<T> P, const T* __restrict__ U,
                                                                const T* __restrict__ V, const T* __restrict__ W,
                                                                const T* __restrict__ Uh, const T* __restrict__ Vh,
                                                                const T* __restrict__ Wh, const T* __restrict__ A0,
                                                                const T* __restrict__ A1, const T* __restrict__ A2,
                                                                T* __restrict__ GU, T* __restrict__ GV,
                                                                T* __restrict__ GW, T* __restrict__ HU,
                                                                T* __restrict__ HV, T* __restrict__ HW,
                                                                VelAdj<T> VA) {
  UF_FACE_THREAD_ALL(P.L);
  const long long o = P.L.at(i, j, k);
  T vb[3];
  Scatter8<T> sb, sf;
  advect_corr_adj<0>(P, U, V, W, Uh, lane_valid ? adj_in<0>(P, A0, i, j, k) : T(0), GU, o, i, j, k, vb, sb, sf);
  if (lane_valid) vel_store<0>(VA, o, vb, false);
  paired_scatter(GU, P.L, sb);
  paired_scatter(HU, P.L, sf);
  advect_corr_adj<1>(P, U, V, W, Vh, lane_valid ? adj_in<1>(P, A1, i, j, k) : T(0), GV, o, i, j, k, vb, sb, sf);
  if (lane_valid) vel_store<1>(VA, o, vb, false);
  paired_scatter(GV, P.L, sb);
  paired_scatter(HV, P.L, sf);
  advect_corr_adj<2>(P, U, V, W, Wh, lane_valid ? adj_in<2>(P, A2, i, j, k) : T(0), GW, o, i, j, k, vb, sb, sf);
  if (lane_valid) vel_store<2>(VA, o, vb, false);
  paired_scatter(GW, P.L, sb);
  paired_scatter(HW, P.L, sf);
}

template <class T>
__global__ __launch_bounds__(kFaceBlock) void k_advect_fwd_adj(Params<T> P, const T* __restrict__ U,
                                                               const T* __restrict__ V, const T* __restrict__ W,
                                                               const T* __restrict__ H0, const T* __restrict__ H1,
                                                               const T* __restrict__ H2, T* __restrict__ GU,
                                                               T* __restrict__ GV, T* __restrict__ GW,
                                                               VelAdj<T> VA) {
  UF_FACE_THREAD_ALL(P.L);
  const long long o = P.L.at(i, j, k);
  T vb[3];
  Scatter8<T> sb;
  advect_fwd_adj<0>(P, U, V, W, lane_valid ? adj_in<0>(P, H0, i, j, k) : T(0), o, i, j, k, vb, sb);
  if (lane_valid) vel_store<0>(VA, o, vb, true);
  paired_scatter(GU, P.L, sb);
  advect_fwd_adj<1>(P, U, V, W, lane_valid ? adj_in<1>(P, H1, i, j, k) : T(0), o, i, j, k, vb, sb);
  if (lane_valid) vel_store<1>(VA, o, vb, true);
  paired_scatter(GV, P.L, sb);
  advect_fwd_adj<2>(P, U, V, W, lane_valid ? adj_in<2>(P, H2, i, j, k) : T(0), o, i, j, k, vb, sb);
  if (lane_valid) vel_store<2>(VA, o, vb, true);
  paired_scatter(GW, P.L, sb);
}

// ------------------------------------------------------------- diffusion --
template <int C, class T>
__device__ __forceinline__ T face_nu(const Params<T>& P, const T* __restrict__ nut, long long o) {
  return P.nu + T(0.5) * (nut[o - stride<C>(P.L)] + nut[o]);
}

// Transpose of out = q + dt nu_f lap(q) at one padded position (interior
// or ghost) of component C: the position's own row plus the rows of its
// six neighbours.
template <int C, class T>
__device__ __forceinline__ T diffuse_adj_value(const Params<T>& P, const T* __restrict__ a, const T* __restrict__ nut,
                                               int i, int j, int k) {
  const Layout& L = P.L;
  T s = T(0);
  const T self = adj_in<C>(P, a, i, j, k);
  if (self != T(0))
    s += self * (T(1) - T(2) * P.dt * face_nu<C>(P, nut, L.at(i, j, k)) * (P.ih2[0] + P.ih2[1] + P.ih2[2]));
  const int d[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
    for (int sg = -1; sg <= 1; sg += 2) {
      const int ni = i + sg * d[ax][0], nj = j + sg * d[ax][1], nk = k + sg * d[ax][2];
      const T an = adj_in<C>(P, a, ni, nj, nk);
      if (an != T(0)) s += an * P.dt * face_nu<C>(P, nut, L.at(ni, nj, nk)) * P.ih2[ax];
    }
  }
  return s;
}

// One thread per padded position; every position of the three outputs is
// written (zero outside [-1, extent] of the component).
template <class T>
__global__ __launch_bounds__(256) void k_diffuse_adj(Params<T> P, const T* __restrict__ A0, const T* __restrict__ A1,
                                                     const T* __restrict__ A2, const T* __restrict__ NUT,
                                                     T* __restrict__ G0, T* __restrict__ G1, T* __restrict__ G2,
                                                     long long nelem) {
  const Layout& L = P.L;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nelem;
       p += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(p / L.SX) - 1;
    const long long r = p - (long long)(i + 1) * L.SX;
    const int j = (int)(r / L.PZ) - 1;
    const int k = (int)(r - (long long)(j + 1) * L.PZ) - 1;
    const bool in_x = i <= L.nx, in_y = j <= L.ny, in_z = k <= L.nz;   // lower bound -1 always holds
    // component C reaches index extent along its own axis (extent + 1 = n + 1 for the normal axis)
    const bool r0 = (i <= L.nx + 1) && in_y && in_z;
    const bool r1 = in_x && (j <= L.ny + 1) && in_z;
    const bool r2 = in_x && in_y && (k <= L.nz + 1);
    G0[p] = r0 ? diffuse_adj_value<0>(P, A0, NUT, i, j, k) : T(0);
    G1[p] = r1 ? diffuse_adj_value<1>(P, A1, NUT, i, j, k) : T(0);
    G2[p] = r2 ? diffuse_adj_value<2>(P, A2, NUT, i, j, k) : T(0);
  }
}

// ------------------------------------------------------------ porosity drag
// Reverse of out = max(0, 1 - dt c_f |V|) V_C: the velocity part through
// face_velocity and the drag-coefficient part, half to each adjacent cell.
template <int C, class T>
__device__ __forceinline__ void drag_adj(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V,
                                         const T* __restrict__ W, const T* __restrict__ Cc, T ob,
                                         T* __restrict__ Cbar, long long o, T vb[3]) {
  vb[0] = vb[1] = vb[2] = T(0);
  if (ob == T(0)) return;
  T vel[3];
  face_velocity<C>(P.L, U, V, W, o, vel);
  const T speed = sqrt(vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]);
  const T cf = T(0.5) * (Cc[o - stride<C>(P.L)] + Cc[o]);
  const T fac = T(1) - P.dt * cf * speed;
  if (!(fac > T(0))) return;   // the face is stopped: no dependence on either input
  const T g = speed > T(0) ? P.dt * cf * vel[C] / speed : T(0);
  vb[0] = -ob * g * vel[0];
  vb[1] = -ob * g * vel[1];
  vb[2] = -ob * g * vel[2];
  vb[C] += ob * fac;
  const T cb = T(-0.5) * ob * P.dt * speed * vel[C];
  if (cb != T(0)) {
    add_to(Cbar + o - stride<C>(P.L), cb);
    add_to(Cbar + o, cb);
  }
}

template <class T>
__global__ __launch_bounds__(kFaceBlock) void k_drag_adj(Params<T> P, const T* __restrict__ U, const T* __restrict__ V,
                                                         const T* __restrict__ W, const T* __restrict__ Cc,
                                                         const T* __restrict__ A0, const T* __restrict__ A1,
                                                         const T* __restrict__ A2, T* __restrict__ Cbar,
                                                         VelAdj<T> VA) {
  UF_FACE_THREAD(P.L);
  const long long o = P.L.at(i, j, k);
  T vb[3];
  drag_adj<0>(P, U, V, W, Cc, adj_in<0>(P, A0, i, j, k), Cbar, o, vb);
  vel_store<0>(VA, o, vb, false);
  drag_adj<1>(P, U, V, W, Cc, adj_in<1>(P, A1, i, j, k), Cbar, o, vb);
  vel_store<1>(VA, o, vb, false);
  drag_adj<2>(P, U, V, W, Cc, adj_in<2>(P, A2, i, j, k), Cbar, o, vb);
  vel_store<2>(VA, o, vb, false);
}

// ---------------------------------------------------------------- ghosts --
// Sign with which the ghost across side (a, hi) of component c follows its
// neighbour (see face_rule): +1 for a copy, -1 at a no-slip wall, 0 where it
// is the inflow constant.
template <class T>
__device__ __forceinline__ T rule_sign(const Params<T>& P, int c, int a, int hi) {
  if (a == c) return T(1);
  const int kind = P.bc[2 * a + hi];
  if (kind == INLET) return T(0);
  if (kind == WALL) return T(-1);
  return T(1);
}

// Reverse of store_face for face (i,j,k) of component C: the adjoint held
// at each ghost written from this face is added to it with the rule's sign
// and the ghost cleared; a fixed face ends with zero.
template <int C, class T>
__device__ __forceinline__ void fold_face(T* __restrict__ q, const Params<T>& P, int i, int j, int k) {
  const Layout& L = P.L;
  const long long o = L.at(i, j, k);
  int ext[3];
  face_ext<C>(L, ext);
  const bool lo0 = i == 0, hi0 = i == ext[0] - 1;
  const bool lo1 = j == 0, hi1 = j == ext[1] - 1;
  const bool lo2 = k == 0, hi2 = k == ext[2] - 1;
  // an interior face has no ghost and is never fixed: nothing to do
  if (!(lo0 || hi0 || lo1 || hi1 || lo2 || hi2)) return;
  T acc = q[o];
  auto take = [&](long long gpos, T s) {
    acc += s * q[gpos];
    q[gpos] = T(0);
  };
  if (lo2) take(o - 1, rule_sign(P, C, 2, 0));
  if (hi2) take(o + 1, rule_sign(P, C, 2, 1));
  if (lo1) take(o - L.PZ, rule_sign(P, C, 1, 0));
  if (hi1) take(o + L.PZ, rule_sign(P, C, 1, 1));
  if (lo0) take(o - L.SX, rule_sign(P, C, 0, 0));
  if (hi0) take(o + L.SX, rule_sign(P, C, 0, 1));
  if (int(lo0 | hi0) + int(lo1 | hi1) + int(lo2 | hi2) >= 2) {
    for (int ox = -1; ox <= 1; ++ox) {
      if ((ox == -1 && !lo0) || (ox == 1 && !hi0)) continue;
      for (int oy = -1; oy <= 1; ++oy) {
        if ((oy == -1 && !lo1) || (oy == 1 && !hi1)) continue;
        for (int oz = -1; oz <= 1; ++oz) {
          if ((oz == -1 && !lo2) || (oz == 1 && !hi2)) continue;
          if (int(ox != 0) + int(oy != 0) + int(oz != 0) < 2) continue;
          T s = T(1);
          if (ox) s *= rule_sign(P, C, 0, ox > 0);
          if (oy) s *= rule_sign(P, C, 1, oy > 0);
          if (oz) s *= rule_sign(P, C, 2, oz > 0);
          take(L.at(i + ox, j + oy, k + oz), s);
        }
      }
    }
  }
  T fixed;
  if (face_dirichlet<C>(P, i, j, k, &fixed)) acc = T(0);
  q[o] = acc;
}

template <class T>
__global__ __launch_bounds__(kFaceBlock) void k_fold(Params<T> P, T* __restrict__ Q0, T* __restrict__ Q1,
                                                     T* __restrict__ Q2) {
  UF_FACE_THREAD(P.L);
  if (owns_face<0, T>(P.L, i, j, k)) fold_face<0>(Q0, P, i, j, k);
  if (owns_face<1, T>(P.L, i, j, k)) fold_face<1>(Q1, P, i, j, k);
  if (owns_face<2, T>(P.L, i, j, k)) fold_face<2>(Q2, P, i, j, k);
}

// Drag-coefficient adjoint of each cell (its face-adjacent ghosts copy it)
// chained to the porosity: c = coef ((1 - phi)/(phi + e))^b, evaluated in
// FP64 (dc/dphi is very large in nearly solid cells), added to phibar.
template <class T>
__global__ __launch_bounds__(256) void k_drag_coef_adj(Params<T> P, const T* __restrict__ Cbar,
                                                       const T* __restrict__ PHI, double* __restrict__ phibar,
                                                       double coef, double e, double b) {
  const Layout& L = P.L;
  const long long n = (long long)L.nx * L.ny * L.nz;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(c % L.nz);
    const long long r = c / L.nz;
    const int j = (int)(r % L.ny);
    const int i = (int)(r / L.ny);
    const long long o = L.at(i, j, k);
    double cb = (double)Cbar[o];
    if (i == 0) cb += (double)Cbar[o - L.SX];
    if (i == L.nx - 1) cb += (double)Cbar[o + L.SX];
    if (j == 0) cb += (double)Cbar[o - L.PZ];
    if (j == L.ny - 1) cb += (double)Cbar[o + L.PZ];
    if (k == 0) cb += (double)Cbar[o - 1];
    if (k == L.nz - 1) cb += (double)Cbar[o + 1];
    if (cb == 0.0) continue;
    const double f = (double)PHI[c];
    const double rr = (1.0 - f) / (f + e);
    const double dcdphi = -coef * b * pow(rr, b - 1.0) * (1.0 + e) / ((f + e) * (f + e));
    phibar[c] += cb * dcdphi;
  }
}

// -------------------------------------------------------- k-omega reverse
// Velocity gradients and |S|^2 at cell o, the same expressions as the
// forward turbulence update.
template <class T>
struct Strain {
  T g[3][3];   // g[c][d] = d u_c / d x_d
  T S2;
};

template <class T>
__device__ __forceinline__ Strain<T> strain_at(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V,
                                               const T* __restrict__ W, long long o) {
  const Layout& L = P.L;
  const long long SX = L.SX, PZ = L.PZ;
  const T h0 = T(0.5) * P.ih[0], h1 = T(0.5) * P.ih[1], h2 = T(0.5) * P.ih[2];
  auto uc = [&](long long q) { return T(0.5) * (U[q] + U[q + SX]); };
  auto vc = [&](long long q) { return T(0.5) * (V[q] + V[q + PZ]); };
  auto wc = [&](long long q) { return T(0.5) * (W[q] + W[q + 1]); };
  Strain<T> s;
  s.g[0][0] = (U[o + SX] - U[o]) * P.ih[0];
  s.g[1][1] = (V[o + PZ] - V[o]) * P.ih[1];
  s.g[2][2] = (W[o + 1] - W[o]) * P.ih[2];
  s.g[0][1] = (uc(o + PZ) - uc(o - PZ)) * h1;
  s.g[0][2] = (uc(o + 1) - uc(o - 1)) * h2;
  s.g[1][0] = (vc(o + SX) - vc(o - SX)) * h0;
  s.g[1][2] = (vc(o + 1) - vc(o - 1)) * h2;
  s.g[2][0] = (wc(o + SX) - wc(o - SX)) * h0;
  s.g[2][1] = (wc(o + PZ) - wc(o - PZ)) * h1;
  const T s01 = T(0.5) * (s.g[0][1] + s.g[1][0]), s02 = T(0.5) * (s.g[0][2] + s.g[2][0]);
  const T s12 = T(0.5) * (s.g[1][2] + s.g[2][1]);
  s.S2 = s.g[0][0] * s.g[0][0] + s.g[1][1] * s.g[1][1] + s.g[2][2] * s.g[2][2] +
         T(2) * (s01 * s01 + s02 * s02 + s12 * s12);
  return s;
}

// nu_t = min(max(k / max(omega, lim), 0), cap), lim = lim_coef |S|, and its
// derivatives where it is not clipped.
template <class T>
struct Nut {
  T nut, dk, dw, dS2;
};

template <class T>
__device__ __forceinline__ Nut<T> nut_of(const Params<T>& P, T kk, T ww, T S2) {
  Nut<T> n;
  const T root = sqrt(S2);
  const T lim = P.lim_coef * root;
  const bool den_w = ww != ww || ww > lim;   // which argument nmax returns
  const T den = den_w ? ww : lim;
  const T r = kk / den;
  n.nut = nmin(nmax(r, T(0)), P.cap);
  const bool live = r > T(0) && r < P.cap;
  n.dk = live ? T(1) / den : T(0);
  const T dden = live ? -r / den : T(0);
  n.dw = den_w ? dden : T(0);
  n.dS2 = (!den_w && root > T(0)) ? dden * P.lim_coef / (T(2) * root) : T(0);
  return n;
}

// Reverse of the k-omega update at one cell (the forward runs on the new
// velocity U and the old k, omega).  kb, wb, nb: adjoints of the new k,
// omega and nu_t; writes the adjoints of the old k and omega (atomic: the
// advection and Laplacian stencils reach the neighbours) and of U.
// Writes, per cell, the adjoints of its velocity gradients (SB.a[0]: the
// diagonal ones times 2 g_dd, SB.a[1]: the symmetric pairs 01, 02, 12 times
// g_cd + g_dc, all times the |S|^2 adjoint) and of its cell-centre velocity
// (SB.a[2]); k_strain_gather moves them to the faces.
template <class T>
__global__ __launch_bounds__(256) void k_turb_adj(Params<T> P, const T* __restrict__ U, const T* __restrict__ V,
                                                  const T* __restrict__ W, const T* __restrict__ K0,
                                                  const T* __restrict__ W0, const T* __restrict__ KB1,
                                                  const T* __restrict__ WB1, const T* __restrict__ NB1,
                                                  T* __restrict__ KB0, T* __restrict__ WB0, VelAdj<T> SB) {
  const Layout& L = P.L;
  const long long n = (long long)L.nx * L.ny * L.nz;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(c % L.nz);
    const long long rr = c / L.nz;
    const int j = (int)(rr % L.ny);
    const int i = (int)(rr / L.ny);
    const long long o = L.at(i, j, k);
    const T kb1 = KB1[o], wb1 = WB1[o], nb1 = NB1[o];
    if (kb1 == T(0) && wb1 == T(0) && nb1 == T(0)) {
#pragma unroll
      for (int q = 0; q < 9; ++q) SB.a[q / 3][q % 3][o] = T(0);
      continue;
    }
    const long long st[3] = {L.SX, (long long)L.PZ, 1LL};
    // forward recompute
    const Strain<T> s = strain_at(P, U, V, W, o);
    const T kk = K0[o], ww = W0[o];
    const Nut<T> nu0 = nut_of(P, kk, ww, s.S2);
    const T vel[3] = {T(0.5) * (U[o] + U[o + L.SX]), T(0.5) * (V[o] + V[o + L.PZ]), T(0.5) * (W[o] + W[o + 1])};
    auto adv = [&](const T* q) {
      const T cq = q[o];
      T a = (nmax(vel[0], T(0)) * (cq - q[o - L.SX]) + nmin(vel[0], T(0)) * (q[o + L.SX] - cq)) * P.ih[0];
      a += (nmax(vel[1], T(0)) * (cq - q[o - L.PZ]) + nmin(vel[1], T(0)) * (q[o + L.PZ] - cq)) * P.ih[1];
      a += (nmax(vel[2], T(0)) * (cq - q[o - 1]) + nmin(vel[2], T(0)) * (q[o + 1] - cq)) * P.ih[2];
      return a;
    };
    auto lap = [&](const T* q) {
      const T cq = q[o];
      return (q[o + L.SX] - T(2) * cq + q[o - L.SX]) * P.ih2[0] + (q[o + L.PZ] - T(2) * cq + q[o - L.PZ]) * P.ih2[1] +
             (q[o + 1] - T(2) * cq + q[o - 1]) * P.ih2[2];
    };
    const T lapK = lap(K0), lapW = lap(W0);
    const T knr = kk + P.dt * (-adv(K0) + T(2) * nu0.nut * s.S2 - T(kCmu) * kk * ww +
                               (P.nu + T(kSigmaStar) * nu0.nut) * lapK);
    const T wnr = ww + P.dt * (-adv(W0) + T(2 * kAlpha) * s.S2 - T(kBeta) * ww * ww + (P.nu + T(kSigma) * nu0.nut) * lapW);
    const bool kfree = knr != knr || knr > P.k_min, wfree = wnr != wnr || wnr > P.w_min;
    const T kn = kfree ? knr : P.k_min, wn = wfree ? wnr : P.w_min;
    // the new eddy viscosity
    const Nut<T> nu1 = nut_of(P, kn, wn, s.S2);
    T s2b = nb1 * nu1.dS2;
    const T bk = kfree ? kb1 + nb1 * nu1.dk : T(0);
    const T bw = wfree ? wb1 + nb1 * nu1.dw : T(0);
    // through the explicit update
    const T nutb = bk * P.dt * (T(2) * s.S2 + T(kSigmaStar) * lapK) + bw * P.dt * T(kSigma) * lapW;
    s2b += bk * P.dt * T(2) * nu0.nut + bw * P.dt * T(2 * kAlpha);
    T kkb = bk * (T(1) - P.dt * T(kCmu) * ww) + nutb * nu0.dk;
    T wwb = -bk * P.dt * T(kCmu) * kk + bw * (T(1) - P.dt * T(2 * kBeta) * ww) + nutb * nu0.dw;
    s2b += nutb * nu0.dS2;
    T velb[3] = {T(0), T(0), T(0)};
    // advection and Laplacian of q with weight cw = (adjoint) dt and diffusivity dq
    auto stencil_adj = [&](const T* q, T* QB, T cw, T dq, T& centre) {
      if (cw == T(0)) return;
      const T cq = q[o];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T up = nmax(vel[a], T(0)), dn = nmin(vel[a], T(0));
        centre += cw * (-(up - dn) * P.ih[a] - T(2) * dq * P.ih2[a]);
        add_to(QB + o - st[a], cw * (up * P.ih[a] + dq * P.ih2[a]));
        add_to(QB + o + st[a], cw * (-dn * P.ih[a] + dq * P.ih2[a]));
        const T slope = vel[a] > T(0) ? cq - q[o - st[a]] : (vel[a] < T(0) ? q[o + st[a]] - cq : T(0));
        velb[a] -= cw * slope * P.ih[a];
      }
    };
    stencil_adj(K0, KB0, bk * P.dt, P.nu + T(kSigmaStar) * nu0.nut, kkb);
    stencil_adj(W0, WB0, bw * P.dt, P.nu + T(kSigma) * nu0.nut, wwb);
    add_to(KB0 + o, kkb);
    add_to(WB0 + o, wwb);
    SB.a[0][0][o] = T(2) * s.g[0][0] * s2b;
    SB.a[0][1][o] = T(2) * s.g[1][1] * s2b;
    SB.a[0][2][o] = T(2) * s.g[2][2] * s2b;
    SB.a[1][0][o] = (s.g[0][1] + s.g[1][0]) * s2b;
    SB.a[1][1][o] = (s.g[0][2] + s.g[2][0]) * s2b;
    SB.a[1][2][o] = (s.g[1][2] + s.g[2][1]) * s2b;
    SB.a[2][0][o] = velb[0];
    SB.a[2][1][o] = velb[1];
    SB.a[2][2][o] = velb[2];
  }
}

// Transpose of the velocity gradients and cell-centre velocities of
// k_turb_adj, as a gather over every padded face position t of component C:
// g_CC of cells t - e_C (+) and t (-); the centred cross differences
// d u_C / d x_d of cells t -/+ e_d and t -/+ e_d - e_C; the cell-centre
// velocity of cells t and t - e_C.  Cells outside the grid give nothing.
template <int C, class T>
__device__ __forceinline__ T strain_gather_value(const Params<T>& P, const VelAdj<T>& SB, int i, int j, int k) {
  const Layout& L = P.L;
  auto val = [&](int a, int b, int ci, int cj, int ck) -> T {
    if (ci < 0 || cj < 0 || ck < 0 || ci >= L.nx || cj >= L.ny || ck >= L.nz) return T(0);
    return SB.a[a][b][L.at(ci, cj, ck)];
  };
  const int ec[3] = {C == 0, C == 1, C == 2};
  T s = (val(0, C, i - ec[0], j - ec[1], k - ec[2]) - val(0, C, i, j, k)) * P.ih[C];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d == C) continue;
    const int pair = (C + d == 1) ? 0 : ((C + d == 2) ? 1 : 2);   // 01, 02, 12
    const int ed[3] = {d == 0, d == 1, d == 2};
    const T q = T(0.25) * P.ih[d];
    s += q * (val(1, pair, i - ed[0], j - ed[1], k - ed[2]) +
              val(1, pair, i - ed[0] - ec[0], j - ed[1] - ec[1], k - ed[2] - ec[2]) -
              val(1, pair, i + ed[0], j + ed[1], k + ed[2]) -
              val(1, pair, i + ed[0] - ec[0], j + ed[1] - ec[1], k + ed[2] - ec[2]));
  }
  s += T(0.5) * (val(2, C, i, j, k) + val(2, C, i - ec[0], j - ec[1], k - ec[2]));
  return s;
}

template <class T>
__global__ __launch_bounds__(256) void k_strain_gather(Params<T> P, VelAdj<T> SB, T* __restrict__ G0,
                                                       T* __restrict__ G1, T* __restrict__ G2, long long nelem) {
  const Layout& L = P.L;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nelem;
       p += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(p / L.SX) - 1;
    const long long r = p - (long long)(i + 1) * L.SX;
    const int j = (int)(r / L.PZ) - 1;
    const int k = (int)(r - (long long)(j + 1) * L.PZ) - 1;
    G0[p] += strain_gather_value<0>(P, SB, i, j, k);
    G1[p] += strain_gather_value<1>(P, SB, i, j, k);
    G2[p] += strain_gather_value<2>(P, SB, i, j, k);
  }
}

// Reverse of store_cell for a cell field: each face-adjacent ghost's
// adjoint goes to its cell, except across an inlet side when the ghost held
// the inlet constant (use_inlet); ghosts cleared.
template <class T>
__global__ __launch_bounds__(256) void k_cell_fold(Params<T> P, T* __restrict__ q, int use_inlet) {
  const Layout& L = P.L;
  const long long n = (long long)L.nx * L.ny * L.nz;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(c % L.nz);
    const long long rr = c / L.nz;
    const int j = (int)(rr % L.ny);
    const int i = (int)(rr / L.ny);
    const int idx[3] = {i, j, k}, nn[3] = {L.nx, L.ny, L.nz};
    const long long st[3] = {L.SX, (long long)L.PZ, 1LL};
    const long long o = L.at(i, j, k);
    T acc = q[o];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int hi = 0; hi < 2; ++hi) {
        if (idx[a] != (hi ? nn[a] - 1 : 0)) continue;
        const long long gpos = o + (hi ? st[a] : -st[a]);
        if (!(use_inlet && P.bc[2 * a + hi] == INLET)) acc += q[gpos];
        q[gpos] = T(0);
      }
    }
    q[o] = acc;
  }
}

// Adjoint of the eddy viscosity the diffusion read: face f of component C
// uses nu + (nu_t[c - e_C] + nu_t[c]) / 2 times dt lap(q)_f, so each cell
// gathers half of dt lap(q)_f a_f from the two faces beside it along each
// axis; a ghost cell copies its interior neighbour, so a boundary cell also
// takes the half that went to its ghost.  Writes nb at interior cells.
template <int C, class T>
__device__ __forceinline__ T nut_face_term(const Params<T>& P, const T* __restrict__ q, const T* __restrict__ a,
                                           int i, int j, int k) {
  const T ab = adj_in<C>(P, a, i, j, k);
  if (ab == T(0)) return T(0);
  const Layout& L = P.L;
  const long long o = L.at(i, j, k);
  const T qc = q[o];
  const T lp = (q[o + L.SX] - T(2) * qc + q[o - L.SX]) * P.ih2[0] +
               (q[o + L.PZ] - T(2) * qc + q[o - L.PZ]) * P.ih2[1] + (q[o + 1] - T(2) * qc + q[o - 1]) * P.ih2[2];
  return T(0.5) * P.dt * lp * ab;
}

template <class T>
__global__ __launch_bounds__(256) void k_diffuse_nut_adj(Params<T> P, const T* __restrict__ Q0,
                                                         const T* __restrict__ Q1, const T* __restrict__ Q2,
                                                         const T* __restrict__ A0, const T* __restrict__ A1,
                                                         const T* __restrict__ A2, T* __restrict__ NB) {
  const Layout& L = P.L;
  const long long n = (long long)L.nx * L.ny * L.nz;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(c % L.nz);
    const long long rr = c / L.nz;
    const int j = (int)(rr % L.ny);
    const int i = (int)(rr / L.ny);
    T s = T(0);
    {
      const T lo = nut_face_term<0>(P, Q0, A0, i, j, k), hi = nut_face_term<0>(P, Q0, A0, i + 1, j, k);
      s += lo + hi + (i == 0 ? lo : T(0)) + (i == L.nx - 1 ? hi : T(0));
    }
    {
      const T lo = nut_face_term<1>(P, Q1, A1, i, j, k), hi = nut_face_term<1>(P, Q1, A1, i, j + 1, k);
      s += lo + hi + (j == 0 ? lo : T(0)) + (j == L.ny - 1 ? hi : T(0));
    }
    {
      const T lo = nut_face_term<2>(P, Q2, A2, i, j, k), hi = nut_face_term<2>(P, Q2, A2, i, j, k + 1);
      s += lo + hi + (k == 0 ? lo : T(0)) + (k == L.nz - 1 ? hi : T(0));
    }
    NB[L.at(i, j, k)] = s;
  }
}

// ---------------------------------------------------------- objective seed
// Derivative of a region objective with respect to the faces of the state:
// each face is half of the cell-centre velocity of its two cells, so
// dJ/du_f = (dJ/dU_c[C] + dJ/dU_c'[C]) / 2 over the adjacent cells inside
// the grid.  kind 0 (mean speeds): dJ/dU_c = (sum over the regions holding
// c of coef_r) U_c / |U_c|; kind 2 (desired field): (sum of coef_r)
// (U_c - U_target,c).  coef_r is precomputed by the host.
// The plane objective at column (i, j): the cell-centre velocity and the
// porosity interpolated between layers k0 and k0 + 1 with weight t, and
// s = sqrt(|u_p|^2 + 1e-12), as the forward evaluates them.
struct PlaneSeed {
  int k0;
  double t, st, smin, wpen, area;
};

template <class T>
__device__ __forceinline__ void plane_column(const Layout& L, const T* __restrict__ U, const T* __restrict__ V,
                                             const T* __restrict__ W, const T* __restrict__ PHI, const PlaneSeed& ps,
                                             int i, int j, double up[3], double& phip, double& s) {
  double uc[2], vc[2], wc[2], ph[2];
  for (int q = 0; q < 2; ++q) {
    const long long o = L.at(i, j, ps.k0 + q);
    uc[q] = 0.5 * ((double)U[o] + (double)U[o + L.SX]);
    vc[q] = 0.5 * ((double)V[o] + (double)V[o + L.PZ]);
    wc[q] = 0.5 * ((double)W[o] + (double)W[o + 1]);
    ph[q] = (double)PHI[((size_t)i * L.ny + j) * L.nz + ps.k0 + q];
  }
  up[0] = (1.0 - ps.t) * uc[0] + ps.t * uc[1];
  up[1] = (1.0 - ps.t) * vc[0] + ps.t * vc[1];
  up[2] = (1.0 - ps.t) * wc[0] + ps.t * wc[1];
  phip = (1.0 - ps.t) * ph[0] + ps.t * ph[1];
  s = sqrt(up[0] * up[0] + up[1] * up[1] + up[2] * up[2] + 1e-12);
}

template <class T>
__device__ __forceinline__ T seed_cell(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V,
                                       const T* __restrict__ W, const int* __restrict__ boxes,
                                       const double* __restrict__ coef, int nreg, int kind,
                                       const T* __restrict__ ut, const PlaneSeed& ps, const T* __restrict__ PHI,
                                       int C, int i, int j, int k) {
  const Layout& L = P.L;
  if (kind == 1) {
    // dJ/ds = area phi_p (2 (s - s_t) - 2 w max(0, s_min - s)), ds/du_p = u_p / s
    if (k != ps.k0 && k != ps.k0 + 1) return T(0);
    double up[3], phip, s;
    plane_column(L, U, V, W, PHI, ps, i, j, up, phip, s);
    const double lo = fmax(0.0, ps.smin - s);
    const double dJds = ps.area * phip * (2.0 * (s - ps.st) - 2.0 * ps.wpen * lo);
    return T((k == ps.k0 ? 1.0 - ps.t : ps.t) * dJds * up[C] / s);
  }
  double cs = 0.0;
  for (int r = 0; r < nreg; ++r) {
    const int* b = boxes + 6 * r;
    if (i >= b[0] && i < b[1] && j >= b[2] && j < b[3] && k >= b[4] && k < b[5]) cs += coef[r];
  }
  if (cs == 0.0) return T(0);
  const long long o = L.at(i, j, k);
  const double uc[3] = {0.5 * ((double)U[o] + (double)U[o + L.SX]), 0.5 * ((double)V[o] + (double)V[o + L.PZ]),
                        0.5 * ((double)W[o] + (double)W[o + 1])};
  if (kind == 0) {
    const double s = sqrt(uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2]);
    return s > 0.0 ? T(cs * uc[C] / s) : T(0);
  }
  const size_t n = (size_t)L.nx * L.ny * L.nz;
  const size_t cidx = ((size_t)i * L.ny + j) * L.nz + k;
  return T(cs * (uc[C] - (double)ut[(size_t)C * n + cidx]));
}

template <class T>
__global__ __launch_bounds__(256) void k_objective_seed(Params<T> P, const T* __restrict__ U, const T* __restrict__ V,
                                                        const T* __restrict__ W, const int* __restrict__ boxes,
                                                        const double* __restrict__ coef, int nreg, int kind,
                                                        const T* __restrict__ ut, PlaneSeed ps,
                                                        const T* __restrict__ PHI, T* __restrict__ out) {
  const Layout& L = P.L;
  const long long n0 = (long long)(L.nx + 1) * L.ny * L.nz, n1 = (long long)L.nx * (L.ny + 1) * L.nz;
  const long long n2 = (long long)L.nx * L.ny * (L.nz + 1);
  const long long ntot = n0 + n1 + n2;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < ntot;
       p += (long long)gridDim.x * blockDim.x) {
    int C = 0;
    long long q = p;
    if (q >= n0) {
      q -= n0;
      C = 1;
      if (q >= n1) {
        q -= n1;
        C = 2;
      }
    }
    const int e0 = L.nx + (C == 0), e1 = L.ny + (C == 1), e2 = L.nz + (C == 2);
    (void)e0;
    const int k = (int)(q % e2);
    const long long r = q / e2;
    const int j = (int)(r % e1);
    const int i = (int)(r / e1);
    const int idx[3] = {i, j, k};
    const int nC = C == 0 ? L.nx : (C == 1 ? L.ny : L.nz);
    T s = T(0);
    if (idx[C] > 0)
      s += seed_cell(P, U, V, W, boxes, coef, nreg, kind, ut, ps, PHI, C, i - (C == 0), j - (C == 1), k - (C == 2));
    if (idx[C] < nC) s += seed_cell(P, U, V, W, boxes, coef, nreg, kind, ut, ps, PHI, C, i, j, k);
    out[p] = T(0.5) * s;
  }
}

// The plane objective's direct porosity weight: dJ/dphi_p = area ((s - s_t)^2
// + w max(0, s_min - s)^2), split (1 - t) / t onto layers k0 and k0 + 1.
template <class T>
__global__ __launch_bounds__(256) void k_plane_phi_seed(Layout L, const T* __restrict__ U, const T* __restrict__ V,
                                                        const T* __restrict__ W, const T* __restrict__ PHI,
                                                        PlaneSeed ps, double* __restrict__ phibar) {
  const int n = L.nx * L.ny;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const int i = c / L.ny, j = c % L.ny;
    double up[3], phip, s;
    plane_column(L, U, V, W, PHI, ps, i, j, up, phip, s);
    const double lo = fmax(0.0, ps.smin - s);
    const double d = ps.area * ((s - ps.st) * (s - ps.st) + ps.wpen * lo * lo);
    const size_t base = ((size_t)i * L.ny + j) * L.nz + ps.k0;
    phibar[base] += (1.0 - ps.t) * d;
    phibar[base + 1] += ps.t * d;
  }
}

// ----------------------------------------------------------------- launchers
template <class T>
static VelAdj<T> vel_adj(const Grid& g) {
  VelAdj<T> V;
  for (int c = 0; c < 3; ++c)
    for (int cp = 0; cp < 3; ++cp) V.a[c][cp] = (T*)g.AV[c][cp];
  return V;
}

template <class T>
static void launch_vel_gather(Grid& g, const Params<T>& P, void* const G[3]) {
  const long long n = (long long)g.nelem;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_vel_gather<T>, dim3(blocks), dim3(256), 0, g.stream, P, vel_adj<T>(g), (T*)G[0], (T*)G[1],
                     (T*)G[2], n);
}

template <class T>
void launch_advect_adj(Grid& g, const Params<T>& P, void* const Qin[3], void* const Qhat[3], void* const Aout[3],
                       void* const Gq[3], void* const Ghat[3]) {
  const dim3 grid = adj_face_grid(P.L);
  hipLaunchKernelGGL(k_advect_corr_adj<T>, grid, dim3(kFaceBlock), 0, g.stream, P, (const T*)Qin[0],
                     (const T*)Qin[1], (const T*)Qin[2], (const T*)Qhat[0], (const T*)Qhat[1], (const T*)Qhat[2],
                     (const T*)Aout[0], (const T*)Aout[1], (const T*)Aout[2], (T*)Gq[0], (T*)Gq[1], (T*)Gq[2],
                     (T*)Ghat[0], (T*)Ghat[1], (T*)Ghat[2], vel_adj<T>(g));
  // qhat's ghosts came from its interior faces: fold them before its reverse
  hipLaunchKernelGGL(k_fold<T>, grid, dim3(kFaceBlock), 0, g.stream, P, (T*)Ghat[0], (T*)Ghat[1], (T*)Ghat[2]);
  hipLaunchKernelGGL(k_advect_fwd_adj<T>, grid, dim3(kFaceBlock), 0, g.stream, P, (const T*)Qin[0],
                     (const T*)Qin[1], (const T*)Qin[2], (const T*)Ghat[0], (const T*)Ghat[1], (const T*)Ghat[2],
                     (T*)Gq[0], (T*)Gq[1], (T*)Gq[2], vel_adj<T>(g));
  launch_vel_gather<T>(g, P, Gq);
}

template <class T>
void launch_diffuse_adj(Grid& g, const Params<T>& P, void* const Aout[3], void* const Gin[3]) {
  const long long n = (long long)g.nelem;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_diffuse_adj<T>, dim3(blocks), dim3(256), 0, g.stream, P, (const T*)Aout[0],
                     (const T*)Aout[1], (const T*)Aout[2], (const T*)g.NUT, (T*)Gin[0], (T*)Gin[1], (T*)Gin[2], n);
}

template <class T>
void launch_drag_adj(Grid& g, const Params<T>& P, void* const Qin[3], void* const Aout[3], void* const Gin[3],
                     void* Cbar) {
  hipLaunchKernelGGL(k_drag_adj<T>, adj_face_grid(P.L), dim3(kFaceBlock), 0, g.stream, P, (const T*)Qin[0],
                     (const T*)Qin[1], (const T*)Qin[2], (const T*)g.C, (const T*)Aout[0], (const T*)Aout[1],
                     (const T*)Aout[2], (T*)Cbar, vel_adj<T>(g));
  launch_vel_gather<T>(g, P, Gin);
}

template <class T>
void launch_fold(Grid& g, const Params<T>& P, void* const A[3]) {
  hipLaunchKernelGGL(k_fold<T>, adj_face_grid(P.L), dim3(kFaceBlock), 0, g.stream, P, (T*)A[0], (T*)A[1], (T*)A[2]);
}

template <class T>
void launch_drag_coef_adj(Grid& g, const Params<T>& P, const void* Cbar, double* phibar) {
  const long long n = (long long)P.L.nx * P.L.ny * P.L.nz;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
  const uf_config& c = g.cfg;
  hipLaunchKernelGGL(k_drag_coef_adj<T>, dim3(blocks), dim3(256), 0, g.stream, P, (const T*)Cbar, (const T*)g.PHI,
                     phibar, c.Cd * c.a, c.e, c.b);
}

template <class T>
void launch_objective_seed(Grid& g, const Params<T>& P, const int* boxes_dev, const double* coef_dev, int nreg,
                           int kind, const void* ut, void* out, const double plane[6], double* phibar) {
  const Layout& L = P.L;
  const long long n = (long long)(L.nx + 1) * L.ny * L.nz + (long long)L.nx * (L.ny + 1) * L.nz +
                      (long long)L.nx * L.ny * (L.nz + 1);
  const int blocks = (int)std::min<long long>((n + 255) / 256, 16384);
  void* const* Q = g.Q[g.cur];
  PlaneSeed ps{0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (plane) ps = PlaneSeed{(int)plane[0], plane[1], plane[2], plane[3], plane[4], plane[5]};
  hipLaunchKernelGGL(k_objective_seed<T>, dim3(blocks), dim3(256), 0, g.stream, P, (const T*)Q[0], (const T*)Q[1],
                     (const T*)Q[2], boxes_dev, coef_dev, nreg, kind, (const T*)ut, ps, (const T*)g.PHI, (T*)out);
  if (plane && phibar) {
    const int cols = L.nx * L.ny;
    hipLaunchKernelGGL(k_plane_phi_seed<T>, dim3(std::min(8192, (cols + 255) / 256)), dim3(256), 0, g.stream, L,
                       (const T*)Q[0], (const T*)Q[1], (const T*)Q[2], (const T*)g.PHI, ps, phibar);
  }
}

static inline int cell_blocks(const Layout& L) {
  const long long n = (long long)L.nx * L.ny * L.nz;
  return (int)std::min<long long>((n + 255) / 256, 8192);
}

template <class T>
void launch_turb_adj(Grid& g, const Params<T>& P, void* const Unew[3], const void* K0, const void* W0,
                     const void* KB1, const void* WB1, const void* NB1, void* KB0, void* WB0, void* const G[3]) {
  // the per-cell values go through the velocity-adjoint arrays, which the
  // next reverse kernel overwrites (its gather reads interior cells only here)
  hipLaunchKernelGGL(k_turb_adj<T>, dim3(cell_blocks(P.L)), dim3(256), 0, g.stream, P, (const T*)Unew[0],
                     (const T*)Unew[1], (const T*)Unew[2], (const T*)K0, (const T*)W0, (const T*)KB1, (const T*)WB1,
                     (const T*)NB1, (T*)KB0, (T*)WB0, vel_adj<T>(g));
  const long long n = (long long)g.nelem;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_strain_gather<T>, dim3(blocks), dim3(256), 0, g.stream, P, vel_adj<T>(g), (T*)G[0], (T*)G[1],
                     (T*)G[2], n);
}

template <class T>
void launch_cell_fold(Grid& g, const Params<T>& P, void* q, int use_inlet) {
  hipLaunchKernelGGL(k_cell_fold<T>, dim3(cell_blocks(P.L)), dim3(256), 0, g.stream, P, (T*)q, use_inlet);
}

template <class T>
void launch_diffuse_nut_adj(Grid& g, const Params<T>& P, void* const Qin[3], void* const Aout[3], void* NB) {
  hipLaunchKernelGGL(k_diffuse_nut_adj<T>, dim3(cell_blocks(P.L)), dim3(256), 0, g.stream, P, (const T*)Qin[0],
                     (const T*)Qin[1], (const T*)Qin[2], (const T*)Aout[0], (const T*)Aout[1], (const T*)Aout[2],
                     (T*)NB);
}

#define UF_INST(T)                                                                                             \
  template void launch_advect_adj<T>(Grid&, const Params<T>&, void* const[3], void* const[3], void* const[3],  \
                                     void* const[3], void* const[3]);                                           \
  template void launch_diffuse_adj<T>(Grid&, const Params<T>&, void* const[3], void* const[3]);                \
  template void launch_drag_adj<T>(Grid&, const Params<T>&, void* const[3], void* const[3], void* const[3],    \
                                   void*);                                                                      \
  template void launch_fold<T>(Grid&, const Params<T>&, void* const[3]);                                        \
  template void launch_drag_coef_adj<T>(Grid&, const Params<T>&, const void*, double*);                        \
  template void launch_objective_seed<T>(Grid&, const Params<T>&, const int*, const double*, int, int,         \
                                         const void*, void*, const double*, double*);                           \
  template void launch_turb_adj<T>(Grid&, const Params<T>&, void* const[3], const void*, const void*,         \
                                   const void*, const void*, const void*, void*, void*, void* const[3]);        \
  template void launch_cell_fold<T>(Grid&, const Params<T>&, void*, int);                                      \
  template void launch_diffuse_nut_adj<T>(Grid&, const Params<T>&, void* const[3], void* const[3], void*);
UF_INST(float)
UF_INST(double)
#undef UF_INST

}  // namespace uf
