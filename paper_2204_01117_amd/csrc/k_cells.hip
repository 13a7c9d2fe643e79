// Cell-centred kernels: the k-omega turbulence update (Sec. 3, solved after
// the projection), the porosity -> drag-coefficient map (Sec. 3 drag law),
// boundary refresh of cell fields and packing between the padded storage
// and the compact layouts of the C ABI.
#include "turb_model.h"
#include "uf_internal.h"

namespace uf {

constexpr int kCellBlock = 256;

__host__ __device__ inline int cell_gx(const Layout& L) { return (L.ny * L.nz + kCellBlock - 1) / kCellBlock; }

// Logical block (bx, i) of a cell kernel launched on xcd_grid(cell_gx, nx):
// XCD-contiguous ranges of the band-major order (band_map), as the face
// kernels, so that the x-neighbours a stencil reads stay in the XCD's L2.
constexpr int kCellBand = 8;
__device__ __forceinline__ bool cell_block(const Layout& L, int& bx, int& i) {
  const int gx = cell_gx(L), gy = L.nx;
  const int per = (int)(gridDim.x >> 3);
  const int b = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  if (b >= gx * gy) return false;
  band_map(gx, gy, kCellBand, b, bx, i);
  return true;
}

// A thread owns cell (i, j, k) of logical block (bx, iplane); threads past
// the plane's cells return.
#define UF_CELL_POINT(L, bx, iplane)                                 \
  const int i = (iplane);                                            \
  const int p = (bx) * kCellBlock + threadIdx.x;                     \
  if (p >= (L).ny * (L).nz) return;                                  \
  const int j = p / (L).nz;                                          \
  const int k = p - j * (L).nz;

#define UF_CELL_THREAD(L)                                            \
  int c_bx, c_by;                                                    \
  if (!cell_block((L), c_bx, c_by)) return;                          \
  UF_CELL_POINT(L, c_bx, c_by)

// k-omega step at one cell.  Velocity gradients: normal derivatives from the
// cell's two faces, cross derivatives as central differences of cell-centred
// velocities (face means; ghost faces beyond the domain).  Strain rate
// S = (grad u + grad u^T)/2, |S|^2 = S_ij S_ij.  Limiter omega~ = max(omega,
// C_lim |S| / sqrt(C_mu/2)) (Wilcox 2006, cited in Sec. 3); eddy viscosity
// nu_t = k / omega~ limited to [0, nu_max - nu] (the paper's von Neumann
// viscosity limiter).  Forward Euler with first-order upwind advection and
// central Laplacians.
template <class T>
__device__ __forceinline__ void turb_cells(const Params<T>& P, const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ W, const T* __restrict__ K0, const T* __restrict__ W0, T* __restrict__ K1, T* __restrict__ W1, T* __restrict__ NUT, int update_kw, int* nf, int bx, int ib) {
  const Layout& L = P.L;
  UF_CELL_POINT(L, bx, ib);
  const long long SX = L.SX, PZ = L.PZ;
  const long long o = L.at(i, j, k);
  const T h0 = T(0.5) * P.ih[0], h1 = T(0.5) * P.ih[1], h2 = T(0.5) * P.ih[2];
  // gradients G[c][d] = d u_c / d x_d
  const T g00 = (U[o + SX] - U[o]) * P.ih[0];
  const T g11 = (V[o + PZ] - V[o]) * P.ih[1];
  const T g22 = (W[o + 1] - W[o]) * P.ih[2];
  auto uc = [&](long long q) { return T(0.5) * (U[q] + U[q + SX]); };
  auto vc = [&](long long q) { return T(0.5) * (V[q] + V[q + PZ]); };
  auto wc = [&](long long q) { return T(0.5) * (W[q] + W[q + 1]); };
  const T g01 = (uc(o + PZ) - uc(o - PZ)) * h1;
  const T g02 = (uc(o + 1) - uc(o - 1)) * h2;
  const T g10 = (vc(o + SX) - vc(o - SX)) * h0;
  const T g12 = (vc(o + 1) - vc(o - 1)) * h2;
  const T g20 = (wc(o + SX) - wc(o - SX)) * h0;
  const T g21 = (wc(o + PZ) - wc(o - PZ)) * h1;
  const T s01 = T(0.5) * (g01 + g10), s02 = T(0.5) * (g02 + g20), s12 = T(0.5) * (g12 + g21);
  const T S2 = g00 * g00 + g11 * g11 + g22 * g22 + T(2) * (s01 * s01 + s02 * s02 + s12 * s12);
  const T lim = P.lim_coef * sqrt(S2);
  const T kk = K0[o], ww = W0[o];
  const T nut = nmin(nmax(kk / nmax(ww, lim), T(0)), P.cap);
  if (!update_kw) {
    store_cell(NUT, P, i, j, k, nut, false, T(0));
    return;
  }
  const T u0 = uc(o), u1 = vc(o), u2 = wc(o);
  auto adv = [&](const T* q) {
    const T c = q[o];
    T a = (nmax(u0, T(0)) * (c - q[o - SX]) + nmin(u0, T(0)) * (q[o + SX] - c)) * P.ih[0];
    a += (nmax(u1, T(0)) * (c - q[o - PZ]) + nmin(u1, T(0)) * (q[o + PZ] - c)) * P.ih[1];
    a += (nmax(u2, T(0)) * (c - q[o - 1]) + nmin(u2, T(0)) * (q[o + 1] - c)) * P.ih[2];
    return a;
  };
  auto lap = [&](const T* q) {
    const T c = q[o];
    return (q[o + SX] - T(2) * c + q[o - SX]) * P.ih2[0] + (q[o + PZ] - T(2) * c + q[o - PZ]) * P.ih2[1] +
           (q[o + 1] - T(2) * c + q[o - 1]) * P.ih2[2];
  };
  T kn = kk + P.dt * (-adv(K0) + T(2) * nut * S2 - T(kCmu) * kk * ww + (P.nu + T(kSigmaStar) * nut) * lap(K0));
  T wn = ww + P.dt * (-adv(W0) + T(2 * kAlpha) * S2 - T(kBeta) * ww * ww + (P.nu + T(kSigma) * nut) * lap(W0));
  kn = nmax(kn, P.k_min);
  wn = nmax(wn, P.w_min);
  if (!(isfinite(kn) && isfinite(wn))) *nf = 1;   // every writer stores 1: no atomic needed
  const T nut_new = nmin(nmax(kn / nmax(wn, lim), T(0)), P.cap);
  store_cell(K1, P, i, j, k, kn, true, P.k_in);
  store_cell(W1, P, i, j, k, wn, true, P.w_in);
  store_cell(NUT, P, i, j, k, nut_new, false, T(0));
}

// gate: as k_project's (the step's k-omega update enqueued with it).
template <class T>
__global__ __launch_bounds__(kCellBlock) void k_turbulence(Params<T> P, const T* __restrict__ U, const T* __restrict__ V, const T* __restrict__ W, const T* __restrict__ K0, const T* __restrict__ W0, T* __restrict__ K1, T* __restrict__ W1, T* __restrict__ NUT, int update_kw, int* nf, const int* __restrict__ gate) {
  if (gate && !*gate) return;
  int bx, ib;
  if (!cell_block(P.L, bx, ib)) return;
  turb_cells(P, U, V, W, K0, W0, K1, W1, NUT, update_kw, nf, bx, ib);
}

// Drag coefficient of each cell: C_d a ((1 - phi)/(phi + e))^b (Sec. 3 drag
// law with the porosity form of its footnote); also keeps phi (compact).
template <class T>
__global__ __launch_bounds__(kCellBlock) void k_porosity(Params<T> P, const T* __restrict__ phi, T* __restrict__ Cc,
                                                         T* __restrict__ PHI, T coef, T e, T b) {
  const Layout& L = P.L;
  UF_CELL_THREAD(L);
  const size_t c = ((size_t)i * L.ny + j) * L.nz + k;
  const T f = phi[c];
  PHI[c] = f;
  store_cell(Cc, P, i, j, k, coef * pow((T(1) - f) / (f + e), b), false, T(0));
}

template <class T>
__global__ __launch_bounds__(kCellBlock) void k_cell_bc(Params<T> P, T* __restrict__ q, int use_inlet, T inlet) {
  const Layout& L = P.L;
  UF_CELL_THREAD(L);
  store_cell(q, P, i, j, k, q[L.at(i, j, k)], use_inlet != 0, inlet);
}

template <class T>
__global__ __launch_bounds__(kCellBlock) void k_cell_fill(Params<T> P, T* __restrict__ q, T value, int use_inlet,
                                                          T inlet) {
  const Layout& L = P.L;
  UF_CELL_THREAD(L);
  store_cell(q, P, i, j, k, value, use_inlet != 0, inlet);
}

// Copy between the compact layout of a field and the padded storage.
template <class T>
__global__ __launch_bounds__(kCellBlock) void k_pack(Layout L, int ex, int ey, int ez, const T* __restrict__ src,
                                                     T* __restrict__ dst, int unpack) {
  const size_t n = (size_t)ex * ey * ez;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(c % ez);
    const size_t r = c / ez;
    const int j = (int)(r % ey);
    const int i = (int)(r / ey);
    const long long o = L.at(i, j, k);
    if (unpack) dst[o] = src[c];
    else dst[c] = src[o];
  }
}

// Sum of the cell-centre wind speed over a box of cells (one FP64 partial per
// block; the caller adds the partials in block order).
template <class T>
__global__ __launch_bounds__(kCellBlock) void k_region_speed(Layout L, const T* __restrict__ U, const T* __restrict__ V,
                                                            const T* __restrict__ W, int i0, int j0, int k0, int ni,
                                                            int nj, int nk, double* __restrict__ part) {
  const long long n = (long long)ni * nj * nk;
  double v[1] = {0.0};
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
    const int k = k0 + (int)(c % nk);
    const long long r = c / nk;
    const int j = j0 + (int)(r % nj);
    const int i = i0 + (int)(r / nj);
    const long long o = L.at(i, j, k);
    const double uc = 0.5 * ((double)U[o] + (double)U[o + L.SX]);
    const double vc = 0.5 * ((double)V[o] + (double)V[o + L.PZ]);
    const double wc = 0.5 * ((double)W[o] + (double)W[o + 1]);
    v[0] += sqrt(uc * uc + vc * vc + wc * wc);
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Pedestrian-plane objective: per column, the cell-centre velocity and the
// porosity interpolated in z at weight t between levels k0 and k0 + 1, the
// speed s = sqrt(|u|^2 + 1e-12), and phi [(s - st)^2 + w max(0, smin - s)^2];
// one FP64 partial per block.
template <class T>
__global__ __launch_bounds__(kCellBlock) void k_plane_objective(Layout L, const T* __restrict__ U,
                                                               const T* __restrict__ V, const T* __restrict__ W,
                                                               const T* __restrict__ PHI, int k0, double t,
                                                               double st, double smin, double wpen,
                                                               double* __restrict__ part) {
  const int n = L.nx * L.ny;
  double v[1] = {0.0};
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const int i = c / L.ny, j = c % L.ny;
    double uc[2], vc[2], wc[2], ph[2];
    for (int q = 0; q < 2; ++q) {
      const long long o = L.at(i, j, k0 + q);
      uc[q] = 0.5 * ((double)U[o] + (double)U[o + L.SX]);
      vc[q] = 0.5 * ((double)V[o] + (double)V[o + L.PZ]);
      wc[q] = 0.5 * ((double)W[o] + (double)W[o + 1]);
      ph[q] = (double)PHI[((size_t)i * L.ny + j) * L.nz + k0 + q];
    }
    const double up = (1.0 - t) * uc[0] + t * uc[1];
    const double vp = (1.0 - t) * vc[0] + t * vc[1];
    const double wp = (1.0 - t) * wc[0] + t * wc[1];
    const double phip = (1.0 - t) * ph[0] + t * ph[1];
    const double s = sqrt(up * up + vp * vp + wp * wp + 1e-12);
    const double lo = fmax(0.0, smin - s);
    v[0] += phip * ((s - st) * (s - st) + wpen * lo * lo);
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

template <class T>
void launch_plane_objective(Grid& g, int k0, double t, double st, double smin, double wpen, double* part,
                            int nblocks) {
  hipLaunchKernelGGL(k_plane_objective<T>, dim3(nblocks), dim3(kCellBlock), 0, g.stream, g.L,
                     (const T*)g.Q[g.cur][0], (const T*)g.Q[g.cur][1], (const T*)g.Q[g.cur][2], (const T*)g.PHI, k0,
                     t, st, smin, wpen, part);
}

// Squared distance between the cell-centre velocity and a desired one over a
// box of cells (one FP64 partial per block).
template <class T>
__global__ __launch_bounds__(kCellBlock) void k_region_field_diff(Layout L, const T* __restrict__ U,
                                                                 const T* __restrict__ V, const T* __restrict__ W,
                                                                 const T* __restrict__ UT, int i0, int j0, int k0,
                                                                 int ni, int nj, int nk, double* __restrict__ part) {
  const long long n = (long long)ni * nj * nk;
  const size_t N = (size_t)L.nx * L.ny * L.nz;
  double v[1] = {0.0};
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
    const int k = k0 + (int)(c % nk);
    const long long r = c / nk;
    const int j = j0 + (int)(r % nj);
    const int i = i0 + (int)(r / nj);
    const long long o = L.at(i, j, k);
    const size_t q = ((size_t)i * L.ny + j) * L.nz + k;
    const double du = 0.5 * ((double)U[o] + (double)U[o + L.SX]) - (double)UT[q];
    const double dv = 0.5 * ((double)V[o] + (double)V[o + L.PZ]) - (double)UT[N + q];
    const double dw = 0.5 * ((double)W[o] + (double)W[o + 1]) - (double)UT[2 * N + q];
    v[0] += du * du + dv * dv + dw * dw;
  }
  block_sum<1>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

template <class T>
void launch_region_field_diff(Grid& g, const int box[6], const void* ut, double* part, int nblocks) {
  hipLaunchKernelGGL(k_region_field_diff<T>, dim3(nblocks), dim3(kCellBlock), 0, g.stream, g.L,
                     (const T*)g.Q[g.cur][0], (const T*)g.Q[g.cur][1], (const T*)g.Q[g.cur][2], (const T*)ut, box[0],
                     box[2], box[4], box[1] - box[0], box[3] - box[2], box[5] - box[4], part);
}

template <class T>
void launch_region_speed(Grid& g, const int box[6], double* part, int nblocks) {
  hipLaunchKernelGGL(k_region_speed<T>, dim3(nblocks), dim3(kCellBlock), 0, g.stream, g.L, (const T*)g.Q[g.cur][0],
                     (const T*)g.Q[g.cur][1], (const T*)g.Q[g.cur][2], box[0], box[2], box[4], box[1] - box[0],
                     box[3] - box[2], box[5] - box[4], part);
}

template <class T>
__global__ __launch_bounds__(kCellBlock) void k_check_range(const T* __restrict__ phi, size_t n, int* flag) {
  int bad = 0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) {
    const T f = phi[c];
    if (!(f >= T(0) && f <= T(1))) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

static inline dim3 cell_grid(const Layout& L) { return xcd_grid(cell_gx(L), L.nx); }

template <class T>
void launch_turb(Grid& g, const Params<T>& P, void* const Q[3], const void* K0, const void* W0, void* K1, void* W1,
                 void* NUT, int update_kw, const int* gate) {
  TimedLaunch tl(g, UF_TK_TURB);
  launch_k(g, k_turbulence<T>, cell_grid(P.L), dim3(kCellBlock), P, (const T*)Q[0],
                     (const T*)Q[1], (const T*)Q[2], (const T*)K0, (const T*)W0, (T*)K1, (T*)W1, (T*)NUT, update_kw,
                     nf_word(g), gate);
}

// The k-omega update of every case of a batch in one persistent launch
// (the cell queue: case c owns [cell0, cell0 + cell_gx * nx)); velocity
// from set sq, k and omega of case c from slot kcs[c] to the other slot,
// nu_t into the case's own array, or into set nut_set's u array when
// nut_set >= 0 (a trial run that leaves the state alone).
template <class T>
__global__ __launch_bounds__(kCellBlock) void k_turb_multi(const MultiCase<T>* __restrict__ mc, CaseStarts cs,
                                                          int band, int sq, const int* __restrict__ kcs,
                                                          int nut_set) {
  const int nb = (int)(gridDim.x >> 3);
  const int xcd = (int)(blockIdx.x & 7u), lid = (int)(blockIdx.x >> 3);
  const int total = cs.start[cs.n];
  const int share = (total + 7) >> 3;
  const int lo = xcd * share, hi = min(total, lo + share);
  for (int lb = lo + lid; lb < hi; lb += nb) {
    const int c = find_case(cs, lb);
    const MultiCase<T>& A = mc[c];
    int bx, ib;
    band_map(cell_gx(A.P.L), A.P.L.nx, band, lb - cs.start[c], bx, ib);
    T* nut = nut_set >= 0 ? A.q[nut_set][0] : A.nut;
    const int kc = kcs[c] & 1;
    turb_cells(A.P, A.q[sq][0], A.q[sq][1], A.q[sq][2], A.k[kc], A.w[kc], A.k[kc ^ 1], A.w[kc ^ 1], nut, 1, A.nf,
               bx, ib);
  }
}

template <class T>
void launch_turb_multi(const MultiCase<T>* mc, const CaseStarts& cs, int band, int blocks, int sq, const int* kcs,
                       int nut_set, hipStream_t stream) {
  hipLaunchKernelGGL(k_turb_multi<T>, dim3((unsigned)blocks), dim3(kCellBlock), 0, stream, mc, cs, band, sq, kcs,
                     nut_set);
}

int cell_queue_blocks(const Layout& L) { return cell_gx(L) * L.nx; }

// Diagnostics of a state, one partial per block and quantity: the largest
// |div_h u| over the cells, the largest dt sum_d |u_d| / h_d with the
// cell-centre velocity (the stability number of the upwind k-omega
// advection), and the number of cells whose eddy viscosity sits at the cap.
// NaN propagates into the maxima.
template <class T>
__global__ __launch_bounds__(kCellBlock) void k_diag(Params<T> P, const T* __restrict__ U, const T* __restrict__ V,
                                                     const T* __restrict__ W, const T* __restrict__ NUT, int turb,
                                                     double* __restrict__ part) {
  const Layout& L = P.L;
  const long long n = (long long)L.nx * L.ny * L.nz;
  double mdiv = 0.0, mcfl = 0.0, clip = 0.0;
  const double ih0 = 1.0 / (double)P.h[0], ih1 = 1.0 / (double)P.h[1], ih2 = 1.0 / (double)P.h[2];
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(c % L.nz);
    const long long r = c / L.nz;
    const int j = (int)(r % L.ny);
    const int i = (int)(r / L.ny);
    const long long o = L.at(i, j, k);
    const double u0 = U[o], u1 = U[o + L.SX], v0 = V[o], v1 = V[o + L.PZ], w0 = W[o], w1 = W[o + 1];
    const double div = (u1 - u0) * ih0 + (v1 - v0) * ih1 + (w1 - w0) * ih2;
    mdiv = nmax(fabs(div), mdiv);
    const double cfl = (double)P.dt * (0.5 * fabs(u0 + u1) * ih0 + 0.5 * fabs(v0 + v1) * ih1 + 0.5 * fabs(w0 + w1) * ih2);
    mcfl = nmax(cfl, mcfl);
    if (turb && NUT[o] >= P.cap) clip += 1.0;
  }
  __shared__ double sh[3][kCellBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    mdiv = nmax(__shfl_xor(mdiv, o, 64), mdiv);
    mcfl = nmax(__shfl_xor(mcfl, o, 64), mcfl);
    clip += __shfl_xor(clip, o, 64);
  }
  if (lane == 0) {
    sh[0][wv] = mdiv;
    sh[1][wv] = mcfl;
    sh[2][wv] = clip;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kCellBlock / 64; ++q) {
      mdiv = nmax(sh[0][q], mdiv);
      mcfl = nmax(sh[1][q], mcfl);
      clip += sh[2][q];
    }
    part[blockIdx.x] = mdiv;
    part[kDiagBlocks + blockIdx.x] = mcfl;
    part[2 * kDiagBlocks + blockIdx.x] = clip;
  }
}

template <class T>
void launch_diag(Grid& g, const Params<T>& P) {
  const int turb = g.cfg.turb_model == UF_TURB_KOMEGA;
  hipLaunchKernelGGL(k_diag<T>, dim3(kDiagBlocks), dim3(kCellBlock), 0, g.stream, P, (const T*)g.Q[g.cur][0],
                     (const T*)g.Q[g.cur][1], (const T*)g.Q[g.cur][2], (const T*)g.NUT, turb, g.diag);
}

template <class T>
void launch_porosity(Grid& g, const Params<T>& P, const void* phi) {
  const uf_config& c = g.cfg;
  hipLaunchKernelGGL(k_porosity<T>, cell_grid(P.L), dim3(kCellBlock), 0, g.stream, P, (const T*)phi, (T*)g.C,
                     (T*)g.PHI, T(c.Cd * c.a), T(c.e), T(c.b));
}

template <class T>
void launch_cell_bc(Grid& g, const Params<T>& P, void* q, int use_inlet, double inlet_value) {
  hipLaunchKernelGGL(k_cell_bc<T>, cell_grid(P.L), dim3(kCellBlock), 0, g.stream, P, (T*)q, use_inlet,
                     T(inlet_value));
}

template <class T>
void launch_cell_fill(Grid& g, const Params<T>& P, void* q, double value, int use_inlet, double inlet_value) {
  hipLaunchKernelGGL(k_cell_fill<T>, cell_grid(P.L), dim3(kCellBlock), 0, g.stream, P, (T*)q, T(value), use_inlet,
                     T(inlet_value));
}

template <class T>
void launch_pack(Grid& g, const Params<T>& P, const void* src, void* dst, int field, int unpack) {
  int e[3] = {P.L.nx, P.L.ny, P.L.nz};
  if (field >= 0 && field < 3) e[field] += 1;
  const size_t n = (size_t)e[0] * e[1] * e[2];
  const int blocks = (int)std::min<size_t>((n + kCellBlock - 1) / kCellBlock, 8192);
  hipLaunchKernelGGL(k_pack<T>, dim3(blocks), dim3(kCellBlock), 0, g.stream, P.L, e[0], e[1], e[2], (const T*)src,
                     (T*)dst, unpack);
}

template <class T>
void launch_check_range(Grid& g, const void* phi, size_t n) {
  const int blocks = (int)std::min<size_t>((n + kCellBlock - 1) / kCellBlock, 4096);
  hipLaunchKernelGGL(k_check_range<T>, dim3(blocks), dim3(kCellBlock), 0, g.stream, (const T*)phi, n, g.flag);
}

template void launch_plane_objective<float>(Grid&, int, double, double, double, double, double*, int);
template void launch_plane_objective<double>(Grid&, int, double, double, double, double, double*, int);
template void launch_region_field_diff<float>(Grid&, const int[6], const void*, double*, int);
template void launch_region_field_diff<double>(Grid&, const int[6], const void*, double*, int);
template void launch_region_speed<float>(Grid&, const int[6], double*, int);
template void launch_region_speed<double>(Grid&, const int[6], double*, int);

#define UF_INST(T)                                                                                            \
  template void launch_turb<T>(Grid&, const Params<T>&, void* const[3], const void*, const void*, void*, void*, \
                               void*, int, const int*);                                                     \
  template void launch_diag<T>(Grid&, const Params<T>&);                                                     \
  template void launch_porosity<T>(Grid&, const Params<T>&, const void*);                                    \
  template void launch_cell_bc<T>(Grid&, const Params<T>&, void*, int, double);                              \
  template void launch_pack<T>(Grid&, const Params<T>&, const void*, void*, int, int);                       \
  template void launch_check_range<T>(Grid&, const void*, size_t);                                           \
  template void launch_cell_fill<T>(Grid&, const Params<T>&, void*, double, int, double);                    \
  template void launch_turb_multi<T>(const MultiCase<T>*, const CaseStarts&, int, int, int, const int*, int, hipStream_t);
UF_INST(float)
UF_INST(double)
#undef UF_INST

}  // namespace uf
