// Cell porosity of triangle-mesh objects (Sec. 3, urban model resolving):
// a bounding-box pass per object, then even-odd ray casting with the
// Moller-Trumbore ray/triangle test, with cut cells resolved by sub-sampling
// each cell sub x sub x sub times.
//
// The rays run along +x.  All sample points of a cell column that share
// (y, z) lie on one such line, so a thread casts ONE line per object: it
// tests the object's triangles once, keeps the sorted x of the crossings,
// and then classifies every sample on the line by the parity of the
// crossings to its right.  A block owns a tile of (j, k) cells of one
// object (sub^2 lines per cell, at most 256 lines), walks the object's
// x-range in chunks of cells, and adds its lines' inside counts per cell in
// LDS (integers: the result does not depend on the order).  Objects combine
// by the minimum porosity (an integer atomic min on the bit pattern, valid
// for non-negative values).
//
// Decisions (hit or miss, left or right of a crossing) are taken in FP64
// with contraction off, so the inside counts are reproducible bit for bit.
#include <algorithm>
#include <mutex>
#include <cmath>
#include <string>
#include <vector>

#include "uf_internal.h"

namespace uf {

constexpr int kVoxThreads = 256;
constexpr int kVoxMaxCross = 14;    // crossings kept per line and object
constexpr int kVoxCellChunk = 4;    // x-cells counted per LDS round
constexpr int kVoxChunk = 64;       // triangle records staged in LDS at a time
constexpr int kTriWords = 11;       // doubles of a record the ray test reads

// One triangle as the ray test uses it: the first vertex, the two edges
// from it and the reciprocal of the determinant for rays along +x (ok = 0
// for a triangle parallel to them).  Written once per call, then staged in
// LDS by the blocks, 64 records at a time, with coalesced loads.
struct alignas(128) TriRec {
  double v0[3], e1[3], e2[3], inv, ok, pad[5];
};

struct VoxItem {
  int obj;
  int i0, i1;     // x cells of the object's bounding box
  int j0, j1;     // the tile's y cells
  int k0, k1;     // the tile's z cells
};

__global__ __launch_bounds__(kVoxThreads) void k_mesh_check(const double* __restrict__ verts, int nverts,
                                                           const int* __restrict__ tris, int ntris, int* flag) {
  int bad = 0;
  const int stride = gridDim.x * blockDim.x;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntris; t += stride)
    for (int c = 0; c < 3; ++c) {
      const int v = tris[3 * t + c];
      if (v < 0 || v >= nverts) bad |= 1;
    }
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nverts; v += stride)
    for (int c = 0; c < 3; ++c)
      if (!isfinite(verts[3 * v + c])) bad |= 2;
  if (bad) atomicOr(flag, bad);
}

// Bounding box of each object's triangle vertices: one block per object.
__global__ __launch_bounds__(kVoxThreads) void k_mesh_aabb(const double* __restrict__ verts,
                                                          const int* __restrict__ tris,
                                                          const int* __restrict__ tri_begin, double* aabb) {
  __shared__ double sh[6][kVoxThreads];
  const int o = blockIdx.x;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int t = tri_begin[o] + threadIdx.x; t < tri_begin[o + 1]; t += blockDim.x)
    for (int c = 0; c < 3; ++c) {
      const double* p = verts + 3 * (size_t)tris[3 * t + c];
      for (int a = 0; a < 3; ++a) {
        lo[a] = fmin(lo[a], p[a]);
        hi[a] = fmax(hi[a], p[a]);
      }
    }
  for (int a = 0; a < 3; ++a) {
    sh[a][threadIdx.x] = lo[a];
    sh[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int a = 0; a < 3; ++a) {
        sh[a][threadIdx.x] = fmin(sh[a][threadIdx.x], sh[a][threadIdx.x + s]);
        sh[3 + a][threadIdx.x] = fmax(sh[3 + a][threadIdx.x], sh[3 + a][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) aabb[6 * o + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kVoxThreads) void k_mesh_prep(const double* __restrict__ verts,
                                                          const int* __restrict__ tris, int ntris,
                                                          TriRec* __restrict__ pre) {
#pragma clang fp contract(off)
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntris; t += gridDim.x * blockDim.x) {
    const double* a = verts + 3 * (size_t)tris[3 * t];
    const double* b = verts + 3 * (size_t)tris[3 * t + 1];
    const double* c = verts + 3 * (size_t)tris[3 * t + 2];
    TriRec r;
    for (int q = 0; q < 3; ++q) {
      r.v0[q] = a[q];
      r.e1[q] = b[q] - a[q];
      r.e2[q] = c[q] - a[q];
    }
    // P = D x E2 with D = +x; det = E1 . P
    const double det = -r.e1[1] * r.e2[2] + r.e1[2] * r.e2[1];
    r.ok = det != 0.0 ? 1.0 : 0.0;
    r.inv = det != 0.0 ? 1.0 / det : 0.0;
    for (int q = 0; q < 5; ++q) r.pad[q] = 0.0;
    pre[t] = r;
  }
}

template <class T>
__global__ __launch_bounds__(kVoxThreads) void k_fill_value(T* __restrict__ q, size_t n, T value) {
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x)
    q[c] = value;
}

__device__ __forceinline__ void atomic_min_nonneg(float* p, float v) {
  atomicMin(reinterpret_cast<unsigned int*>(p), __float_as_uint(v));
}
__device__ __forceinline__ void atomic_min_nonneg(double* p, double v) {
  atomicMin(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}

template <class T>
__global__ __launch_bounds__(kVoxThreads) void k_voxelize(const VoxItem* __restrict__ items,
                                                         const TriRec* __restrict__ pre,
                                                         const int* __restrict__ tri_begin,
                                                         const double* __restrict__ phi_obj, int ny, int nz,
                                                         double dx, double dy, double dz, int sub,
                                                         T* __restrict__ phi, int* flag) {
#pragma clang fp contract(off)
  __shared__ double s_x[kVoxMaxCross][kVoxThreads];
  __shared__ int s_cnt[kVoxCellChunk][kVoxThreads];
  __shared__ double s_tri[kVoxChunk][kTriWords + 1];

  const VoxItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int cj = it.j1 - it.j0, ck = it.k1 - it.k0;
  const int LK = ck * sub;
  const int nlines = cj * sub * LK;
  const bool act = tid < nlines;
  const int lj = act ? tid / LK : 0, lk = act ? tid % LK : 0;
  const int jc = it.j0 + lj / sub, kc = it.k0 + lk / sub;
  const int cell = (lj / sub) * ck + lk / sub;   // the thread's cell within the tile
  const double ys = ((double)jc + ((double)(lj % sub) + 0.5) / (double)sub) * dy;
  const double zs = ((double)kc + ((double)(lk % sub) + 0.5) / (double)sub) * dz;

  // crossings of this line with the object's surface
  int n = 0;
  bool over = false;
  const int t_begin = tri_begin[it.obj], t_end = tri_begin[it.obj + 1];
  for (int t0 = t_begin; t0 < t_end; t0 += kVoxChunk) {
    const int m = min(kVoxChunk, t_end - t0);
    __syncthreads();   // the previous chunk is done with
    for (int w = tid; w < m * kTriWords; w += kVoxThreads) {
      const int q = w / kTriWords, f = w % kTriWords;
      s_tri[q][f] = reinterpret_cast<const double*>(pre + t0 + q)[f];
    }
    __syncthreads();
    if (act) {
      for (int q = 0; q < m; ++q) {
        const double* r = s_tri[q];   // v0 (0..2), e1 (3..5), e2 (6..8), inv, ok
        if (r[10] == 0.0) continue;
        const double ty = ys - r[1], tz = zs - r[2];
        const double u = (-ty * r[8] + tz * r[7]) * r[9];
        const double qx = ty * r[5] - tz * r[4];
        const double v = qx * r[9];
        if (u >= 0.0 && v >= 0.0 && u + v <= 1.0) {
          const double xc = r[0] + u * r[3] + v * r[6];
          if (n < kVoxMaxCross) s_x[n][tid] = xc;
          else over = true;
          ++n;
        }
      }
    }
  }
  if (over) atomicOr(flag, 4);
  n = min(n, kVoxMaxCross);
  // sort the crossings (few per line)
  for (int a = 1; a < n; ++a) {
    const double x = s_x[a][tid];
    int b = a - 1;
    while (b >= 0 && s_x[b][tid] > x) {
      s_x[b + 1][tid] = s_x[b][tid];
      --b;
    }
    s_x[b + 1][tid] = x;
  }

  // walk the x cells: a sample is inside when an odd number of crossings
  // lies to its right
  const int ncell = cj * ck;
  const double rsub3 = (double)sub * (double)sub * (double)sub;
  const double solid = 1.0 - phi_obj[it.obj];
  int p = 0;
  for (int c0 = it.i0; c0 < it.i1; c0 += kVoxCellChunk) {
    const int cm = min(kVoxCellChunk, it.i1 - c0);
    for (int q = tid; q < kVoxCellChunk * kVoxThreads; q += kVoxThreads) (&s_cnt[0][0])[q] = 0;
    __syncthreads();
    if (act) {
      for (int ii = 0; ii < cm; ++ii) {
        int cnt = 0;
        for (int s = 0; s < sub; ++s) {
          const double xs = ((double)(c0 + ii) + ((double)s + 0.5) / (double)sub) * dx;
          while (p < n && s_x[p][tid] <= xs) ++p;
          cnt += (n - p) & 1;
        }
        if (cnt) atomicAdd(&s_cnt[ii][cell], cnt);
      }
    }
    __syncthreads();
    for (int q = tid; q < cm * ncell; q += kVoxThreads) {
      const int ii = q / ncell, cc = q % ncell;
      const int c = s_cnt[ii][cc];
      if (!c) continue;
      const double f = (double)c / rsub3;
      const T val = (T)(1.0 - f * solid);
      const int j = it.j0 + cc / ck, k = it.k0 + cc % ck;
      atomic_min_nonneg(&phi[((size_t)(c0 + ii) * ny + j) * nz + k], val);
    }
    __syncthreads();
  }
}

// Smoothed object indicator (design parameters move object faces within a
// cell continuously): per cell centre the product of logistic steps of
// width s across each object's faces (no lower step for objects standing on
// the ground), and the porosity min(1, min_o 1 - I_o (1 - phi_o)).  Objects:
// 8 doubles each, kind (0 box: x0 x1 y0 y1 z0 z1 phi; 1 cylinder: cx cy R
// z0 z1 phi), FP64 throughout.
__device__ __forceinline__ double logistic(double t) {
  const double e = exp(-fabs(t));
  return t >= 0.0 ? 1.0 / (1.0 + e) : e / (1.0 + e);
}

template <class T>
__global__ __launch_bounds__(kVoxThreads) void k_smooth_porosity(const double* __restrict__ obj, int nobj, int nx,
                                                                int ny, int nz, double dx, double dy, double dz,
                                                                double s, T* __restrict__ phi) {
  const size_t n = (size_t)nx * ny * nz;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(c % nz);
    const int j = (int)((c / nz) % ny);
    const int i = (int)(c / ((size_t)nz * ny));
    const double px = ((double)i + 0.5) * dx, py = ((double)j + 0.5) * dy, pz = ((double)k + 0.5) * dz;
    double v = 1.0;
    for (int o = 0; o < nobj; ++o) {
      const double* a = obj + 8 * o;
      double ind, po;
      if (a[7] == 0.0) {
        const double fx = logistic((px - a[0]) / s) * logistic((a[1] - px) / s);
        const double fy = logistic((py - a[2]) / s) * logistic((a[3] - py) / s);
        const double fz = logistic((a[5] - pz) / s) * (a[4] > 0.0 ? logistic((pz - a[4]) / s) : 1.0);
        ind = fx * fy * fz;
        po = a[6];
      } else {
        const double rho = sqrt((px - a[0]) * (px - a[0]) + (py - a[1]) * (py - a[1]));
        const double fr = logistic((a[2] - rho) / s);
        const double fz = logistic((a[4] - pz) / s) * (a[3] > 0.0 ? logistic((pz - a[3]) / s) : 1.0);
        ind = fr * fz;
        po = a[5];
      }
      v = fmin(v, 1.0 - ind * (1.0 - po));
    }
    phi[c] = (T)v;
  }
}

// Reverse of k_smooth_porosity.  A cell's porosity follows the first object
// reaching the minimum (none while it stays 1): phi = 1 - I (1 - phi_o), so
// dphi/dphi_o = I and dphi/dp = -(1 - phi_o) dI/dp for a face or radius
// parameter p, where dI/dp = I (1 - L) dt/dp for the logistic factor L(t)
// that holds p (1 - L(t) = L(-t), no division).  Each block sums
// phibar dphi/dp per object parameter (8 slots per object) in LDS and
// writes its row of partials; the host adds the rows in block order.  The
// sums take a fixed order, so the result is the same bits on every run: the
// block takes 256 cells at a time, each cell's object and seven terms go to
// LDS, and for each object present the first cell that holds it adds the
// terms of all its cells, in cell order, to that object's slots (no two
// threads write one slot).
__global__ __launch_bounds__(kVoxThreads) void k_smooth_porosity_grad(const double* __restrict__ obj, int nobj,
                                                                     int nx, int ny, int nz, double dx, double dy,
                                                                     double dz, double s,
                                                                     const double* __restrict__ phibar,
                                                                     double* __restrict__ part) {
  extern __shared__ double acc[];
  __shared__ int sb[kVoxThreads];           // object of each cell of the round (-1: none)
  __shared__ double sv[7][kVoxThreads];     // its seven terms phibar dphi/dp
  const int nslot = 8 * nobj;
  for (int q = threadIdx.x; q < nslot; q += blockDim.x) acc[q] = 0.0;
  const size_t n = (size_t)nx * ny * nz;
  const int t = threadIdx.x;
  for (size_t base = (size_t)blockIdx.x * blockDim.x; base < n; base += (size_t)gridDim.x * blockDim.x) {
    const size_t c = base + t;
    int bsel = -1;
    double term[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double pb = c < n ? phibar[c] : 0.0;
    if (pb != 0.0) {
      const int k = (int)(c % nz);
      const int j = (int)((c / nz) % ny);
      const int i = (int)(c / ((size_t)nz * ny));
      const double px = ((double)i + 0.5) * dx, py = ((double)j + 0.5) * dy, pz = ((double)k + 0.5) * dz;
      double v = 1.0;
      int best = -1;
      for (int o = 0; o < nobj; ++o) {
        const double* a = obj + 8 * o;
        double ind, po;
        if (a[7] == 0.0) {
          const double fx = logistic((px - a[0]) / s) * logistic((a[1] - px) / s);
          const double fy = logistic((py - a[2]) / s) * logistic((a[3] - py) / s);
          const double fz = logistic((a[5] - pz) / s) * (a[4] > 0.0 ? logistic((pz - a[4]) / s) : 1.0);
          ind = fx * fy * fz;
          po = a[6];
        } else {
          const double rho = sqrt((px - a[0]) * (px - a[0]) + (py - a[1]) * (py - a[1]));
          const double fr = logistic((a[2] - rho) / s);
          const double fz = logistic((a[4] - pz) / s) * (a[3] > 0.0 ? logistic((pz - a[3]) / s) : 1.0);
          ind = fr * fz;
          po = a[5];
        }
        const double val = 1.0 - ind * (1.0 - po);
        if (val < v) {
          v = val;
          best = o;
        }
      }
      if (best >= 0) {
        const double* a = obj + 8 * best;
        double d[7];   // dphi / d(parameter), in the object's parameter order
        if (a[7] == 0.0) {
          const double fx = logistic((px - a[0]) / s) * logistic((a[1] - px) / s);
          const double fy = logistic((py - a[2]) / s) * logistic((a[3] - py) / s);
          const double fz = logistic((a[5] - pz) / s) * (a[4] > 0.0 ? logistic((pz - a[4]) / s) : 1.0);
          const double ind = fx * fy * fz, m = -(1.0 - a[6]) * ind / s;
          d[0] = -m * logistic(-(px - a[0]) / s);
          d[1] = m * logistic(-(a[1] - px) / s);
          d[2] = -m * logistic(-(py - a[2]) / s);
          d[3] = m * logistic(-(a[3] - py) / s);
          d[4] = a[4] > 0.0 ? -m * logistic(-(pz - a[4]) / s) : 0.0;
          d[5] = m * logistic(-(a[5] - pz) / s);
          d[6] = ind;
        } else {
          const double ex = px - a[0], ey = py - a[1];
          const double rho = sqrt(ex * ex + ey * ey);
          const double fr = logistic((a[2] - rho) / s);
          const double fz = logistic((a[4] - pz) / s) * (a[3] > 0.0 ? logistic((pz - a[3]) / s) : 1.0);
          const double ind = fr * fz, m = -(1.0 - a[5]) * ind / s;
          const double dr = m * logistic(-(a[2] - rho) / s);   // along R; the centre moves rho by -e/rho
          d[0] = rho > 0.0 ? dr * ex / rho : 0.0;
          d[1] = rho > 0.0 ? dr * ey / rho : 0.0;
          d[2] = dr;
          d[3] = a[3] > 0.0 ? -m * logistic(-(pz - a[3]) / s) : 0.0;
          d[4] = m * logistic(-(a[4] - pz) / s);
          d[5] = ind;
          d[6] = 0.0;
        }
#pragma unroll
        for (int q = 0; q < 7; ++q) term[q] = pb * d[q];
        bsel = best;
      }
    }
    __syncthreads();   // the previous round's reduction is done with sb, sv
    sb[t] = bsel;
#pragma unroll
    for (int q = 0; q < 7; ++q) sv[q][t] = term[q];
    __syncthreads();
    // the first cell of the round holding its object reduces that object
    bool lead = bsel >= 0 && (t == 0 || sb[t - 1] != bsel);
    for (int u = 0; lead && u < t - 1; ++u) lead = sb[u] != bsel;
    if (lead) {
      double sum[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (int u = t; u < (int)blockDim.x; ++u) {
        if (sb[u] != bsel) continue;
#pragma unroll
        for (int q = 0; q < 7; ++q) sum[q] += sv[q][u];
      }
#pragma unroll
      for (int q = 0; q < 7; ++q) acc[8 * bsel + q] += sum[q];
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nslot; q += blockDim.x) part[(size_t)blockIdx.x * nslot + q] = acc[q];
}

namespace {
struct DevBuf {
  void* p = nullptr;
  explicit DevBuf(size_t bytes) {
    if (bytes) UF_HIP_CHECK(hipMalloc(&p, bytes));
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  template <class X>
  X* as() const {
    return static_cast<X*>(p);
  }
};

// Cells an interval overlaps, clamped to [0, n] in floating point first (so
// far-away coordinates cannot overflow the integer conversion).
int cell_lo(double v, double h, int n) { return (int)std::min(std::max(std::floor(v / h), 0.0), (double)n); }
int cell_hi(double v, double h, int n) { return (int)std::max(std::min(std::ceil(v / h), (double)n), 0.0); }
}  // namespace

// Host side of uf_voxelize (arguments validated by the caller).  Returns an
// empty string, or the message of an input error found on the device.
std::string voxelize_run(const uf_mesh_set& m, int dtype, void* phi, hipStream_t stream, double* cast_ms) {
  if (cast_ms) *cast_ms = 0.0;
  const size_t ncells = (size_t)m.nx * m.ny * m.nz;
  const int fill_blocks = (int)std::min<size_t>(4096, (ncells + kVoxThreads - 1) / kVoxThreads);
  DevBuf flag(sizeof(int));
  UF_HIP_CHECK(hipMemsetAsync(flag.p, 0, sizeof(int), stream));
  if (m.ntris > 0 || m.nverts > 0) {
    const int blocks = std::max(1, std::min(1024, (std::max(m.ntris, m.nverts) + kVoxThreads - 1) / kVoxThreads));
    hipLaunchKernelGGL(k_mesh_check, dim3(blocks), dim3(kVoxThreads), 0, stream, m.verts_dev, m.nverts,
                       m.tris_dev, m.ntris, flag.as<int>());
  }
  int hflag = 0;
  UF_HIP_CHECK(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, stream));
  UF_HIP_CHECK(hipStreamSynchronize(stream));
  if (hflag & 1) return "a triangle refers to a vertex index outside [0, nverts)";
  if (hflag & 2) return "a vertex coordinate is not finite";

  if (dtype == UF_F32)
    hipLaunchKernelGGL(k_fill_value<float>, dim3(fill_blocks), dim3(kVoxThreads), 0, stream, (float*)phi, ncells,
                       1.0f);
  else
    hipLaunchKernelGGL(k_fill_value<double>, dim3(fill_blocks), dim3(kVoxThreads), 0, stream, (double*)phi, ncells,
                       1.0);
  if (m.nobj == 0 || m.ntris == 0) {
    UF_HIP_CHECK(hipGetLastError());
    UF_HIP_CHECK(hipStreamSynchronize(stream));
    return "";
  }

  // first pass: bounding boxes (and the triangles in the form the ray test reads)
  DevBuf begin(sizeof(int) * (m.nobj + 1)), aabb(sizeof(double) * 6 * m.nobj), pobj(sizeof(double) * m.nobj);
  DevBuf pre(sizeof(TriRec) * (size_t)m.ntris);
  hipLaunchKernelGGL(k_mesh_prep, dim3(std::max(1, std::min(4096, (m.ntris + kVoxThreads - 1) / kVoxThreads))),
                     dim3(kVoxThreads), 0, stream, m.verts_dev, m.tris_dev, m.ntris, pre.as<TriRec>());
  UF_HIP_CHECK(hipMemcpyAsync(begin.p, m.tri_begin, sizeof(int) * (m.nobj + 1), hipMemcpyHostToDevice, stream));
  UF_HIP_CHECK(hipMemcpyAsync(pobj.p, m.phi_obj, sizeof(double) * m.nobj, hipMemcpyHostToDevice, stream));
  hipLaunchKernelGGL(k_mesh_aabb, dim3(m.nobj), dim3(kVoxThreads), 0, stream, m.verts_dev, m.tris_dev,
                     begin.as<int>(), aabb.as<double>());
  UF_HIP_CHECK(hipGetLastError());
  std::vector<double> box(6 * (size_t)m.nobj);
  UF_HIP_CHECK(hipMemcpyAsync(box.data(), aabb.p, sizeof(double) * box.size(), hipMemcpyDeviceToHost, stream));
  UF_HIP_CHECK(hipStreamSynchronize(stream));

  // second pass: one work item per object and tile of (j, k) cells
  const int tc = std::max(1, 16 / m.sub);   // tile side in cells: (tc sub)^2 <= 256 lines
  std::vector<VoxItem> items;
  for (int o = 0; o < m.nobj; ++o) {
    if (m.tri_begin[o + 1] == m.tri_begin[o]) continue;
    const double* b = &box[6 * (size_t)o];
    const int i0 = cell_lo(b[0], m.dx, m.nx), i1 = cell_hi(b[3], m.dx, m.nx);
    const int j0 = cell_lo(b[1], m.dy, m.ny), j1 = cell_hi(b[4], m.dy, m.ny);
    const int k0 = cell_lo(b[2], m.dz, m.nz), k1 = cell_hi(b[5], m.dz, m.nz);
    if (i0 >= i1 || j0 >= j1 || k0 >= k1) continue;
    for (int j = j0; j < j1; j += tc)
      for (int k = k0; k < k1; k += tc)
        items.push_back(VoxItem{o, i0, i1, j, std::min(j + tc, j1), k, std::min(k + tc, k1)});
  }
  if (!items.empty()) {
    DevBuf ditems(sizeof(VoxItem) * items.size());
    UF_HIP_CHECK(hipMemcpyAsync(ditems.p, items.data(), sizeof(VoxItem) * items.size(), hipMemcpyHostToDevice,
                                stream));
    struct Events {
      hipEvent_t e[2] = {nullptr, nullptr};
      ~Events() {
        for (auto& x : e)
          if (x) (void)hipEventDestroy(x);
      }
    } evs;
    hipEvent_t* ev = evs.e;
    if (cast_ms)
      for (int q = 0; q < 2; ++q) UF_HIP_CHECK(hipEventCreate(&ev[q]));
    if (dtype == UF_F32)
      hipExtLaunchKernelGGL(k_voxelize<float>, dim3((unsigned)items.size()), dim3(kVoxThreads), 0, stream, ev[0],
                            ev[1], 0, ditems.as<VoxItem>(), pre.as<TriRec>(), begin.as<int>(),
                            pobj.as<double>(), m.ny, m.nz, m.dx, m.dy, m.dz, m.sub, (float*)phi, flag.as<int>());
    else
      hipExtLaunchKernelGGL(k_voxelize<double>, dim3((unsigned)items.size()), dim3(kVoxThreads), 0, stream, ev[0],
                            ev[1], 0, ditems.as<VoxItem>(), pre.as<TriRec>(), begin.as<int>(),
                            pobj.as<double>(), m.ny, m.nz, m.dx, m.dy, m.dz, m.sub, (double*)phi, flag.as<int>());
    UF_HIP_CHECK(hipGetLastError());
    UF_HIP_CHECK(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, stream));
    UF_HIP_CHECK(hipStreamSynchronize(stream));
    if (cast_ms) {
      float ms = 0.0f;
      UF_HIP_CHECK(hipEventElapsedTime(&ms, ev[0], ev[1]));
      *cast_ms = ms;
    }
    if (hflag & 4) return "a sample line crosses an object's surface more than 14 times";
  } else {
    UF_HIP_CHECK(hipStreamSynchronize(stream));
  }
  return "";
}

}  // namespace uf

namespace uf {

void smooth_porosity_run(const uf_smooth_objects& o, int dtype, void* phi, hipStream_t stream) {
  std::vector<double> obj;
  for (int b = 0; b < o.nboxes; ++b) {
    for (int q = 0; q < 7; ++q) obj.push_back(o.boxes[7 * b + q]);
    obj.push_back(0.0);
  }
  for (int c = 0; c < o.ncyls; ++c) {
    for (int q = 0; q < 6; ++q) obj.push_back(o.cylinders[6 * c + q]);
    obj.push_back(0.0);
    obj.push_back(1.0);
  }
  const int nobj = o.nboxes + o.ncyls;
  DevBuf dobj(sizeof(double) * std::max<size_t>(obj.size(), 1));
  if (!obj.empty())
    UF_HIP_CHECK(hipMemcpyAsync(dobj.p, obj.data(), sizeof(double) * obj.size(), hipMemcpyHostToDevice, stream));
  const size_t n = (size_t)o.nx * o.ny * o.nz;
  const int blocks = (int)std::min<size_t>(8192, (n + kVoxThreads - 1) / kVoxThreads);
  if (dtype == UF_F32)
    hipLaunchKernelGGL(k_smooth_porosity<float>, dim3(blocks), dim3(kVoxThreads), 0, stream, dobj.as<double>(), nobj,
                       o.nx, o.ny, o.nz, o.dx, o.dy, o.dz, o.width, (float*)phi);
  else
    hipLaunchKernelGGL(k_smooth_porosity<double>, dim3(blocks), dim3(kVoxThreads), 0, stream, dobj.as<double>(),
                       nobj, o.nx, o.ny, o.nz, o.dx, o.dy, o.dz, o.width, (double*)phi);
  UF_HIP_CHECK(hipGetLastError());
  UF_HIP_CHECK(hipStreamSynchronize(stream));
}

}  // namespace uf

namespace uf {

// Host side of uf_smooth_porosity_grad (arguments validated by the caller).
void smooth_porosity_grad_run(const uf_smooth_objects& o, const double* phibar, double* grad, hipStream_t stream) {
  std::vector<double> obj;
  for (int b = 0; b < o.nboxes; ++b) {
    for (int q = 0; q < 7; ++q) obj.push_back(o.boxes[7 * b + q]);
    obj.push_back(0.0);
  }
  for (int c = 0; c < o.ncyls; ++c) {
    for (int q = 0; q < 6; ++q) obj.push_back(o.cylinders[6 * c + q]);
    obj.push_back(0.0);
    obj.push_back(1.0);
  }
  const int nobj = o.nboxes + o.ncyls;
  const int ng = 7 * o.nboxes + 6 * o.ncyls;
  for (int q = 0; q < ng; ++q) grad[q] = 0.0;
  if (nobj == 0) return;
  const size_t n = (size_t)o.nx * o.ny * o.nz;
  const int blocks = (int)std::min<size_t>(1024, (n + kVoxThreads - 1) / kVoxThreads);
  const size_t nslot = 8 * (size_t)nobj;
  DevBuf dobj(sizeof(double) * obj.size());
  DevBuf dpart(sizeof(double) * nslot * blocks);
  UF_HIP_CHECK(hipMemcpyAsync(dobj.p, obj.data(), sizeof(double) * obj.size(), hipMemcpyHostToDevice, stream));
  hipLaunchKernelGGL(k_smooth_porosity_grad, dim3(blocks), dim3(kVoxThreads), sizeof(double) * nslot, stream,
                     dobj.as<double>(), nobj, o.nx, o.ny, o.nz, o.dx, o.dy, o.dz, o.width, phibar,
                     dpart.as<double>());
  UF_HIP_CHECK(hipGetLastError());
  std::vector<double> part(nslot * blocks);
  UF_HIP_CHECK(hipMemcpyAsync(part.data(), dpart.p, sizeof(double) * part.size(), hipMemcpyDeviceToHost, stream));
  UF_HIP_CHECK(hipStreamSynchronize(stream));
  std::vector<double> tot(nslot, 0.0);
  for (int b = 0; b < blocks; ++b)
    for (size_t q = 0; q < nslot; ++q) tot[q] += part[(size_t)b * nslot + q];
  for (int b = 0; b < o.nboxes; ++b)
    for (int q = 0; q < 7; ++q) grad[7 * b + q] = tot[8 * b + q];
  for (int c = 0; c < o.ncyls; ++c)
    for (int q = 0; q < 6; ++q) grad[7 * o.nboxes + 6 * c + q] = tot[8 * (o.nboxes + c) + q];
}

}  // namespace uf

// ------------------------------------------ allocation-free porosity gradient
// uf_smooth_porosity_grad_noalloc works in one fixed device array per GPU
// instead of allocating: the caller's box and cylinder rows, the packed
// objects the gradient kernel reads, the per-block partial rows and the
// summed gradient.  8 MiB, held by each GPU the library runs on until the
// process ends.  Every call on a GPU reuses it, so calls that overlap on one
// GPU (several host threads, or streams not ordered with each other) race.
namespace uf {

constexpr size_t kScratchDoubles = size_t(1) << 20;
constexpr size_t kScrMaxObj = UF_NOALLOC_MAX_OBJECTS;
constexpr size_t kScrBoxes = 0;                         // 7 per box, as the caller passes them
constexpr size_t kScrCyls = kScrBoxes + 7 * kScrMaxObj; // 6 per cylinder
constexpr size_t kScrPacked = kScrCyls + 6 * kScrMaxObj;  // 8 per object
constexpr size_t kScrGrad = kScrPacked + 8 * kScrMaxObj;  // 7 per box, then 6 per cylinder
constexpr size_t kScrPart = 32 * kScrMaxObj;            // partial rows, to the end
static_assert(kScrGrad + 7 * kScrMaxObj <= kScrPart, "scratch regions overlap");
static_assert(kScrPart % 32 == 0, "partial rows start 256-byte aligned");

static __device__ __align__(256) double scratch[kScratchDoubles];

// The objects in the form k_smooth_porosity_grad reads: a box is its seven
// values and a zero, a cylinder its six values, a zero and a one (the mark
// that tells the two kinds apart).
__global__ __launch_bounds__(kVoxThreads) void k_pack_objects(const double* __restrict__ boxes, int nb,
                                                              const double* __restrict__ cyls, int nc,
                                                              double* __restrict__ obj) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nb + nc) return;
  double* dst = obj + 8 * (size_t)o;
  if (o < nb) {
    for (int q = 0; q < 7; ++q) dst[q] = boxes[7 * (size_t)o + q];
    dst[7] = 0.0;
  } else {
    const double* src = cyls + 6 * (size_t)(o - nb);
    for (int q = 0; q < 6; ++q) dst[q] = src[q];
    dst[6] = 0.0;
    dst[7] = 1.0;
  }
}

// Sum of the partial rows, block by block in block order (one thread per
// gradient entry), into the caller's order: 7 per box, then 6 per cylinder.
__global__ __launch_bounds__(kVoxThreads) void k_sum_rows(const double* __restrict__ part, int rows, int nslot,
                                                          int nb, int nc, double* __restrict__ grad) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int ng = 7 * nb + 6 * nc;
  if (q >= ng) return;
  const int slot = q < 7 * nb ? 8 * (q / 7) + q % 7 : 8 * (nb + (q - 7 * nb) / 6) + (q - 7 * nb) % 6;
  double s = 0.0;
  for (int b = 0; b < rows; ++b) s += part[(size_t)b * nslot + slot];
  grad[q] = s;
}

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxScratchDevices] = {};

// Device address of this GPU's scratch, looked up once per device with that
// device current.  Host code uses this address only: the array's own name
// is a host-side stand-in.
double* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxScratchDevices) throw HipError("device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    UF_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw HipError("hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  return g_scratch_dev[dev];
}
}  // namespace

// Host side of uf_smooth_porosity_grad_noalloc (arguments validated by the
// caller, at most kScrMaxObj objects; the current device is the stream's).
void smooth_porosity_grad_noalloc_run(const uf_smooth_objects& o, const double* phibar, double* grad,
                                      hipStream_t stream) {
  const int nb = o.nboxes, nc = o.ncyls, nobj = nb + nc;
  const int ng = 7 * nb + 6 * nc;
  for (int q = 0; q < ng; ++q) grad[q] = 0.0;
  if (nobj == 0) return;
  int dev = 0;
  UF_HIP_CHECK(hipGetDevice(&dev));
  double* s = scratch_on(dev);
  const size_t n = (size_t)o.nx * o.ny * o.nz;
  const size_t nslot = 8 * (size_t)nobj;
  const size_t fit = (kScratchDoubles - kScrPart) / nslot;   // partial rows the scratch holds (>= 124)
  const int blocks = (int)std::min<size_t>(std::min<size_t>(1024, (n + kVoxThreads - 1) / kVoxThreads), fit);
  if (nb) UF_HIP_CHECK(hipMemcpyAsync(s + kScrBoxes, o.boxes, sizeof(double) * 7 * nb, hipMemcpyHostToDevice, stream));
  if (nc)
    UF_HIP_CHECK(hipMemcpyAsync(s + kScrCyls, o.cylinders, sizeof(double) * 6 * nc, hipMemcpyHostToDevice, stream));
  const int ob = (nobj + kVoxThreads - 1) / kVoxThreads;
  hipLaunchKernelGGL(k_pack_objects, dim3(ob), dim3(kVoxThreads), 0, stream, s + kScrBoxes, nb, s + kScrCyls, nc,
                     s + kScrPacked);
  hipLaunchKernelGGL(k_smooth_porosity_grad, dim3(blocks), dim3(kVoxThreads), sizeof(double) * nslot, stream,
                     s + kScrPacked, nobj, o.nx, o.ny, o.nz, o.dx, o.dy, o.dz, o.width, phibar, s + kScrPart);
  hipLaunchKernelGGL(k_sum_rows, dim3((ng + kVoxThreads - 1) / kVoxThreads), dim3(kVoxThreads), 0, stream,
                     s + kScrPart, blocks, (int)nslot, nb, nc, s + kScrGrad);
  UF_HIP_CHECK(hipGetLastError());
  UF_HIP_CHECK(hipMemcpyAsync(grad, s + kScrGrad, sizeof(double) * ng, hipMemcpyDeviceToHost, stream));
  UF_HIP_CHECK(hipStreamSynchronize(stream));
}

}  // namespace uf
