// Host-side grid object and the launchers of the step kernels.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/uf.h"
#include "uf_device.h"

namespace uf {

// State of one pressure solve, kept in device memory and updated by block 0
// of the CG kernels (deterministic FP64 reductions).
struct CgState {
  double bb;         // ||b||^2
  double rr;         // ||r||^2 after the last update
  double rzh[2];     // r.z of iteration t in rzh[t & 1], published by block 0 of the d/q kernel
  double tol2_bb;    // stopping threshold on ||r||^2 (criterion 0) or r.z (criterion 1)
  int iter;          // iterations done
  int done;          // 1 once converged, stopped at maxit, or non-finite
  int noconv;        // stopped at maxit
  int nonfinite;     // NaN/Inf seen
  int zero_rhs;      // b == 0: the solution is 0
  int maxit;
  int criterion;
  int nf_state;      // 1 once the drag or k-omega stage wrote a NaN/Inf (sticky; the solves leave it)
  int restart;       // 1 when the initial guess was worse than zero and the solve started from x = 0
};

// One level of the multigrid hierarchy (level 0 is the fine grid).
struct MgLevel {
  Layout L;
  double w[3] = {0, 0, 0};   // stencil weight per axis (1/h^2 on level 0)
  int coarsen[3] = {0, 0, 0};// 1 if this axis is halved towards the next level
  void* x = nullptr;         // correction
  void* r = nullptr;         // right-hand side (restricted residual)
  void* t = nullptr;         // scratch
};

// Launch shape of the d/q kernel: tiles of (512 / kt) x kt columns, njt x nkt
// of them per plane, gy chunks of ilen planes.
struct AdLaunch {
  dim3 grid;
  int kt, njt, nkt, ilen, gy, blocks;
};
AdLaunch ad_launch(const Layout& L);

struct CgLaunch {
  dim3 grid;   // 1-D launch of the logical gx x gy blocks (see xcd_block)
  int ilen;    // x-planes marched by each block
  int gx, gy;
};

// One case of a batched launch (uf_batch): its step parameters and buffers.
template <class T>
struct MultiCase {
  Params<T> P;
  T* q[3][3];        // the grid's three (u, v, w) sets
  T* nut;
  const T* cc;       // drag coefficient per cell
  const T* x;        // pressure
  T* k[2];
  T* w[2];
  int* nf;           // the state's non-finite flag
};

// Face stages of the batched launch.
enum { MS_ADVECT_FWD = 0, MS_ADVECT_CORR, MS_DIFFUSE, MS_DRAG, MS_PROJECT, MS_NFACE };

// Most cases of one batch.
constexpr int kMaxBatchCases = UF_BATCH_MAX_GRIDS;

// Where each case's logical blocks start in a batched launch's queue
// (ascending, start[n] = all blocks).  Passed by value, so that a block
// finds its case in the kernel's argument segment.
struct CaseStarts {
  int n;
  int start[kMaxBatchCases + 1];
};

// The case owning logical block lb: the largest c with start[c] <= lb.
__host__ __device__ inline int find_case(const CaseStarts& cs, int lb) {
  int lo = 0, hi = cs.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cs.start[mid] <= lb) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct Grid {
  uf_config cfg{};
  std::vector<double> profile;
  int bc[6];
  Layout L{};
  size_t nelem = 0;          // padded elements per field
  size_t esize = 4;          // bytes per element
  hipStream_t stream = nullptr;
  // device buffers (element type = dtype)
  void* Q[3][3] = {};        // three sets of (u, v, w)
  int cur = 0;               // set holding the state
  void* K[2] = {};
  void* Wo[2] = {};
  int kcur = 0;
  void* NUT = nullptr;
  void* C = nullptr;         // drag coefficient per cell
  void* PHI = nullptr;       // porosity, compact nx*ny*nz
  void* inflow = nullptr;    // [2][nz+2]
  // pressure solve
  void* X = nullptr;         // pressure (the CG iterate)
  void* R = nullptr;         // residual after an even number of updates
  void* R2 = nullptr;        // ... after an odd number (the update reads one, writes the other)
  void* Z = nullptr;
  void* D[2] = {};
  void* Qv = nullptr;
  void* Xsave = nullptr;        // the pressure state kept across uf_pressure_solve (allocated on first use)
  int dpar = 0;
  double* partials = nullptr;   // 5 slots of part_stride partial sums
  double* obj_part = nullptr;   // objective partials (allocated on first use)
  void* obj_meta = nullptr;     // region boxes and seed coefficients of the objective gradient
  // adjoint workspace (allocated on the first uf_adjoint_step)
  void* AS[4][3] = {};          // recomputed forward: state n, predictor, advected, diffused
  void* AA[3][3] = {};          // adjoint work sets
  void* AV[3][3] = {};          // per-face velocity-vector adjoints (zero outside the face thread range)
  void* AT[10] = {};            // k-omega reverse: k, omega, nu_t of step n; their adjoints at n+1 and
                                // at n; the pressure of the forward recompute
  int fwd_last_iters = 0;
  void* AU[2][3] = {};          // recomputed u* and u^{n+1}
  void* Cbar = nullptr;         // drag-coefficient adjoint (padded cells)
  void* XA = nullptr;           // adjoint pressure, the warm start of the next adjoint solve
  void* inflow0 = nullptr;      // zero inflow table (homogeneous boundary values)
  int adj_last_iters = 0;
  size_t part_stride = 0;
  size_t cg_nb = 0;             // blocks of the fine-grid CG kernels
  size_t cg_nb_rz = 0;          // blocks of the kernel that writes the r.z partials
  size_t cg_nb_dq = 0;          // blocks of the d/q kernel
  size_t cg_nb_rr = 0;          // partials of the r.r slot (the largest of its writers)
  bool mg_fused = false;        // CG update folded into the level-0 restriction
  int* flags = nullptr;         // [cg_maxit + 2]
  int* exec = nullptr;          // [cg_maxit + 2]
  CgState* st = nullptr;     // device
  CgState* st_host = nullptr;  // pinned
  int* flag = nullptr;       // device int used by validation kernels
  int* flag_host = nullptr;  // pinned
  double* diag = nullptr;    // [3][kDiagBlocks] partials of the end-of-call diagnostics
  double* diag_host = nullptr;  // pinned copy
  hipEvent_t ev_status = nullptr, ev0 = nullptr, ev1 = nullptr;
  // second stream of the pressure solve: the iterate's update x += alpha d
  // of a CG iteration runs there beside the coarse multigrid levels, forked
  // after the level-0 restriction and joined before the next iteration
  hipStream_t xstream = nullptr;
  hipEvent_t ev_xfork = nullptr, ev_xjoin = nullptr;
  bool xpending = false;        // an update on xstream not yet joined (join_x)
  std::vector<MgLevel> mg;
  int mg_lt = 0;                // first level of the single-workgroup kernel
  bool mg_tail_lds = true;      // the small levels fit the LDS pool of the single-workgroup kernel
  int mg_nc = 0;                // cells of the coarsest level
  void* mg_cinv = nullptr;      // dense inverse of the coarsest operator
  void* mg_table = nullptr;     // device copy of the level descriptors
  double mg_omega = 0.8;        // Jacobi weight of the smoother
  int last_iters = 0;
  int cg_t = 0;                 // CG iterations enqueued in the current solve
  // kernel timer (see uf_kernel_timer_enable)
  uint32_t timer_mask = 0;
  std::vector<hipEvent_t> timer_pool;
  std::vector<int> timer_id;       // kernel of each recorded pair
  size_t timer_used = 0;           // pairs recorded since the last flush
  int timer_cur = -1;              // timer id of the launch in the current TimedLaunch scope
  double timer_ms[UF_TK_COUNT] = {};
  long long timer_n[UF_TK_COUNT] = {};
  int k_in_valid = 1;
  double k_in = 0, w_in = 0, nu_max = 0;
};

// Make the grid's stream wait for the iterate update last forked onto the
// second solve stream, if it has not yet: before the next iteration's d/q
// kernel (which overwrites the d that update reads) and before anything
// reads the pressure after a solve.  The solve's status check runs before
// the join, beside the last update.
void join_x(Grid& g);

// Device memory of the grid: its configured allocator, else hipMalloc.
void* galloc(Grid& g, size_t bytes);
void gfree(Grid& g, void* p);
// Host data to the grid's device memory, in order on the grid's stream;
// returns when the copy is complete.  (A plain hipMemcpy runs on the null
// stream, which is not ordered with a non-blocking grid stream.)
void upload(Grid& g, void* dst, const void* src, size_t bytes);

// End-of-call diagnostics (uf_step_stats.max_div, max_cfl, nut_clip_frac).
constexpr int kDiagBlocks = 512;
template <class T> void launch_diag(Grid& g, const Params<T>& P);

// Residual buffer after m CG updates.
inline void* resid(const Grid& g, int m) { return (m & 1) ? g.R2 : g.R; }

// Launchers (T = float or double), defined in the kernel sources.
template <class T> Params<T> make_params(const Grid& g);
template <class T> void launch_advect(Grid& g, const Params<T>& P, void* const Qin[3], void* const Qhat[3], void* const Qout[3]);
template <class T> void launch_diffuse(Grid& g, const Params<T>& P, void* const Qin[3], void* const Qout[3]);
template <class T> void launch_drag(Grid& g, const Params<T>& P, void* const Qin[3], void* const Qout[3]);
template <class T> void launch_project(Grid& g, const Params<T>& P, void* const Qin[3], void* const Qout[3], const int* gate = nullptr);
template <class T> void launch_face_bc(Grid& g, const Params<T>& P, void* q, int comp);
template <class T> void launch_turb(Grid& g, const Params<T>& P, void* const Q[3], const void* K0, const void* W0, void* K1, void* W1, void* NUT, int update_kw, const int* gate = nullptr);
// device word the drag and k-omega kernels set on a non-finite output
inline int* nf_word(Grid& g) { return &g.st->nf_state; }
template <class T> void launch_cell_bc(Grid& g, const Params<T>& P, void* q, int use_inlet, double inlet_value);
// batched launches (one persistent launch for every case of a batch)
template <class T>
void launch_faces_multi(int stage, const MultiCase<T>* mc, const CaseStarts& cs, int band, int blocks, int sin,
                        int saux, int sout, hipStream_t stream);
template <class T>
void launch_turb_multi(const MultiCase<T>* mc, const CaseStarts& cs, int band, int blocks, int sq, const int* kcs,
                       int nut_set, hipStream_t stream);
int cell_queue_blocks(const Layout& L);
template <class T> void launch_porosity(Grid& g, const Params<T>& P, const void* phi);
template <class T> void launch_pack(Grid& g, const Params<T>& P, const void* src_padded, void* dst, int field, int unpack);
template <class T> void launch_check_range(Grid& g, const void* phi, size_t n);
// pressure solve
CgLaunch cg_launch(const Layout& L);
template <class T> void launch_cg_start(Grid& g, const Params<T>& P, void* const Qs[3], const void* b);
template <class T> void launch_cg_precond(Grid& g, const Params<T>& P, int m);
template <class T> void launch_cg_iteration(Grid& g, const Params<T>& P, int t);
void launch_cg_status(Grid& g, int t_end);
template <class T> void launch_apply(Grid& g, const Params<T>& P, int op, const void* x, void* y);
template <class T> void launch_region_speed(Grid& g, const int box[6], double* part, int nblocks);
template <class T>
void launch_region_field_diff(Grid& g, const int box[6], const void* ut, double* part, int nblocks);
template <class T>
void launch_plane_objective(Grid& g, int k0, double t, double st, double smin, double wpen, double* part,
                            int nblocks);
std::string voxelize_run(const uf_mesh_set& m, int dtype, void* phi, hipStream_t stream, double* cast_ms);
void smooth_porosity_run(const uf_smooth_objects& o, int dtype, void* phi, hipStream_t stream);
void smooth_porosity_grad_run(const uf_smooth_objects& o, const double* phibar, double* grad, hipStream_t stream);
void smooth_porosity_grad_noalloc_run(const uf_smooth_objects& o, const double* phibar, double* grad,
                                      hipStream_t stream);
// reverse (adjoint) stages
template <class T> void launch_advect_adj(Grid& g, const Params<T>& P, void* const Qin[3], void* const Qhat[3], void* const Aout[3], void* const Gq[3], void* const Ghat[3]);
template <class T> void launch_diffuse_adj(Grid& g, const Params<T>& P, void* const Aout[3], void* const Gin[3]);
template <class T> void launch_drag_adj(Grid& g, const Params<T>& P, void* const Qin[3], void* const Aout[3], void* const Gin[3], void* Cbar);
template <class T> void launch_fold(Grid& g, const Params<T>& P, void* const A[3]);
template <class T> void launch_drag_coef_adj(Grid& g, const Params<T>& P, const void* Cbar, double* phibar);
template <class T> void launch_objective_seed(Grid& g, const Params<T>& P, const int* boxes_dev, const double* coef_dev, int nreg, int kind, const void* ut, void* out, const double plane[6], double* phibar);
template <class T> void launch_turb_adj(Grid& g, const Params<T>& P, void* const Unew[3], const void* K0, const void* W0, const void* KB1, const void* WB1, const void* NB1, void* KB0, void* WB0, void* const G[3]);
template <class T> void launch_cell_fold(Grid& g, const Params<T>& P, void* q, int use_inlet);
template <class T> void launch_diffuse_nut_adj(Grid& g, const Params<T>& P, void* const Qin[3], void* const Aout[3], void* NB);
template <class T> void mg_setup(Grid& g);
template <class T> void mg_precond(Grid& g, const Params<T>& P, int m);
template <class T> void mg_iteration_update(Grid& g, const Params<T>& P, int t, const void* Dnew);
size_t mg_fused_blocks(const Grid& g);
// Whether the CG iterations run x += alpha d on the second solve stream
// (the level-0 restriction marches and carries the residual update only).
bool mg_splits_update(const Grid& g);
template <class T> void mg_apply(Grid& g, const Params<T>& P, const void* r, void* z);
void mg_free(Grid& g);

// Marks the one kernel launched (through launch_k) in its scope as kernel
// id of the timer.
struct TimedLaunch {
  Grid& g;
  int prev;
  TimedLaunch(Grid& g_, int id_);
  ~TimedLaunch();
};
void timer_flush(Grid& g);
// Start/stop events for the launch being made, when the kernel timer covers
// it (the pair is then recorded for the next timer_flush); else false.
bool timer_pair(Grid& g, hipEvent_t* e0, hipEvent_t* e1);

// Launch on g.stream.  A timed launch carries its events in the dispatch
// itself, so they time the kernel alone (no separate marker packets).
template <typename... Args, typename... A>
inline void launch_k(Grid& g, void (*kernel)(Args...), dim3 grid, dim3 block, A... args);

size_t padded_bytes(const Grid& g);
void set_error(const std::string& msg);
const char* hip_error_name(hipError_t e);

}  // namespace uf

#define UF_HIP_CHECK(expr)                                                        \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess) {                                                       \
      throw uf::HipError(std::string(#expr) + ": " + hipGetErrorString(_e));      \
    }                                                                             \
  } while (0)

namespace uf {
struct HipError {
  std::string msg;
  explicit HipError(std::string m) : msg(std::move(m)) {}
};
template <typename... Args, typename... A>
inline void launch_k(Grid& g, void (*kernel)(Args...), dim3 grid, dim3 block, A... args) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timer_pair(g, &e0, &e1))
    hipExtLaunchKernelGGL(kernel, grid, block, 0, g.stream, e0, e1, 0, static_cast<Args>(args)...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, g.stream, static_cast<Args>(args)...);
}

// launch_k whose dispatch also completes an event, for another stream to
// wait on: `done`, or the timer's stop event when the kernel timer covers
// the launch (returned).  Outside stream capture the event travels in the
// dispatch itself; a separate record would put a marker packet between
// this kernel and the next one on g.stream (about 6 us at the queue).
template <typename... Args, typename... A>
inline hipEvent_t launch_k_done(Grid& g, hipEvent_t done, void (*kernel)(Args...), dim3 grid, dim3 block,
                                A... args) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  UF_HIP_CHECK(hipStreamIsCapturing(g.stream, &cap));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timer_pair(g, &e0, &e1)) {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, g.stream, e0, e1, 0, static_cast<Args>(args)...);
    return e1;
  }
  if (cap != hipStreamCaptureStatusNone) {
    hipLaunchKernelGGL(kernel, grid, block, 0, g.stream, static_cast<Args>(args)...);
    UF_HIP_CHECK(hipEventRecord(done, g.stream));
  } else {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, g.stream, nullptr, done, 0, static_cast<Args>(args)...);
  }
  return done;
}

}  // namespace uf
