// C ABI of the RANS step library: grid creation and validation, state I/O,
// the time-step driver and the pressure-CG host loop.  See include/uf.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "face_ops.h"
#include "uf_internal.h"

namespace uf {

static thread_local std::string g_last_error;
void set_error(const std::string& m) { g_last_error = m; }

size_t mg_fine_blocks(const Layout& L);
template <class T> void launch_face_init(Grid& g, const Params<T>& P, void* const Q[3]);
template <class T> void launch_cell_fill(Grid& g, const Params<T>& P, void* q, double value, int use_inlet,
                                         double inlet_value);

static const double kCmu = 0.09, kClim = 7.0 / 8.0;
static const int kBatchThreads = 4;   // host threads of uf_step_batch

TimedLaunch::TimedLaunch(Grid& g_, int id_) : g(g_), prev(g_.timer_cur) { g.timer_cur = id_; }

TimedLaunch::~TimedLaunch() { g.timer_cur = prev; }

bool timer_pair(Grid& g, hipEvent_t* e0, hipEvent_t* e1) {
  const int id = g.timer_cur;
  if (id < 0 || !((g.timer_mask >> id) & 1u)) return false;
  if (2 * g.timer_used + 2 > g.timer_pool.size()) timer_flush(g);
  *e0 = g.timer_pool[2 * g.timer_used];
  *e1 = g.timer_pool[2 * g.timer_used + 1];
  g.timer_id[g.timer_used] = id;
  g.timer_used++;
  g.timer_cur = -1;   // one launch per scope
  return true;
}

// Wait for the recorded events and add their intervals to the totals.
void timer_flush(Grid& g) {
  if (!g.timer_used) return;
  UF_HIP_CHECK(hipEventSynchronize(g.timer_pool[2 * g.timer_used - 1]));
  for (size_t q = 0; q < g.timer_used; ++q) {
    float ms = 0;
    UF_HIP_CHECK(hipEventElapsedTime(&ms, g.timer_pool[2 * q], g.timer_pool[2 * q + 1]));
    g.timer_ms[g.timer_id[q]] += ms;
    g.timer_n[g.timer_id[q]] += 1;
  }
  g.timer_used = 0;
}
static const size_t S_NSLOT_HOST = 5;   // partial-sum slots of the pressure solve

template <class T>
Params<T> make_params(const Grid& g) {
  Params<T> P{};
  P.L = g.L;
  for (int s = 0; s < 6; ++s) P.bc[s] = g.bc[s];
  const double h[3] = {g.cfg.dx, g.cfg.dy, g.cfg.dz};
  for (int a = 0; a < 3; ++a) {
    P.h[a] = T(h[a]);
    P.ih[a] = T(1.0 / h[a]);
    P.ih2[a] = T(1.0 / (h[a] * h[a]));
    P.dth[a] = T(g.cfg.dt / h[a]);
  }
  P.dt = T(g.cfg.dt);
  P.nu = T(g.cfg.nu);
  P.rho = T(g.cfg.rho);
  P.dt_rho = T(g.cfg.dt / g.cfg.rho);
  P.rho_dt = T(g.cfg.rho / g.cfg.dt);
  P.cap = T(g.nu_max - g.cfg.nu);
  P.k_in = T(g.k_in);
  P.w_in = T(g.w_in);
  P.k_min = T(g.cfg.k_min);
  P.w_min = T(g.cfg.omega_min);
  P.lim_coef = T(kClim / std::sqrt(kCmu / 2.0));
  P.inflow = (const T*)g.inflow;
  return P;
}

void* galloc(Grid& g, size_t bytes) {
  void* p = nullptr;
  if (g.cfg.alloc) {
    p = g.cfg.alloc(bytes, g.cfg.alloc_ctx);
    if (!p) throw HipError("the grid's allocator returned NULL for " + std::to_string(bytes) + " bytes");
    return p;
  }
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) throw HipError(std::string("hipMalloc: ") + hipGetErrorString(e));
  return p;
}

void join_x(Grid& g) {
  if (!g.xpending) return;
  UF_HIP_CHECK(hipStreamWaitEvent(g.stream, g.ev_xjoin, 0));
  g.xpending = false;
}

void upload(Grid& g, void* dst, const void* src, size_t bytes) {
  UF_HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, g.stream));
  UF_HIP_CHECK(hipStreamSynchronize(g.stream));
}

void gfree(Grid& g, void* p) {
  if (!p) return;
  if (g.cfg.free) g.cfg.free(p, g.cfg.alloc_ctx);
  else (void)hipFree(p);
}

}  // namespace uf

using namespace uf;

struct uf_grid_s : public Grid {};

namespace {

uf_status fail(uf_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

#define UF_GUARD_BEGIN try {
#define UF_GUARD_END                                          \
  }                                                           \
  catch (const HipError& e) {                                 \
    return fail(UF_EDEVICE, e.msg);                           \
  }                                                           \
  catch (const std::exception& e) {                           \
    return fail(UF_EDEVICE, e.what());                        \
  }

void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw HipError(std::string("kernel launch: ") + hipGetErrorString(e));
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0; }

// Resolve UF_BC_AUTO: a vertical side is an inlet when the wind blows into
// the domain through it, an outlet otherwise; ground wall, sky slip.
void resolve_bc(const uf_config& c, int out[6]) {
  const double th = c.wind_dir_deg * (M_PI / 180.0);
  const double wx = std::cos(th), wy = std::sin(th);
  const double inward[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
  for (int s = 0; s < 6; ++s) {
    if (c.bc[s] != UF_BC_AUTO) {
      out[s] = c.bc[s];
    } else if (s < 4) {
      out[s] = (inward[s][0] * wx + inward[s][1] * wy > 1e-12) ? UF_BC_INLET : UF_BC_OUTLET;
    } else {
      out[s] = s == 4 ? UF_BC_WALL : UF_BC_SLIP;
    }
  }
}

double nu_max_of(const uf_config& c) {
  return 1.0 / (2.0 * c.dt * (1.0 / (c.dx * c.dx) + 1.0 / (c.dy * c.dy) + 1.0 / (c.dz * c.dz)));
}

std::string validate(const uf_config& c) {
  if (c.nx < 1 || c.ny < 1 || c.nz < 1) return "grid sizes must be >= 1";
  if (c.nx > 32768 || c.ny > 32768 || c.nz > 32768) return "grid size above 32768";
  if ((double)(c.nx + 3) * (c.ny + 3) * (c.nz + 3) > 2.0e9) return "grid too large";
  if (!finite_pos(c.dx) || !finite_pos(c.dy) || !finite_pos(c.dz)) return "dx, dy, dz must be finite and > 0";
  if (!finite_pos(c.dt)) return "dt must be finite and > 0";
  if (c.dtype != UF_F32 && c.dtype != UF_F64) return "dtype must be UF_F32 or UF_F64";
  for (int s = 0; s < 6; ++s)
    if (c.bc[s] < UF_BC_AUTO || c.bc[s] > UF_BC_SLIP) return "unknown boundary kind";
  int bc[6];
  resolve_bc(c, bc);
  bool outlet = false;
  for (int s = 0; s < 6; ++s) outlet |= bc[s] == UF_BC_OUTLET;
  if (!outlet) return "at least one side must be an outlet (the pressure matrix is singular otherwise)";
  if (c.inflow_kind < UF_INFLOW_UNIFORM || c.inflow_kind > UF_INFLOW_PROFILE) return "unknown inflow kind";
  if (!std::isfinite(c.u_ref) || !std::isfinite(c.wind_dir_deg)) return "u_ref and wind_dir_deg must be finite";
  if (c.inflow_kind == UF_INFLOW_LOGLAW &&
      (!finite_pos(c.z0) || !finite_pos(c.karman) || !finite_pos(c.z_ref) || c.z_ref <= c.z0))
    return "log-law inflow needs 0 < z0 < z_ref and karman > 0";
  if (c.inflow_kind == UF_INFLOW_PROFILE) {
    if (!c.inflow_profile) return "inflow_profile is NULL";
    for (int k = 0; k < c.nz; ++k)
      if (!std::isfinite(c.inflow_profile[k])) return "inflow_profile holds a non-finite value";
  }
  if (!std::isfinite(c.nu) || c.nu < 0) return "nu must be finite and >= 0";
  if (!finite_pos(c.rho)) return "rho must be finite and > 0";
  if (c.nu > nu_max_of(c)) return "nu exceeds the explicit-diffusion stability bound 1/(2 dt sum h^-2)";
  if (c.turb_model != UF_TURB_OFF && c.turb_model != UF_TURB_KOMEGA) return "unknown turbulence model";
  if (c.turb_model == UF_TURB_KOMEGA) {
    if (!finite_pos(c.turb_I) || !finite_pos(std::fabs(c.u_ref))) return "k-omega needs turb_I > 0 and u_ref != 0";
    if (!std::isfinite(c.turb_L)) return "turb_L must be finite";
    if (!std::isfinite(c.k_min) || !std::isfinite(c.omega_min) || c.k_min < 0 || c.omega_min < 0)
      return "k_min and omega_min must be finite and >= 0";
  }
  if (!std::isfinite(c.Cd) || !std::isfinite(c.a) || !std::isfinite(c.b) || c.Cd < 0 || c.a < 0)
    return "drag constants must be finite, Cd and a >= 0";
  if (!finite_pos(c.e)) return "e must be finite and > 0";
  if (c.precond != UF_PC_NONE && c.precond != UF_PC_JACOBI && c.precond != UF_PC_AI1 && c.precond != UF_PC_AI2 &&
      c.precond != UF_PC_MG)
    return "unknown preconditioner";
  if (!(c.ai_omega > 0 && c.ai_omega < 2)) return "ai_omega must lie in (0, 2)";
  if (!finite_pos(c.cg_tol)) return "cg_tol must be finite and > 0";
  if (c.cg_maxit < 1 || c.cg_maxit > 1000000) return "cg_maxit must be in [1, 1e6]";
  if (c.cg_criterion != 0 && c.cg_criterion != 1) return "cg_criterion must be 0 or 1";
  if (c.stages < 0 || c.stages > UF_STAGE_ALL) return "unknown stage bits";
  if ((c.alloc == nullptr) != (c.free == nullptr)) return "set both alloc and free, or neither";
  return "";
}

void free_grid(Grid* g) {
  auto f = [g](void*& p) {
    if (p) gfree(*g, p);
    p = nullptr;
  };
  for (auto& s : g->Q)
    for (auto& q : s) f(q);
  for (auto& q : g->K) f(q);
  for (auto& q : g->Wo) f(q);
  f(g->NUT);
  f(g->C);
  f(g->PHI);
  f(g->Xsave);
  f(g->inflow);
  f(g->X);
  f(g->R);
  f(g->R2);
  f(g->Z);
  f(g->D[0]);
  f(g->D[1]);
  f(g->Qv);
  for (auto& set : g->AS)
    for (auto& q : set) f(q);
  for (auto& set : g->AA)
    for (auto& q : set) f(q);
  for (auto& set : g->AV)
    for (auto& q : set) f(q);
  for (auto& set : g->AU)
    for (auto& q : set) f(q);
  for (auto& q : g->AT) f(q);
  f(g->Cbar);
  f(g->XA);
  f(g->inflow0);
  f(g->obj_meta);
  void* pp = g->partials;
  f(pp);
  g->partials = nullptr;
  void* po = g->obj_part;
  f(po);
  g->obj_part = nullptr;
  void* pfl = g->flags;
  f(pfl);
  g->flags = nullptr;
  void* pex = g->exec;
  f(pex);
  g->exec = nullptr;
  void* ps = g->st;
  f(ps);
  g->st = nullptr;
  void* pf = g->flag;
  f(pf);
  g->flag = nullptr;
  void* pd = g->diag;
  f(pd);
  g->diag = nullptr;
  if (g->diag_host) (void)hipHostFree(g->diag_host);
  g->diag_host = nullptr;
  if (g->st_host) (void)hipHostFree(g->st_host);
  if (g->flag_host) (void)hipHostFree(g->flag_host);
  g->st_host = nullptr;
  g->flag_host = nullptr;
  if (g->ev_status) (void)hipEventDestroy(g->ev_status);
  if (g->ev0) (void)hipEventDestroy(g->ev0);
  if (g->ev1) (void)hipEventDestroy(g->ev1);
  g->ev_status = g->ev0 = g->ev1 = nullptr;
  if (g->ev_xfork) (void)hipEventDestroy(g->ev_xfork);
  if (g->ev_xjoin) (void)hipEventDestroy(g->ev_xjoin);
  g->ev_xfork = g->ev_xjoin = nullptr;
  if (g->xstream) (void)hipStreamDestroy(g->xstream);
  g->xstream = nullptr;
  for (hipEvent_t e : g->timer_pool) (void)hipEventDestroy(e);
  g->timer_pool.clear();
  mg_free(*g);
}

// Copy the CG status to the host behind the work enqueued so far; the host
// waits for it in wait_status.
void post_status(Grid& g) {
  UF_HIP_CHECK(hipMemcpyAsync(g.st_host, g.st, sizeof(CgState), hipMemcpyDeviceToHost, g.stream));
  UF_HIP_CHECK(hipEventRecord(g.ev_status, g.stream));
}

void wait_status(Grid& g) { UF_HIP_CHECK(hipEventSynchronize(g.ev_status)); }

struct SolveResult {
  int iters = 0;
  double rel = 0;
  int noconv = 0, nonfinite = 0;
  int nf_state = 0;   // the state's non-finite flag as of this solve's status
  bool first_final = false;   // the first chunk's status already ended the solve
};

// Pressure solve: r0 = b - A x0 and the stopping threshold, the first
// preconditioner application, then iterations enqueued in chunks with the
// device status read after each chunk.  The first chunk is as long as the
// previous solve, so a steady run needs one host round trip per solve;
// iterations enqueued past convergence return at once.
template <class T>
void solve_chunk(Grid& g, const Params<T>& P) {
  const int maxit = g.cfg.cg_maxit;
  int t = g.cg_t;
  int m = t == 0 ? (g.last_iters > 0 ? g.last_iters : 4) : std::max(1, t / 8);
  if (t + m > maxit) m = maxit - t;
  if (m < 1) m = 1;
  for (int q = 0; q < m; ++q, ++t) launch_cg_iteration<T>(g, P, t);
  launch_cg_status(g, t);
  check_launch();
  post_status(g);
  g.cg_t = t;
}

// Enqueue the start of a solve and its first chunk (no host wait).
template <class T>
void solve_begin(Grid& g, const Params<T>& P, void* const Qs[3], const void* b) {
  launch_cg_start<T>(g, P, Qs, b);
  launch_cg_precond<T>(g, P, 0);
  check_launch();
  g.cg_t = 0;
  solve_chunk<T>(g, P);
}

// Wait for the posted status; enqueue further chunks until the solve ends.
template <class T>
SolveResult solve_end(Grid& g, const Params<T>& P) {
  const int maxit = g.cfg.cg_maxit;
  bool first = true, first_final = false;
  while (true) {
    wait_status(g);
    if (first) first_final = g.st_host->done != 0;
    first = false;
    if (g.st_host->done || g.cg_t >= maxit) break;
    solve_chunk<T>(g, P);
  }
  join_x(g);
  SolveResult res;
  res.first_final = first_final;
  const CgState& s = *g.st_host;
  res.iters = s.iter;
  res.rel = s.bb > 0 ? std::sqrt(s.rr / s.bb) : 0.0;
  res.noconv = s.noconv;
  res.nonfinite = s.nonfinite;
  res.nf_state = s.nf_state;
  g.last_iters = s.iter;
  return res;
}

template <class T>
SolveResult solve_pressure(Grid& g, const Params<T>& P, void* const Qs[3], const void* b) {
  solve_begin<T>(g, P, Qs, b);
  return solve_end<T>(g, P);
}

struct StepAccum {
  int iters_total = 0, last_iters = 0, max_iters = 0, noconv = 0, nonfinite = 0;
  int nf_state = 0;   // non-finite value written by the drag or k-omega stage
  double last_rel = 0;
};

int free_set(const Grid& g, int avoid) {
  for (int s = 0; s < 3; ++s)
    if (s != g.cur && s != avoid) return s;
  return -1;
}

// A step in two halves: step_begin enqueues everything up to the first
// chunk of the pressure solve; step_end waits for the solve and enqueues the
// projection and the turbulence model.
template <class T>
void step_begin(Grid& g, const Params<T>& P) {
  const int st = g.cfg.stages;
  {
    if (st & UF_STAGE_ADVECT) {
      const int hat = free_set(g, -1), out = free_set(g, hat);
      launch_advect<T>(g, P, g.Q[g.cur], g.Q[hat], g.Q[out]);
      g.cur = out;
    }
    if (st & UF_STAGE_DIFFUSE) {
      const int out = free_set(g, -1);
      launch_diffuse<T>(g, P, g.Q[g.cur], g.Q[out]);
      g.cur = out;
    }
    if (st & UF_STAGE_DRAG) {
      const int out = free_set(g, -1);
      launch_drag<T>(g, P, g.Q[g.cur], g.Q[out]);
      g.cur = out;
    }
    check_launch();
    if (st & UF_STAGE_PROJECT) solve_begin<T>(g, P, g.Q[g.cur], nullptr);
  }
}

template <class T>
void step_end(Grid& g, const Params<T>& P, StepAccum& acc) {
  const int st = g.cfg.stages;
  const bool turb = (st & UF_STAGE_TURB) && g.cfg.turb_model == UF_TURB_KOMEGA;
  {
    if (st & UF_STAGE_PROJECT) {
      // The projection and the k-omega update are enqueued before the host
      // reads whether the first chunk of iterations ended the solve, gated
      // on the device's verdict (the status the host then reads): in the
      // usual case they run without waiting for that read; when the solve
      // goes on they skip, and run again after it.
      const int out = free_set(g, -1);
      const int kn = g.kcur ^ 1;
      const int* gate = &g.st->done;
      join_x(g);
      launch_project<T>(g, P, g.Q[g.cur], g.Q[out], gate);
      if (turb) launch_turb<T>(g, P, g.Q[out], g.K[g.kcur], g.Wo[g.kcur], g.K[kn], g.Wo[kn], g.NUT, 1, gate);
      SolveResult r = solve_end<T>(g, P);
      acc.iters_total += r.iters;
      acc.last_iters = r.iters;
      acc.max_iters = std::max(acc.max_iters, r.iters);
      acc.last_rel = r.rel;
      acc.noconv |= r.noconv;
      acc.nonfinite |= r.nonfinite;
      acc.nf_state |= r.nf_state;
      if (!r.first_final) {
        launch_project<T>(g, P, g.Q[g.cur], g.Q[out]);
        if (turb) launch_turb<T>(g, P, g.Q[out], g.K[g.kcur], g.Wo[g.kcur], g.K[kn], g.Wo[kn], g.NUT, 1);
      }
      g.cur = out;
      if (turb) g.kcur = kn;
    } else if (turb) {
      const int kn = g.kcur ^ 1;
      launch_turb<T>(g, P, g.Q[g.cur], g.K[g.kcur], g.Wo[g.kcur], g.K[kn], g.Wo[kn], g.NUT, 1);
      g.kcur = kn;
    }
    check_launch();
  }
}

template <class T>
void run_steps(Grid& g, int nsteps, StepAccum& acc) {
  const Params<T> P = make_params<T>(g);
  for (int n = 0; n < nsteps; ++n) {
    step_begin<T>(g, P);
    step_end<T>(g, P, acc);
  }
}

// Enqueue the end-of-call diagnostics and the copy of the non-finite flag
// (read by finish_stats once the stream has reached them).
void post_diag(Grid& g) {
  if (g.esize == 4) launch_diag<float>(g, make_params<float>(g));
  else launch_diag<double>(g, make_params<double>(g));
  check_launch();
  UF_HIP_CHECK(hipMemcpyAsync(g.diag_host, g.diag, 3 * kDiagBlocks * sizeof(double), hipMemcpyDeviceToHost,
                              g.stream));
  UF_HIP_CHECK(hipMemcpyAsync(g.flag_host, nf_word(g), sizeof(int), hipMemcpyDeviceToHost, g.stream));
}

void fill_stats(uf_step_stats* stats, StepAccum& acc, float ms, const Grid& g) {
  // the stream has passed post_diag: the partials and the flag are on the host
  double mdiv = 0, mcfl = 0, clip = 0;
  for (int b = 0; b < kDiagBlocks; ++b) {
    const double d = g.diag_host[b], c = g.diag_host[kDiagBlocks + b];
    mdiv = (d != d || d > mdiv) ? d : mdiv;
    mcfl = (c != c || c > mcfl) ? c : mcfl;
    clip += g.diag_host[2 * kDiagBlocks + b];
  }
  acc.nf_state |= *g.flag_host;
  stats->cg_iters = acc.last_iters;
  stats->cg_iters_total = acc.iters_total;
  stats->cg_rel_residual = acc.last_rel;
  stats->converged = !(acc.noconv || acc.nonfinite);
  stats->nonfinite = acc.nonfinite || acc.nf_state;
  stats->ms = ms;
  stats->cg_iters_max = acc.max_iters;
  stats->max_div = mdiv;
  stats->max_cfl = mcfl;
  stats->nut_clip_frac = clip / ((double)g.L.nx * g.L.ny * g.L.nz);
}

template <class T>
void init_state(Grid& g) {
  const Params<T> P = make_params<T>(g);
  launch_face_init<T>(g, P, g.Q[g.cur]);
  launch_cell_fill<T>(g, P, g.K[g.kcur], g.k_in, 1, g.k_in);
  launch_cell_fill<T>(g, P, g.Wo[g.kcur], g.w_in, 1, g.w_in);
  if (g.cfg.turb_model == UF_TURB_KOMEGA)
    launch_turb<T>(g, P, g.Q[g.cur], g.K[g.kcur], g.Wo[g.kcur], nullptr, nullptr, g.NUT, 0);
  check_launch();
}

template <class T>
void upload_inflow(Grid& g) {
  const uf_config& c = g.cfg;
  const int nz = c.nz;
  std::vector<T> tab(2 * (nz + 2));
  const double th = c.wind_dir_deg * (M_PI / 180.0);
  const double dir[2] = {std::cos(th), std::sin(th)};
  for (int k = -1; k <= nz; ++k) {
    double s = 0;
    if (c.inflow_kind == UF_INFLOW_UNIFORM) {
      s = c.u_ref;
    } else if (c.inflow_kind == UF_INFLOW_LOGLAW) {
      // Sec. 5.1: u(z) = (u*/kappa) ln(z/z0), u* fixed by u(z_ref) = u_ref
      const double ustar = c.u_ref * c.karman / std::log(c.z_ref / c.z0);
      const double z = (k + 0.5) * c.dz;
      s = z > c.z0 ? ustar / c.karman * std::log(z / c.z0) : 0.0;
    } else {
      const int kk = k < 0 ? 0 : (k > nz - 1 ? nz - 1 : k);
      s = g.profile[kk];
    }
    tab[0 * (nz + 2) + (k + 1)] = T(s * dir[0]);
    tab[1 * (nz + 2) + (k + 1)] = T(s * dir[1]);
  }
  upload(g, g.inflow, tab.data(), tab.size() * sizeof(T));
}

template <class T>
void fill_phi_one(Grid& g) {
  std::vector<T> ones((size_t)g.L.nx * g.L.ny * g.L.nz, T(1));
  upload(g, g.PHI, ones.data(), ones.size() * sizeof(T));
}

int64_t extent(const uf_config* c, int32_t f, int32_t d[3]) {
  int e[3] = {c->nx, c->ny, c->nz};
  if (f < 0 || f > UF_PHI) return -1;
  if (f < 3) e[f] += 1;
  if (d) {
    d[0] = e[0];
    d[1] = e[1];
    d[2] = e[2];
  }
  return (int64_t)e[0] * e[1] * e[2];
}

// Reverse of one step (see uf_adjoint_step).  The forward stages before
// the projection are recomputed from the given state into the adjoint
// workspace; then each enabled stage is reversed, last first.
void adjoint_alloc(Grid& g) {
  if (g.XA) return;
  const size_t bytes = g.nelem * g.esize;
  for (auto& set : g.AS)
    for (auto& q : set) q = galloc(g, bytes);
  for (auto& set : g.AA)
    for (auto& q : set) q = galloc(g, bytes);
  for (auto& set : g.AV)
    for (auto& q : set) {
      q = galloc(g, bytes);
      UF_HIP_CHECK(hipMemsetAsync(q, 0, bytes, g.stream));
    }
  for (auto& set : g.AU)
    for (auto& q : set) q = galloc(g, bytes);
  for (auto& q : g.AT) q = galloc(g, bytes);
  UF_HIP_CHECK(hipMemsetAsync(g.AT[9], 0, bytes, g.stream));   // recompute pressure: zero start and ghosts
  g.Cbar = galloc(g, bytes);
  g.XA = galloc(g, bytes);
  UF_HIP_CHECK(hipMemsetAsync(g.XA, 0, bytes, g.stream));   // zero start and zero ghosts
  const size_t tab = 2 * (size_t)(g.L.nz + 2) * g.esize;
  g.inflow0 = galloc(g, tab);
  UF_HIP_CHECK(hipMemsetAsync(g.inflow0, 0, tab, g.stream));
}

// The adjoint solve and the recompute's forward solve run in the pressure
// array, each with its own warm start: swap one in for the scope and back
// out on every path.
struct PressureSwap {
  Grid& g;
  void*& other;
  int& other_iters;
  int saved_iters;
  PressureSwap(Grid& g_, void*& x, int& iters) : g(g_), other(x), other_iters(iters), saved_iters(g_.last_iters) {
    std::swap(g.X, other);
    g.last_iters = other_iters;
  }
  ~PressureSwap() {
    other_iters = g.last_iters;
    g.last_iters = saved_iters;
    std::swap(g.X, other);
  }
};

// The eddy viscosity the recomputed diffusion reads (the state's own).
struct NutSwap {
  Grid& g;
  void*& other;
  NutSwap(Grid& g_, void*& n) : g(g_), other(n) { std::swap(g.NUT, other); }
  ~NutSwap() { std::swap(g.NUT, other); }
};

// k-omega fields of the reverse step (indices into Grid::AT)
enum { AT_K = 0, AT_W, AT_NUT, AT_KB1, AT_WB1, AT_NB1, AT_KB0, AT_WB0, AT_NB0, AT_XF };

template <class T>
SolveResult adjoint_step(Grid& g, const void* const* state, const void* const* state_next,
                         const void* const* adj_next, void* const* adj_out, double* phibar) {
  adjoint_alloc(g);
  const Params<T> P = make_params<T>(g);
  Params<T> P0 = P;   // homogeneous boundary values: fixed faces and inlet ghosts are zero
  P0.inflow = (const T*)g.inflow0;
  const int st = g.cfg.stages;
  const bool turb = g.cfg.turb_model == UF_TURB_KOMEGA && (st & UF_STAGE_TURB);
  const size_t bytes = g.nelem * g.esize;
  auto zero = [&](void* const set[3]) {
    for (int c = 0; c < 3; ++c) UF_HIP_CHECK(hipMemsetAsync(set[c], 0, bytes, g.stream));
  };
  // forward recompute, as in step_begin / step_end
  for (int c = 0; c < 3; ++c) {
    launch_pack<T>(g, P, state[c], g.AS[0][c], c, 1);
    launch_face_bc<T>(g, P, g.AS[0][c], c);
  }
  if (turb) {
    launch_pack<T>(g, P, state[3], g.AT[AT_K], UF_K, 1);
    launch_cell_bc<T>(g, P, g.AT[AT_K], 1, g.k_in);
    launch_pack<T>(g, P, state[4], g.AT[AT_W], UF_OMEGA, 1);
    launch_cell_bc<T>(g, P, g.AT[AT_W], 1, g.w_in);
    launch_pack<T>(g, P, state[5], g.AT[AT_NUT], UF_NUT, 1);
    launch_cell_bc<T>(g, P, g.AT[AT_NUT], 0, 0.0);
  }
  void* const* x = g.AS[0];
  if (st & UF_STAGE_ADVECT) {
    launch_advect<T>(g, P, g.AS[0], g.AS[1], g.AS[2]);
    x = g.AS[2];
  }
  void* const* diff_in = x;
  if (st & UF_STAGE_DIFFUSE) {
    if (turb) {
      NutSwap ns(g, g.AT[AT_NUT]);
      launch_diffuse<T>(g, P, x, g.AS[3]);
    } else {
      launch_diffuse<T>(g, P, x, g.AS[3]);
    }
    x = g.AS[3];
  }
  void* const* drag_in = x;
  void* const* unew = x;
  SolveResult fres;
  if (turb && state_next) {   // u^{n+1} given: the turbulence reverse linearises there
    for (int c = 0; c < 3; ++c) {
      launch_pack<T>(g, P, state_next[c], g.AU[1][c], c, 1);
      launch_face_bc<T>(g, P, g.AU[1][c], c);
    }
    unew = g.AU[1];
  } else if (turb) {   // recompute u^{n+1}
    if (st & UF_STAGE_DRAG) {
      launch_drag<T>(g, P, x, g.AU[0]);
      x = g.AU[0];
    }
    if (st & UF_STAGE_PROJECT) {
      // from zero, so that the recomputed u^{n+1} -- and every branch the
      // turbulence reverse takes at it -- depends on this call's inputs only
      UF_HIP_CHECK(hipMemsetAsync(g.AT[AT_XF], 0, bytes, g.stream));
      g.fwd_last_iters = 0;
      PressureSwap ps(g, g.AT[AT_XF], g.fwd_last_iters);
      fres = solve_pressure<T>(g, P, x, nullptr);
      launch_project<T>(g, P, x, g.AU[1]);
      x = g.AU[1];
    }
    unew = x;
  }
  check_launch();
  // reverse
  void* const* A0 = g.AA[0];
  void* const* A1 = g.AA[1];
  void* const* A2 = g.AA[2];
  auto other = [&](void* const* a) { return a == A0 ? A1 : A0; };
  zero(A0);
  for (int c = 0; c < 3; ++c) launch_pack<T>(g, P, adj_next[c], A0[c], c, 1);
  launch_fold<T>(g, P, A0);   // no ghosts yet: clears the fixed faces
  if (turb) {
    const int fields[3] = {UF_K, UF_OMEGA, UF_NUT};
    for (int q = 0; q < 3; ++q) {
      UF_HIP_CHECK(hipMemsetAsync(g.AT[AT_KB1 + q], 0, bytes, g.stream));
      launch_pack<T>(g, P, adj_next[3 + q], g.AT[AT_KB1 + q], fields[q], 1);
    }
    for (int q = AT_KB0; q <= AT_NB0; ++q) UF_HIP_CHECK(hipMemsetAsync(g.AT[q], 0, bytes, g.stream));
    launch_turb_adj<T>(g, P, unew, g.AT[AT_K], g.AT[AT_W], g.AT[AT_KB1], g.AT[AT_WB1], g.AT[AT_NB1],
                       g.AT[AT_KB0], g.AT[AT_WB0], A0);
    launch_cell_fold<T>(g, P, g.AT[AT_KB0], 1);
    launch_cell_fold<T>(g, P, g.AT[AT_WB0], 1);
    launch_fold<T>(g, P, A0);   // ghosts of u^{n+1} that the turbulence update read
  }
  void* const* a = A0;
  SolveResult res;
  if (st & UF_STAGE_PROJECT) {
    PressureSwap ps(g, g.XA, g.adj_last_iters);
    res = solve_pressure<T>(g, P0, a, nullptr);
    launch_project<T>(g, P0, a, A1);
    a = A1;
  }
  if (st & UF_STAGE_DRAG) {
    void* const* d = other(a);
    zero(d);
    UF_HIP_CHECK(hipMemsetAsync(g.Cbar, 0, bytes, g.stream));
    launch_drag_adj<T>(g, P, drag_in, a, d, g.Cbar);
    launch_fold<T>(g, P, d);
    if (phibar) launch_drag_coef_adj<T>(g, P, g.Cbar, phibar);
    a = d;
  }
  if (st & UF_STAGE_DIFFUSE) {
    void* const* d = other(a);
    if (turb) {
      launch_diffuse_nut_adj<T>(g, P, diff_in, a, g.AT[AT_NB0]);
      NutSwap ns(g, g.AT[AT_NUT]);   // the eddy viscosity of step n, not the grid's current one
      launch_diffuse_adj<T>(g, P, a, d);
    } else {
      launch_diffuse_adj<T>(g, P, a, d);
    }
    launch_fold<T>(g, P, d);
    a = d;
  }
  if (st & UF_STAGE_ADVECT) {
    void* const* h = other(a);
    zero(A2);
    zero(h);
    launch_advect_adj<T>(g, P, g.AS[0], g.AS[1], a, A2, h);
    launch_fold<T>(g, P, A2);
    a = A2;
  }
  for (int c = 0; c < 3; ++c) launch_pack<T>(g, P, a[c], adj_out[c], c, 0);
  if (turb) {
    launch_pack<T>(g, P, g.AT[AT_KB0], adj_out[3], UF_K, 0);
    launch_pack<T>(g, P, g.AT[AT_WB0], adj_out[4], UF_OMEGA, 0);
    launch_pack<T>(g, P, g.AT[AT_NB0], adj_out[5], UF_NUT, 0);
  }
  check_launch();
  res.noconv |= fres.noconv;
  res.nonfinite |= fres.nonfinite;
  return res;
}

std::string check_smooth_objects(const uf_smooth_objects* o) {
  if (o->nx < 1 || o->ny < 1 || o->nz < 1) return "grid sizes must be >= 1";
  if ((double)o->nx * o->ny * o->nz > 4.0e9) return "grid too large";
  if (!finite_pos(o->dx) || !finite_pos(o->dy) || !finite_pos(o->dz) || !finite_pos(o->width))
    return "cell sizes and the step width must be positive and finite";
  if (o->nboxes < 0 || o->ncyls < 0 || o->nboxes > 65536 || o->ncyls > 65536) return "object count out of range";
  if ((o->nboxes > 0 && !o->boxes) || (o->ncyls > 0 && !o->cylinders)) return "NULL object array";
  for (int b = 0; b < o->nboxes; ++b) {
    for (int q = 0; q < 7; ++q)
      if (!std::isfinite(o->boxes[7 * b + q])) return "non-finite box value";
    if (!(o->boxes[7 * b + 6] >= 0.0 && o->boxes[7 * b + 6] <= 1.0)) return "box phi outside [0, 1]";
  }
  for (int c = 0; c < o->ncyls; ++c) {
    for (int q = 0; q < 6; ++q)
      if (!std::isfinite(o->cylinders[6 * c + q])) return "non-finite cylinder value";
    if (o->cylinders[6 * c + 2] < 0.0) return "negative cylinder radius";
    if (!(o->cylinders[6 * c + 5] >= 0.0 && o->cylinders[6 * c + 5] <= 1.0)) return "cylinder phi outside [0, 1]";
  }
  return "";
}

}  // namespace

namespace {
// ------------------------------------------------------------- batches ---
// A batch advances several grids together.  Each face stage of the step
// (predictor, corrector, diffusion, drag, projection) and the k-omega
// update is one launch for every case, walking one queue of the cases'
// blocks (k_faces_multi, k_turb_multi).  Each case's pressure solve (its
// start and a fixed number of CG iterations, iterations past convergence
// returning at once) is a hipGraph of its own, replayed on the case's own
// stream so that the solves of the cases overlap; the face stages before
// the solve and the projection and k-omega update after it are two more
// graphs on the batch's stream.  Between them the host reads every case's
// solve status and enqueues further iterations for a case that needs them,
// and re-captures a case's solve when its iteration count moves away from
// the captured one.  The stage launches' band width and grid size come
// from uf_batch_autotune.
struct BatchTune {
  int band[6];
  int blocks[6];   // 0: one block per logical block (no persistent walk)
  float ms[6];
};

struct Batch {
  std::vector<Grid*> g;
  size_t esize = 4;
  hipStream_t origin = nullptr;
  std::vector<hipStream_t> cs;     // one stream per case (its solve)
  std::vector<hipStream_t> own;    // the grids' streams while a call runs on the batch's
  std::vector<hipEvent_t> ev_case;
  hipEvent_t ev_fork = nullptr, ev_end = nullptr;
  void* table = nullptr;           // MultiCase<T>[n] on the device
  CaseStarts faces{}, cells{};     // the cases' blocks in the face and cell queues
  int turb = 0;
  BatchTune tune{};
  std::vector<int> kcap;           // CG iterations in each case's solve graph
  int* kc_dev = nullptr;           // each case's k/omega slot, read by the k-omega launch
  int* kc_host = nullptr;          // pinned staging of the slots
  hipGraphExec_t front = nullptr, back = nullptr;
  std::vector<hipGraphExec_t> solve;
};

int stage_blocks(const BatchTune& t, int s, int total) {
  const int want = t.blocks[s] > 0 ? t.blocks[s] : total;
  return 8 * ((std::min(want, total) + 7) / 8);
}

void drop_solve(Batch& b, size_t c) {
  if (b.solve[c]) (void)hipGraphExecDestroy(b.solve[c]);
  b.solve[c] = nullptr;
}

void drop_graphs(Batch& b) {
  if (b.front) (void)hipGraphExecDestroy(b.front);
  if (b.back) (void)hipGraphExecDestroy(b.back);
  b.front = b.back = nullptr;
  for (size_t c = 0; c < b.solve.size(); ++c) drop_solve(b, c);
}

// Release the batch's streams, events, graphs and case table.
void release_batch(Batch* b) {
  drop_graphs(*b);
  for (auto s : b->cs)
    if (s) (void)hipStreamDestroy(s);
  for (auto e : b->ev_case)
    if (e) (void)hipEventDestroy(e);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_end) (void)hipEventDestroy(b->ev_end);
  if (b->origin) (void)hipStreamDestroy(b->origin);
  if (b->table) (void)hipFree(b->table);
  if (b->kc_dev) (void)hipFree(b->kc_dev);
  if (b->kc_host) (void)hipHostFree(b->kc_host);
  b->kc_dev = nullptr;
  b->kc_host = nullptr;
  b->cs.clear();
  b->ev_case.clear();
  b->ev_fork = b->ev_end = nullptr;
  b->origin = nullptr;
  b->table = nullptr;
}

template <class T>
void build_table(Batch& b) {
  std::vector<MultiCase<T>> tab(b.g.size());
  int face = 0, cell = 0;
  b.faces.n = b.cells.n = (int)b.g.size();
  for (size_t c = 0; c < b.g.size(); ++c) {
    Grid& g = *b.g[c];
    MultiCase<T>& m = tab[c];
    m.P = make_params<T>(g);
    for (int s2 = 0; s2 < 3; ++s2)
      for (int q = 0; q < 3; ++q) m.q[s2][q] = (T*)g.Q[s2][q];
    m.nut = (T*)g.NUT;
    m.cc = (const T*)g.C;
    m.x = (const T*)g.X;
    for (int q = 0; q < 2; ++q) {
      m.k[q] = (T*)g.K[q];
      m.w[q] = (T*)g.Wo[q];
    }
    m.nf = nf_word(g);
    b.faces.start[c] = face;
    b.cells.start[c] = cell;
    face += face_gx(g.L) * (g.L.nx + 1);
    cell += cell_queue_blocks(g.L);
  }
  b.faces.start[b.g.size()] = face;
  b.cells.start[b.g.size()] = cell;
  UF_HIP_CHECK(hipMalloc(&b.table, sizeof(MultiCase<T>) * tab.size()));
  UF_HIP_CHECK(hipMemcpyAsync(b.table, tab.data(), sizeof(MultiCase<T>) * tab.size(), hipMemcpyHostToDevice,
                              b.origin));
  UF_HIP_CHECK(hipStreamSynchronize(b.origin));
}

// The face stages of a step or of a trial run: (stage, in, aux, out) sets.
struct FaceRun {
  int stage, sin, saux, sout;
};
const FaceRun kFront[4] = {{MS_ADVECT_FWD, 0, 0, 1}, {MS_ADVECT_CORR, 0, 1, 2}, {MS_DIFFUSE, 2, 0, 0},
                           {MS_DRAG, 0, 0, 1}};
const FaceRun kTrial[5] = {{MS_ADVECT_FWD, 0, 0, 1}, {MS_ADVECT_CORR, 0, 1, 2}, {MS_DIFFUSE, 2, 0, 1},
                           {MS_DRAG, 1, 0, 2}, {MS_PROJECT, 2, 0, 1}};

template <class T>
void enqueue_face(Batch& b, const FaceRun& r, hipStream_t st) {
  // the corrector's queue has three entries per face block (one per component)
  const int entries = (r.stage == MS_ADVECT_CORR ? 3 : 1) * b.faces.start[b.faces.n];
  launch_faces_multi<T>(r.stage, (const MultiCase<T>*)b.table, b.faces, b.tune.band[r.stage],
                        stage_blocks(b.tune, r.stage, entries), r.sin, r.saux, r.sout, st);
}

template <class T>
void enqueue_turb(Batch& b, int nut_set, hipStream_t st) {
  launch_turb_multi<T>((const MultiCase<T>*)b.table, b.cells, b.tune.band[5],
                       stage_blocks(b.tune, 5, b.cells.start[b.cells.n]), 0, b.kc_dev, nut_set, st);
}

// Each case's k/omega slot to the device, behind the work on the origin stream.
void post_slots(Batch& b) {
  for (size_t c = 0; c < b.g.size(); ++c) b.kc_host[c] = b.g[c]->kcur;
  UF_HIP_CHECK(hipMemcpyAsync(b.kc_dev, b.kc_host, sizeof(int) * b.g.size(), hipMemcpyHostToDevice, b.origin));
}

// Capture what `body` enqueues on stream st into *exec.
template <class F>
void capture(hipStream_t st, hipGraphExec_t* exec, F body) {
  hipGraph_t graph = nullptr;
  UF_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  try {
    body();
  } catch (...) {
    (void)hipStreamEndCapture(st, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  UF_HIP_CHECK(hipStreamEndCapture(st, &graph));
  const hipError_t e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  UF_HIP_CHECK(e);
}

// Front of a step: the face stages up to the drag (the state in set 0, the
// drag output in set 1).
template <class T>
void capture_front(Batch& b) {
  capture(b.origin, &b.front, [&] {
    for (const FaceRun& r : kFront) enqueue_face<T>(b, r, b.origin);
  });
}

// Case c's solve on its stream: the start from the drag output, the first
// preconditioner application, kcap[c] iterations, the status to the host.
template <class T>
void capture_solve(Batch& b, size_t c) {
  Grid& g = *b.g[c];
  capture(b.cs[c], &b.solve[c], [&] {
    const Params<T> P = make_params<T>(g);
    launch_cg_start<T>(g, P, g.Q[1], nullptr);
    launch_cg_precond<T>(g, P, 0);
    for (int t = 0; t < b.kcap[c]; ++t) launch_cg_iteration<T>(g, P, t);
    launch_cg_status(g, b.kcap[c]);
    UF_HIP_CHECK(hipMemcpyAsync(g.st_host, g.st, sizeof(CgState), hipMemcpyDeviceToHost, b.cs[c]));
    join_x(g);
  });
}

// Back of a step: the projection (set 1 to set 0) and the k-omega update
// from each case's current slot.
template <class T>
void capture_back(Batch& b) {
  capture(b.origin, &b.back, [&] {
    enqueue_face<T>(b, FaceRun{MS_PROJECT, 1, 0, 0}, b.origin);
    if (b.turb) enqueue_turb<T>(b, -1, b.origin);
  });
}

// The grids run on the batch's streams for the duration of a call (the
// captured kernels are bound to them); their own streams are ordered
// before and after it.
void enter_batch(Batch& b) {
  for (size_t c = 0; c < b.g.size(); ++c) {
    Grid& g = *b.g[c];
    b.own[c] = g.stream;
    UF_HIP_CHECK(hipEventRecord(b.ev_case[c], g.stream));
    UF_HIP_CHECK(hipStreamWaitEvent(b.origin, b.ev_case[c], 0));
    g.stream = b.cs[c];
  }
}

void leave_batch(Batch& b) {
  UF_HIP_CHECK(hipEventRecord(b.ev_end, b.origin));
  for (size_t c = 0; c < b.g.size(); ++c) {
    Grid& g = *b.g[c];
    UF_HIP_CHECK(hipStreamWaitEvent(b.cs[c], b.ev_end, 0));
    UF_HIP_CHECK(hipEventRecord(b.ev_case[c], b.cs[c]));
    g.stream = b.own[c];
    UF_HIP_CHECK(hipStreamWaitEvent(g.stream, b.ev_case[c], 0));
  }
}

template <class T>
void batch_steps(Batch& b, int nsteps, std::vector<StepAccum>& acc) {
  const int n = (int)b.g.size();
  for (int s2 = 0; s2 < nsteps; ++s2) {
    if (!b.front) capture_front<T>(b);
    if (!b.back) capture_back<T>(b);
    for (int c = 0; c < n; ++c)
      if (!b.solve[c]) capture_solve<T>(b, c);
    UF_HIP_CHECK(hipGraphLaunch(b.front, b.origin));
    UF_HIP_CHECK(hipEventRecord(b.ev_fork, b.origin));
    for (int c = 0; c < n; ++c) {
      UF_HIP_CHECK(hipStreamWaitEvent(b.cs[c], b.ev_fork, 0));
      UF_HIP_CHECK(hipGraphLaunch(b.solve[c], b.cs[c]));
      UF_HIP_CHECK(hipEventRecord(b.ev_case[c], b.cs[c]));
    }
    for (int c = 0; c < n; ++c) {
      Grid& g = *b.g[c];
      const Params<T> P = make_params<T>(g);
      UF_HIP_CHECK(hipEventSynchronize(b.ev_case[c]));
      g.cg_t = b.kcap[c];
      // further iterations past the captured ones, as the single-grid loop runs them
      while (!g.st_host->done && g.cg_t < g.cfg.cg_maxit) {
        solve_chunk<T>(g, P);
        wait_status(g);
      }
      join_x(g);
      const CgState& st = *g.st_host;
      g.last_iters = st.iter;
      acc[c].iters_total += st.iter;
      acc[c].last_iters = st.iter;
      acc[c].max_iters = std::max(acc[c].max_iters, st.iter);
      acc[c].last_rel = st.bb > 0 ? std::sqrt(st.rr / st.bb) : 0.0;
      acc[c].noconv |= st.noconv;
      acc[c].nonfinite |= st.nonfinite;
      acc[c].nf_state |= st.nf_state;
      // a solve graph too short (or far too long) for this case is captured again
      if (st.iter > b.kcap[c] || st.iter + 4 < b.kcap[c]) {
        b.kcap[c] = std::min(g.cfg.cg_maxit, st.iter + 2);
        UF_HIP_CHECK(hipStreamSynchronize(b.cs[c]));
        drop_solve(b, c);
      }
      UF_HIP_CHECK(hipEventRecord(b.ev_case[c], b.cs[c]));
      UF_HIP_CHECK(hipStreamWaitEvent(b.origin, b.ev_case[c], 0));
    }
    post_slots(b);
    UF_HIP_CHECK(hipGraphLaunch(b.back, b.origin));
    for (int c = 0; c < n; ++c) b.g[c]->kcur ^= 1;
  }
}

// Trial launches of every stage with each candidate band width and grid
// size, on the sets a step overwrites anyway (set 0, k, omega, nu_t and the
// pressure are only read); the fastest of three runs of each is kept.
template <class T>
void autotune(Batch& b) {
  const int bands[3] = {4, 8, 16};
  const int per_cu[4] = {2, 4, 8, 0};
  hipEvent_t e0, e1;
  UF_HIP_CHECK(hipEventCreate(&e0));
  UF_HIP_CHECK(hipEventCreate(&e1));
  try {
    post_slots(b);
    for (int st = 0; st < 6; ++st) {
      if (st == 5 && !b.turb) {
        b.tune.ms[5] = 0.f;
        continue;
      }
      float best = 1e30f;
      int bb = 8, bp = 0;
      for (int band : bands)
        for (int pc : per_cu) {
          BatchTune t = b.tune;
          t.band[st] = band;
          t.blocks[st] = pc ? pc * 256 : 0;
          std::swap(t, b.tune);
          float fastest = 1e30f;
          for (int rep = 0; rep < 3; ++rep) {
            UF_HIP_CHECK(hipEventRecord(e0, b.origin));
            if (st < 5) enqueue_face<T>(b, kTrial[st], b.origin);
            else enqueue_turb<T>(b, 2, b.origin);
            UF_HIP_CHECK(hipEventRecord(e1, b.origin));
            UF_HIP_CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            UF_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
            fastest = std::min(fastest, ms);
          }
          std::swap(t, b.tune);
          if (fastest < best) {
            best = fastest;
            bb = band;
            bp = pc ? pc * 256 : 0;
          }
        }
      b.tune.band[st] = bb;
      b.tune.blocks[st] = bp;
      b.tune.ms[st] = best;
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

}  // namespace

struct uf_batch_s : public Batch {};

extern "C" {

const char* uf_last_error(void) { return g_last_error.c_str(); }

uf_status uf_resolve_bc(const uf_config* cfg, int32_t out[6]) {
  if (!cfg || !out) return fail(UF_EINVAL, "NULL argument");
  if (!std::isfinite(cfg->wind_dir_deg)) return fail(UF_EINVAL, "wind_dir_deg must be finite");
  for (int s = 0; s < 6; ++s)
    if (cfg->bc[s] < UF_BC_AUTO || cfg->bc[s] > UF_BC_SLIP) return fail(UF_EINVAL, "unknown boundary kind");
  int bc[6];
  resolve_bc(*cfg, bc);
  for (int s = 0; s < 6; ++s) out[s] = bc[s];
  return UF_OK;
}

int64_t uf_field_extent(const uf_config* cfg, int32_t field, int32_t dims[3]) {
  if (!cfg) return -1;
  return extent(cfg, field, dims);
}

uf_status uf_create_grid(const uf_config* cfg, uf_grid* out) {
  if (!cfg || !out) return fail(UF_EINVAL, "NULL argument");
  const std::string err = validate(*cfg);
  if (!err.empty()) return fail(UF_EINVAL, err);
  uf_grid_s* g = new uf_grid_s();
  UF_GUARD_BEGIN
  g->cfg = *cfg;
  if (cfg->inflow_kind == UF_INFLOW_PROFILE) g->profile.assign(cfg->inflow_profile, cfg->inflow_profile + cfg->nz);
  g->cfg.inflow_profile = nullptr;
  resolve_bc(*cfg, g->bc);
  for (int s = 0; s < 6; ++s) g->cfg.bc[s] = g->bc[s];
  g->stream = (hipStream_t)cfg->stream;
  Layout& L = g->L;
  L.nx = cfg->nx;
  L.ny = cfg->ny;
  L.nz = cfg->nz;
  L.PZ = cfg->nz + 3;
  L.SX = (long long)(cfg->ny + 3) * L.PZ;
  g->nelem = (size_t)(cfg->nx + 3) * L.SX;
  g->esize = cfg->dtype == UF_F64 ? 8 : 4;
  g->nu_max = nu_max_of(*cfg);
  const double I = cfg->turb_I, U = std::fabs(cfg->u_ref);
  const double Lt = cfg->turb_L > 0 ? cfg->turb_L : 0.1 * cfg->nz * cfg->dz;
  g->k_in = 1.5 * (I * U) * (I * U);
  g->w_in = std::sqrt(g->k_in) / (std::pow(kCmu, 0.25) * Lt);
  const size_t bytes = g->nelem * g->esize;
  std::vector<void**> bufs;
  for (auto& s : g->Q)
    for (auto& q : s) bufs.push_back(&q);
  for (auto& q : g->K) bufs.push_back(&q);
  for (auto& q : g->Wo) bufs.push_back(&q);
  for (void** q : {&g->NUT, &g->C, &g->X, &g->R, &g->R2, &g->Z, &g->D[0], &g->D[1], &g->Qv}) bufs.push_back(q);
  try {
    for (void** q : bufs) {
      *q = galloc(*g, bytes);
      UF_HIP_CHECK(hipMemsetAsync(*q, 0, bytes, g->stream));
    }
    g->PHI = galloc(*g, (size_t)cfg->nx * cfg->ny * cfg->nz * g->esize);
    g->inflow = galloc(*g, 2 * (cfg->nz + 2) * g->esize);
    const CgLaunch cl = cg_launch(L);
    g->cg_nb = (size_t)cl.gx * cl.gy;
    g->cg_nb_rz = cfg->precond == UF_PC_MG ? mg_fine_blocks(L) : g->cg_nb;
    g->cg_nb_dq = (size_t)ad_launch(L).blocks;
    g->cg_nb_rr = g->cg_nb;
    g->flags = (int*)galloc(*g, sizeof(int) * (cfg->cg_maxit + 2));
    g->exec = (int*)galloc(*g, sizeof(int) * (cfg->cg_maxit + 2));
    UF_HIP_CHECK(hipMemsetAsync(g->flags, 0, sizeof(int) * (cfg->cg_maxit + 2), g->stream));
    UF_HIP_CHECK(hipMemsetAsync(g->exec, 0, sizeof(int) * (cfg->cg_maxit + 2), g->stream));
    g->st = (CgState*)galloc(*g, sizeof(CgState));
    g->flag = (int*)galloc(*g, sizeof(int));
    g->diag = (double*)galloc(*g, 3 * kDiagBlocks * sizeof(double));
  } catch (const HipError& e) {
    free_grid(g);
    delete g;
    return fail(UF_ENOMEM, e.msg);
  }
  UF_HIP_CHECK(hipMemsetAsync(g->st, 0, sizeof(CgState), g->stream));
  UF_HIP_CHECK(hipHostMalloc((void**)&g->st_host, sizeof(CgState), hipHostMallocDefault));
  UF_HIP_CHECK(hipHostMalloc((void**)&g->flag_host, sizeof(int), hipHostMallocDefault));
  UF_HIP_CHECK(hipHostMalloc((void**)&g->diag_host, 3 * kDiagBlocks * sizeof(double), hipHostMallocDefault));
  UF_HIP_CHECK(hipEventCreateWithFlags(&g->ev_status, hipEventDisableTiming));
  UF_HIP_CHECK(hipEventCreate(&g->ev0));
  UF_HIP_CHECK(hipEventCreate(&g->ev1));
  UF_HIP_CHECK(hipStreamSynchronize(g->stream));
  if (g->esize == 4) {
    upload_inflow<float>(*g);
    fill_phi_one<float>(*g);
    if (cfg->precond == UF_PC_MG) mg_setup<float>(*g);
  } else {
    upload_inflow<double>(*g);
    fill_phi_one<double>(*g);
    if (cfg->precond == UF_PC_MG) mg_setup<double>(*g);
  }
  // partial-sum slots, sized for every kernel that writes them (the
  // multigrid hierarchy decides whether the level-0 restriction is one)
  {
    const size_t fused = mg_fused_blocks(*g);
    g->mg_fused = fused > 0;
    g->cg_nb_rr = std::max(g->cg_nb, fused);
    g->part_stride = std::max(std::max(g->cg_nb, g->cg_nb_rr), std::max(g->cg_nb_rz, g->cg_nb_dq));
    g->partials = (double*)galloc(*g, S_NSLOT_HOST * g->part_stride * sizeof(double));
    UF_HIP_CHECK(hipMemsetAsync(g->partials, 0, S_NSLOT_HOST * g->part_stride * sizeof(double), g->stream));
  }
  if (mg_splits_update(*g)) {
    // only grids whose iterations use it get the second stream: every
    // stream takes one of the process's few hardware queues, and a batch of
    // grids with idle second streams left fewer queues to its case streams
    UF_HIP_CHECK(hipStreamCreateWithFlags(&g->xstream, hipStreamNonBlocking));
    UF_HIP_CHECK(hipEventCreate(&g->ev_xfork));   // completed inside a dispatch (hipExtLaunchKernel)
    UF_HIP_CHECK(hipEventCreateWithFlags(&g->ev_xjoin, hipEventDisableTiming));
  }
  if (g->esize == 4) init_state<float>(*g);
  else init_state<double>(*g);
  UF_HIP_CHECK(hipStreamSynchronize(g->stream));
  *out = g;
  return UF_OK;
  }
  catch (const HipError& e) {
    free_grid(g);
    delete g;
    return fail(UF_EDEVICE, e.msg);
  }
}

uf_status uf_destroy_grid(uf_grid g) {
  if (!g) return fail(UF_EINVAL, "NULL grid");
  (void)hipStreamSynchronize(g->stream);
  // every fork onto the second solve stream is joined back into the grid's
  // stream within the enqueueing call, unless that call failed half-way
  if (g->xstream) (void)hipStreamSynchronize(g->xstream);
  free_grid(g);
  delete g;
  return UF_OK;
}

uf_status uf_kernel_timer_enable(uf_grid g, uint32_t mask) {
  if (!g) return fail(UF_EINVAL, "NULL grid");
  if (mask >> UF_TK_COUNT) return fail(UF_EINVAL, "unknown kernel bit in the timer mask");
  UF_GUARD_BEGIN
  timer_flush(*g);
  if (mask && g->timer_pool.empty()) {
    const size_t pairs = 4096;
    g->timer_pool.resize(2 * pairs);
    g->timer_id.assign(pairs, 0);
    // no system-scope release on each event: only device timestamps are needed
    for (auto& e : g->timer_pool) UF_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
  g->timer_mask = mask;
  g->timer_used = 0;
  for (int q = 0; q < UF_TK_COUNT; ++q) {
    g->timer_ms[q] = 0.0;
    g->timer_n[q] = 0;
  }
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_kernel_timer_read(uf_grid g, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!g || !total_ms || !launches) return fail(UF_EINVAL, "NULL argument");
  if (kernel < 0 || kernel >= UF_TK_COUNT) return fail(UF_EINVAL, "unknown kernel id");
  UF_GUARD_BEGIN
  timer_flush(*g);
  *total_ms = g->timer_ms[kernel];
  *launches = g->timer_n[kernel];
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_voxelize(const uf_mesh_set* m, int32_t dtype, void* phi_dev, void* stream, double* cast_ms) {
  if (!m || !phi_dev) return fail(UF_EINVAL, "NULL argument");
  if (dtype != UF_F32 && dtype != UF_F64) return fail(UF_EINVAL, "dtype must be UF_F32 or UF_F64");
  if (m->nx < 1 || m->ny < 1 || m->nz < 1) return fail(UF_EINVAL, "grid sizes must be >= 1");
  if ((double)m->nx * m->ny * m->nz > 4.0e9) return fail(UF_EINVAL, "grid too large");
  if (!finite_pos(m->dx) || !finite_pos(m->dy) || !finite_pos(m->dz))
    return fail(UF_EINVAL, "cell sizes must be positive and finite");
  if (m->sub < 1 || m->sub > 16) return fail(UF_EINVAL, "sub must be in 1..16");
  if (m->nobj < 0 || m->nverts < 0 || m->ntris < 0) return fail(UF_EINVAL, "negative count");
  if (m->nobj > 0 && (!m->tri_begin || !m->phi_obj)) return fail(UF_EINVAL, "NULL tri_begin or phi_obj");
  if (m->ntris > 0 && (!m->tris_dev || !m->verts_dev)) return fail(UF_EINVAL, "NULL mesh arrays");
  if (m->nobj > 0) {
    if (m->tri_begin[0] != 0 || m->tri_begin[m->nobj] != m->ntris)
      return fail(UF_EINVAL, "tri_begin must start at 0 and end at ntris");
    for (int o = 0; o < m->nobj; ++o) {
      if (m->tri_begin[o + 1] < m->tri_begin[o]) return fail(UF_EINVAL, "tri_begin must be non-decreasing");
      if (!(m->phi_obj[o] >= 0.0 && m->phi_obj[o] <= 1.0)) return fail(UF_EINVAL, "phi_obj outside [0, 1]");
    }
  } else if (m->ntris != 0) {
    return fail(UF_EINVAL, "triangles without objects");
  }
  UF_GUARD_BEGIN
  const std::string err = voxelize_run(*m, dtype, phi_dev, (hipStream_t)stream, cast_ms);
  if (!err.empty()) return fail(UF_EINVAL, err);
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_smooth_porosity(const uf_smooth_objects* o, int32_t dtype, void* phi_dev, void* stream) {
  if (!o || !phi_dev) return fail(UF_EINVAL, "NULL argument");
  if (dtype != UF_F32 && dtype != UF_F64) return fail(UF_EINVAL, "dtype must be UF_F32 or UF_F64");
  const std::string bad = check_smooth_objects(o);
  if (!bad.empty()) return fail(UF_EINVAL, bad);
  UF_GUARD_BEGIN
  smooth_porosity_run(*o, dtype, phi_dev, (hipStream_t)stream);
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_smooth_porosity_grad(const uf_smooth_objects* o, const double* phibar_dev, double* grad_host,
                                  void* stream) {
  if (!o || !phibar_dev || !grad_host) return fail(UF_EINVAL, "NULL argument");
  const std::string bad = check_smooth_objects(o);
  if (!bad.empty()) return fail(UF_EINVAL, bad);
  if ((long long)o->nboxes + o->ncyls > UF_MAX_GRAD_OBJECTS)
    return fail(UF_EINVAL, "more objects than the gradient kernel holds");
  UF_GUARD_BEGIN
  smooth_porosity_grad_run(*o, phibar_dev, grad_host, (hipStream_t)stream);
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_smooth_porosity_grad_noalloc(const uf_smooth_objects* o, const double* phibar_dev, double* grad_host,
                                          void* stream) {
  if (!o || !phibar_dev || !grad_host) return fail(UF_EINVAL, "NULL argument");
  const std::string bad = check_smooth_objects(o);
  if (!bad.empty()) return fail(UF_EINVAL, bad);
  if ((long long)o->nboxes + o->ncyls > UF_NOALLOC_MAX_OBJECTS)
    return fail(UF_EINVAL, "more objects than the allocation-free gradient's scratch holds (UF_NOALLOC_MAX_OBJECTS)");
  UF_GUARD_BEGIN
  if (stream) {
    int sdev = -1, cur = -1;
    UF_HIP_CHECK(hipStreamGetDevice((hipStream_t)stream, &sdev));
    UF_HIP_CHECK(hipGetDevice(&cur));
    if (sdev != cur) return fail(UF_EINVAL, "the stream belongs to another device than the current one");
  }
  smooth_porosity_grad_noalloc_run(*o, phibar_dev, grad_host, (hipStream_t)stream);
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_set_stream(uf_grid g, void* stream) {
  if (!g) return fail(UF_EINVAL, "NULL grid");
  g->stream = (hipStream_t)stream;
  return UF_OK;
}

uf_status uf_set_porosity(uf_grid g, const void* phi_dev) {
  if (!g || !phi_dev) return fail(UF_EINVAL, "NULL argument");
  UF_GUARD_BEGIN
  const size_t n = (size_t)g->L.nx * g->L.ny * g->L.nz;
  UF_HIP_CHECK(hipMemsetAsync(g->flag, 0, sizeof(int), g->stream));
  if (g->esize == 4) launch_check_range<float>(*g, phi_dev, n);
  else launch_check_range<double>(*g, phi_dev, n);
  check_launch();
  UF_HIP_CHECK(hipMemcpyAsync(g->flag_host, g->flag, sizeof(int), hipMemcpyDeviceToHost, g->stream));
  UF_HIP_CHECK(hipStreamSynchronize(g->stream));
  if (*g->flag_host) return fail(UF_EINVAL, "porosity must be finite and in [0, 1]");
  if (g->esize == 4) launch_porosity<float>(*g, make_params<float>(*g), phi_dev);
  else launch_porosity<double>(*g, make_params<double>(*g), phi_dev);
  check_launch();
  UF_HIP_CHECK(hipMemsetAsync(nf_word(*g), 0, sizeof(int), g->stream));
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_set_field(uf_grid g, int32_t field, const void* src) {
  if (!g || !src) return fail(UF_EINVAL, "NULL argument");
  if (field < 0 || field > UF_PHI) return fail(UF_EINVAL, "unknown field");
  if (field == UF_PHI) return uf_set_porosity(g, src);
  UF_GUARD_BEGIN
  auto go = [&](auto tag) {
    using T = decltype(tag);
    const Params<T> P = make_params<T>(*g);
    void* dst = nullptr;
    switch (field) {
      case UF_U: case UF_V: case UF_W: dst = g->Q[g->cur][field]; break;
      case UF_P: dst = g->X; break;
      case UF_K: dst = g->K[g->kcur]; break;
      case UF_OMEGA: dst = g->Wo[g->kcur]; break;
      case UF_NUT: dst = g->NUT; break;
    }
    launch_pack<T>(*g, P, src, dst, field, 1);
    if (field <= UF_W) launch_face_bc<T>(*g, P, dst, field);
    else if (field == UF_K) launch_cell_bc<T>(*g, P, dst, 1, g->k_in);
    else if (field == UF_OMEGA) launch_cell_bc<T>(*g, P, dst, 1, g->w_in);
    else if (field == UF_NUT) launch_cell_bc<T>(*g, P, dst, 0, 0.0);
  };
  if (g->esize == 4) go(float());
  else go(double());
  check_launch();
  UF_HIP_CHECK(hipMemsetAsync(nf_word(*g), 0, sizeof(int), g->stream));
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_get_field(uf_grid g, int32_t field, void* dst) {
  if (!g || !dst) return fail(UF_EINVAL, "NULL argument");
  if (field < 0 || field > UF_PHI) return fail(UF_EINVAL, "unknown field");
  UF_GUARD_BEGIN
  if (field == UF_PHI) {
    UF_HIP_CHECK(hipMemcpyAsync(dst, g->PHI, (size_t)g->L.nx * g->L.ny * g->L.nz * g->esize,
                                hipMemcpyDeviceToDevice, g->stream));
    return UF_OK;
  }
  auto go = [&](auto tag) {
    using T = decltype(tag);
    const Params<T> P = make_params<T>(*g);
    const void* src = nullptr;
    switch (field) {
      case UF_U: case UF_V: case UF_W: src = g->Q[g->cur][field]; break;
      case UF_P: src = g->X; break;
      case UF_K: src = g->K[g->kcur]; break;
      case UF_OMEGA: src = g->Wo[g->kcur]; break;
      case UF_NUT: src = g->NUT; break;
    }
    launch_pack<T>(*g, P, src, dst, field, 0);
  };
  if (g->esize == 4) go(float());
  else go(double());
  check_launch();
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_step(uf_grid g, int32_t nsteps, uf_step_stats* stats) {
  if (!g) return fail(UF_EINVAL, "NULL grid");
  if (nsteps < 0) return fail(UF_EINVAL, "nsteps must be >= 0");
  UF_GUARD_BEGIN
  StepAccum acc;
  UF_HIP_CHECK(hipEventRecord(g->ev0, g->stream));
  if (g->esize == 4) run_steps<float>(*g, nsteps, acc);
  else run_steps<double>(*g, nsteps, acc);
  UF_HIP_CHECK(hipEventRecord(g->ev1, g->stream));
  if (stats) {
    post_diag(*g);
    UF_HIP_CHECK(hipStreamSynchronize(g->stream));
    float ms = 0;
    UF_HIP_CHECK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
    fill_stats(stats, acc, ms, *g);
  }
  if (acc.nonfinite) return fail(UF_ENONFINITE, "non-finite value in the pressure solve");
  if (acc.nf_state) return fail(UF_ENONFINITE, "non-finite value written by the drag or k-omega stage");
  if (acc.noconv) return fail(UF_ENOCONV, "pressure CG reached cg_maxit");
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_step_batch(const uf_grid* grids, int32_t n, int32_t nsteps, uf_step_stats* stats) {
  if (!grids || n < 1) return fail(UF_EINVAL, "need at least one grid");
  if (nsteps < 0) return fail(UF_EINVAL, "nsteps must be >= 0");
  for (int i = 0; i < n; ++i) {
    if (!grids[i]) return fail(UF_EINVAL, "NULL grid in the batch");
    for (int j = 0; j < i; ++j)
      if (grids[j] == grids[i]) return fail(UF_EINVAL, "a grid appears twice in the batch");
  }
  UF_GUARD_BEGIN
  std::vector<StepAccum> acc(n);
  for (int i = 0; i < n; ++i) UF_HIP_CHECK(hipEventRecord(grids[i]->ev0, grids[i]->stream));
  // a few host threads, each owning every nw-th grid: each runs the rounds
  // below on its grids, so that enqueueing the many small kernels of the
  // cases proceeds in parallel (each grid's kernel sequence is unchanged)
  const int nw = std::max(1, std::min(n, kBatchThreads));
  std::vector<std::string> errs(nw);
  auto work = [&](int w) {
    try {
      for (int s = 0; s < nsteps; ++s) {
        // every owned case's step up to its first CG chunk, then the waits
        // in order: while the host waits for one case the others' work runs
        for (int i = w; i < n; i += nw) {
          Grid& g = *grids[i];
          if (g.esize == 4) step_begin<float>(g, make_params<float>(g));
          else step_begin<double>(g, make_params<double>(g));
        }
        for (int i = w; i < n; i += nw) {
          Grid& g = *grids[i];
          if (g.esize == 4) step_end<float>(g, make_params<float>(g), acc[i]);
          else step_end<double>(g, make_params<double>(g), acc[i]);
        }
      }
    } catch (const HipError& e) {
      errs[w] = e.msg;
    } catch (const std::exception& e) {
      errs[w] = e.what();
    }
  };
  if (nw == 1) {
    work(0);
  } else {
    std::vector<std::thread> pool;
    for (int w = 0; w < nw; ++w) pool.emplace_back(work, w);
    for (auto& t : pool) t.join();
  }
  for (const auto& e : errs)
    if (!e.empty()) return fail(UF_EDEVICE, e);
  for (int i = 0; i < n; ++i) UF_HIP_CHECK(hipEventRecord(grids[i]->ev1, grids[i]->stream));
  if (stats) {
    for (int i = 0; i < n; ++i) post_diag(*grids[i]);
    for (int i = 0; i < n; ++i) {
      UF_HIP_CHECK(hipStreamSynchronize(grids[i]->stream));
      float ms = 0;
      UF_HIP_CHECK(hipEventElapsedTime(&ms, grids[i]->ev0, grids[i]->ev1));
      fill_stats(&stats[i], acc[i], ms, *grids[i]);
    }
  }
  for (int i = 0; i < n; ++i) {
    if (acc[i].nonfinite)
      return fail(UF_ENONFINITE, "non-finite value in the pressure solve of batch entry " + std::to_string(i));
    if (acc[i].nf_state)
      return fail(UF_ENONFINITE, "non-finite value written by the drag or k-omega stage of batch entry " +
                                     std::to_string(i));
    if (acc[i].noconv)
      return fail(UF_ENOCONV, "pressure CG reached cg_maxit in batch entry " + std::to_string(i));
  }
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_pressure_solve(uf_grid g, const void* b_dev, void* x_dev, uf_step_stats* stats) {
  if (!g || !b_dev || !x_dev) return fail(UF_EINVAL, "NULL argument");
  UF_GUARD_BEGIN
  SolveResult r;
  // the solve runs in the grid's pressure array: keep the state's pressure
  // and the warm-start chunk length, and put them back afterwards
  const size_t bytes = g->nelem * g->esize;
  if (!g->Xsave) g->Xsave = galloc(*g, bytes);
  UF_HIP_CHECK(hipMemcpyAsync(g->Xsave, g->X, bytes, hipMemcpyDeviceToDevice, g->stream));
  const int last_iters = g->last_iters;
  auto go = [&](auto tag) {
    using T = decltype(tag);
    const Params<T> P = make_params<T>(*g);
    launch_pack<T>(*g, P, b_dev, g->Qv, UF_P, 1);
    launch_pack<T>(*g, P, x_dev, g->X, UF_P, 1);
    check_launch();
    r = solve_pressure<T>(*g, P, g->Q[g->cur], g->Qv);
    launch_pack<T>(*g, P, g->X, x_dev, UF_P, 0);
    check_launch();
  };
  if (g->esize == 4) go(float());
  else go(double());
  UF_HIP_CHECK(hipMemcpyAsync(g->X, g->Xsave, bytes, hipMemcpyDeviceToDevice, g->stream));
  g->last_iters = last_iters;
  UF_HIP_CHECK(hipStreamSynchronize(g->stream));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->cg_iters = r.iters;
    stats->cg_iters_total = r.iters;
    stats->cg_iters_max = r.iters;
    stats->cg_rel_residual = r.rel;
    stats->converged = !(r.noconv || r.nonfinite);
    stats->nonfinite = r.nonfinite;
  }
  if (r.nonfinite) return fail(UF_ENONFINITE, "non-finite value in the pressure solve");
  if (r.noconv) return fail(UF_ENOCONV, "pressure CG reached cg_maxit");
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_apply_operator(uf_grid g, int32_t op, const void* x_dev, void* y_dev) {
  if (!g || !x_dev || !y_dev) return fail(UF_EINVAL, "NULL argument");
  if (op != UF_OP_POISSON && op != UF_OP_PRECOND) return fail(UF_EINVAL, "unknown operator");
  UF_GUARD_BEGIN
  auto go = [&](auto tag) {
    using T = decltype(tag);
    const Params<T> P = make_params<T>(*g);
    launch_pack<T>(*g, P, x_dev, g->R, UF_P, 1);
    if (op == UF_OP_PRECOND && g->cfg.precond == UF_PC_MG) mg_apply<T>(*g, P, g->R, g->Z);
    else launch_apply<T>(*g, P, op, g->R, g->Z);
    launch_pack<T>(*g, P, g->Z, y_dev, UF_P, 0);
  };
  if (g->esize == 4) go(float());
  else go(double());
  check_launch();
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_objective(uf_grid g, const uf_objective_spec* spec, double* J_host, void* dJ_dstate_dev) {
  if (!g || !spec || !J_host) return fail(UF_EINVAL, "NULL argument");
  if (spec->kind == UF_OBJ_PLANE) {
    const double dz = g->cfg.dz;
    const int nz = g->L.nz;
    if (nz < 2) return fail(UF_EINVAL, "the plane objective needs nz >= 2");
    if (!std::isfinite(spec->z_plane) || spec->z_plane < 0.5 * dz || spec->z_plane > (nz - 0.5) * dz)
      return fail(UF_EINVAL, "z_plane must lie between the first and the last cell centre");
    if (!std::isfinite(spec->s_target) || !std::isfinite(spec->s_min) || !std::isfinite(spec->w_penalty) ||
        spec->w_penalty < 0)
      return fail(UF_EINVAL, "non-finite or negative plane objective parameter");
    UF_GUARD_BEGIN
    constexpr int kBlocks = 256;
    if (!g->obj_part) g->obj_part = (double*)galloc(*g, sizeof(double) * kBlocks * UF_MAX_REGIONS);
    const double zc = spec->z_plane / dz - 0.5;
    const int k0 = std::min(std::max((int)std::floor(zc), 0), nz - 2);
    const double t = zc - k0;
    const long long cols = (long long)g->L.nx * g->L.ny;
    const int nb = (int)std::min<long long>(kBlocks, (cols + 255) / 256);
    if (g->esize == 4)
      launch_plane_objective<float>(*g, k0, t, spec->s_target, spec->s_min, spec->w_penalty, g->obj_part, nb);
    else
      launch_plane_objective<double>(*g, k0, t, spec->s_target, spec->s_min, spec->w_penalty, g->obj_part, nb);
    check_launch();
    std::vector<double> host(nb);
    UF_HIP_CHECK(hipMemcpyAsync(host.data(), g->obj_part, nb * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    UF_HIP_CHECK(hipStreamSynchronize(g->stream));
    double J = 0.0;
    for (int q = 0; q < nb; ++q) J += host[q];
    *J_host = J * g->cfg.dx * g->cfg.dy;
    if (dJ_dstate_dev) {
      const double plane[6] = {(double)k0, t, spec->s_target, spec->s_min, spec->w_penalty, g->cfg.dx * g->cfg.dy};
      double* phibar = (double*)spec->dJ_dphi_accum_dev;
      if (g->esize == 4)
        launch_objective_seed<float>(*g, make_params<float>(*g), nullptr, nullptr, 0, 1, nullptr, dJ_dstate_dev,
                                     plane, phibar);
      else
        launch_objective_seed<double>(*g, make_params<double>(*g), nullptr, nullptr, 0, 1, nullptr, dJ_dstate_dev,
                                      plane, phibar);
      check_launch();
    }
    return UF_OK;
    UF_GUARD_END
  }
  if (spec->kind != UF_OBJ_REGIONS && spec->kind != UF_OBJ_FIELD) return fail(UF_EINVAL, "unknown objective kind");
  const bool field = spec->kind == UF_OBJ_FIELD;
  const int nr = spec->nregions;
  if (nr < 1 || nr > UF_MAX_REGIONS || !spec->boxes) return fail(UF_EINVAL, "region count out of range");
  if (!field && !std::isfinite(spec->u_target)) return fail(UF_EINVAL, "non-finite target speed");
  if (field && !spec->u_target_dev) return fail(UF_EINVAL, "NULL desired velocity field");
  const int n[3] = {g->L.nx, g->L.ny, g->L.nz};
  for (int r = 0; r < nr; ++r)
    for (int a = 0; a < 3; ++a) {
      const int lo = spec->boxes[6 * r + 2 * a], hi = spec->boxes[6 * r + 2 * a + 1];
      if (lo < 0 || hi > n[a] || lo >= hi) return fail(UF_EINVAL, "target region empty or outside the grid");
    }
  UF_GUARD_BEGIN
  constexpr int kBlocks = 256;
  if (!g->obj_part) g->obj_part = (double*)galloc(*g, sizeof(double) * kBlocks * UF_MAX_REGIONS);
  std::vector<int> nb(nr);
  for (int r = 0; r < nr; ++r) {
    const int* b = spec->boxes + 6 * r;
    const long long cells = (long long)(b[1] - b[0]) * (b[3] - b[2]) * (b[5] - b[4]);
    nb[r] = (int)std::min<long long>(kBlocks, (cells + 255) / 256);
    double* part = g->obj_part + (size_t)r * kBlocks;
    if (field) {
      if (g->esize == 4) launch_region_field_diff<float>(*g, b, spec->u_target_dev, part, nb[r]);
      else launch_region_field_diff<double>(*g, b, spec->u_target_dev, part, nb[r]);
    } else {
      if (g->esize == 4) launch_region_speed<float>(*g, b, part, nb[r]);
      else launch_region_speed<double>(*g, b, part, nb[r]);
    }
  }
  check_launch();
  std::vector<double> host((size_t)kBlocks * nr);
  UF_HIP_CHECK(hipMemcpyAsync(host.data(), g->obj_part, host.size() * sizeof(double), hipMemcpyDeviceToHost,
                              g->stream));
  UF_HIP_CHECK(hipStreamSynchronize(g->stream));
  double J = 0.0;
  std::vector<double> coef(nr);   // dJ per unit of the region's cell term (the gradient seed)
  for (int r = 0; r < nr; ++r) {
    const int* b = spec->boxes + 6 * r;
    double s = 0.0;
    for (int q = 0; q < nb[r]; ++q) s += host[(size_t)r * kBlocks + q];
    const double cells = (double)(b[1] - b[0]) * (b[3] - b[2]) * (b[5] - b[4]);
    if (field) {
      J += std::sqrt(s);
      coef[r] = s > 0 ? 1.0 / std::sqrt(s) : 0.0;
    } else {
      const double mean = s / cells;
      J += (mean - spec->u_target) * (mean - spec->u_target);
      coef[r] = 2.0 * (mean - spec->u_target) / cells;
    }
  }
  *J_host = J;
  if (dJ_dstate_dev) {
    const size_t meta = UF_MAX_REGIONS * (6 * sizeof(int) + sizeof(double));
    if (!g->obj_meta) g->obj_meta = galloc(*g, meta);
    double* coef_dev = (double*)g->obj_meta;
    int* boxes_dev = (int*)(coef_dev + UF_MAX_REGIONS);
    UF_HIP_CHECK(hipMemcpyAsync(coef_dev, coef.data(), nr * sizeof(double), hipMemcpyHostToDevice, g->stream));
    UF_HIP_CHECK(
        hipMemcpyAsync(boxes_dev, spec->boxes, 6 * nr * sizeof(int), hipMemcpyHostToDevice, g->stream));
    const int kind = field ? 2 : 0;
    if (g->esize == 4)
      launch_objective_seed<float>(*g, make_params<float>(*g), boxes_dev, coef_dev, nr, kind, spec->u_target_dev,
                                   dJ_dstate_dev, nullptr, nullptr);
    else
      launch_objective_seed<double>(*g, make_params<double>(*g), boxes_dev, coef_dev, nr, kind,
                                    spec->u_target_dev, dJ_dstate_dev, nullptr, nullptr);
    check_launch();
    UF_HIP_CHECK(hipStreamSynchronize(g->stream));   // the host tables above are copied from
  }
  return UF_OK;
  UF_GUARD_END
}

namespace {
uf_status adjoint_entry(uf_grid g, const void* const* state_n_dev, const void* const* state_np1_dev,
                        const void* const* adj_np1_dev, void* const* adj_n_dev, void* dJ_dphi_accum_dev) {
  if (!g || !state_n_dev || !adj_np1_dev || !adj_n_dev) return fail(UF_EINVAL, "NULL argument");
  const bool turb = g->cfg.turb_model == UF_TURB_KOMEGA && (g->cfg.stages & UF_STAGE_TURB);
  const int nf = turb ? 6 : 3;
  for (int c = 0; c < nf; ++c)
    if (!state_n_dev[c] || !adj_np1_dev[c] || !adj_n_dev[c]) return fail(UF_EINVAL, "NULL field pointer");
  if (turb && state_np1_dev)
    for (int c = 0; c < 3; ++c)
      if (!state_np1_dev[c]) return fail(UF_EINVAL, "NULL field pointer");
  if (!turb) state_np1_dev = nullptr;
  UF_GUARD_BEGIN
  SolveResult r;
  if (g->esize == 4)
    r = adjoint_step<float>(*g, state_n_dev, state_np1_dev, adj_np1_dev, adj_n_dev, (double*)dJ_dphi_accum_dev);
  else
    r = adjoint_step<double>(*g, state_n_dev, state_np1_dev, adj_np1_dev, adj_n_dev, (double*)dJ_dphi_accum_dev);
  if (r.nonfinite) return fail(UF_ENONFINITE, "non-finite value in a pressure solve of the reverse step");
  if (r.noconv) return fail(UF_ENOCONV, "a pressure CG of the reverse step reached cg_maxit");
  return UF_OK;
  UF_GUARD_END
}
}  // namespace

uf_status uf_adjoint_step(uf_grid g, const void* const* state_n_dev, const void* const* adj_np1_dev,
                          void* const* adj_n_dev, void* dJ_dphi_accum_dev) {
  return adjoint_entry(g, state_n_dev, nullptr, adj_np1_dev, adj_n_dev, dJ_dphi_accum_dev);
}

uf_status uf_adjoint_step_at(uf_grid g, const void* const* state_n_dev, const void* const* state_np1_dev,
                             const void* const* adj_np1_dev, void* const* adj_n_dev, void* dJ_dphi_accum_dev) {
  if (!state_np1_dev) return fail(UF_EINVAL, "NULL argument");
  return adjoint_entry(g, state_n_dev, state_np1_dev, adj_np1_dev, adj_n_dev, dJ_dphi_accum_dev);
}

uf_status uf_batch_create(const uf_grid* grids, int32_t n, uf_batch* out) {
  if (!grids || !out || n < 1) return fail(UF_EINVAL, "need at least one grid and an output handle");
  if (n > kMaxBatchCases)
    return fail(UF_EINVAL, "a batch holds at most " + std::to_string(kMaxBatchCases) + " grids");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!grids[i]) return fail(UF_EINVAL, "NULL grid in the batch");
    for (int j = 0; j < i; ++j)
      if (grids[j] == grids[i]) return fail(UF_EINVAL, "a grid appears twice in the batch");
    const Grid& g = *grids[i];
    const Grid& g0 = *grids[0];
    if (g.esize != g0.esize) return fail(UF_EINVAL, "the grids of a batch share one dtype");
    const int all = UF_STAGE_ADVECT | UF_STAGE_DIFFUSE | UF_STAGE_DRAG | UF_STAGE_PROJECT;
    if ((g.cfg.stages & all) != all) return fail(UF_EINVAL, "a batch runs the full step (every stage)");
    if (((g.cfg.stages & UF_STAGE_TURB) && g.cfg.turb_model == UF_TURB_KOMEGA) !=
        ((g0.cfg.stages & UF_STAGE_TURB) && g0.cfg.turb_model == UF_TURB_KOMEGA))
      return fail(UF_EINVAL, "the grids of a batch all run the k-omega update, or none does");
    if (!offsets_fit_32(g.L, g.esize)) return fail(UF_EINVAL, "a grid of the batch is too large (4 GiB per field)");
  }
  UF_GUARD_BEGIN
  uf_batch_s* b = new uf_batch_s();
  try {
    for (int i = 0; i < n; ++i) b->g.push_back(grids[i]);
    b->esize = grids[0]->esize;
    b->turb = (grids[0]->cfg.stages & UF_STAGE_TURB) && grids[0]->cfg.turb_model == UF_TURB_KOMEGA;
    b->cs.assign(n, nullptr);
    b->own.assign(n, nullptr);
    b->ev_case.assign(n, nullptr);
    b->solve.assign(n, nullptr);
    UF_HIP_CHECK(hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking));
    for (int i = 0; i < n; ++i) {
      UF_HIP_CHECK(hipStreamCreateWithFlags(&b->cs[i], hipStreamNonBlocking));
      UF_HIP_CHECK(hipEventCreateWithFlags(&b->ev_case[i], hipEventDisableTiming));
    }
    UF_HIP_CHECK(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    UF_HIP_CHECK(hipEventCreateWithFlags(&b->ev_end, hipEventDisableTiming));
    for (int st = 0; st < 6; ++st) {
      b->tune.band[st] = 8;
      b->tune.blocks[st] = 0;
      b->tune.ms[st] = 0.f;
    }
    for (int i = 0; i < n; ++i) b->kcap.push_back(std::max(4, grids[i]->last_iters + 2));
    UF_HIP_CHECK(hipMalloc(&b->kc_dev, sizeof(int) * n));
    UF_HIP_CHECK(hipHostMalloc(&b->kc_host, sizeof(int) * n, hipHostMallocDefault));
    if (b->esize == 4) build_table<float>(*b);
    else build_table<double>(*b);
  } catch (...) {
    release_batch(b);
    delete b;
    throw;
  }
  *out = b;
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_batch_destroy(uf_batch b) {
  if (!b) return fail(UF_EINVAL, "NULL batch");
  (void)hipStreamSynchronize(b->origin);
  release_batch(b);
  delete b;
  return UF_OK;
}

// The state must sit in set 0 with the same k/omega slot in every grid
// (grids stepped only by full steps are).
static std::string batch_ready(const Batch& b) {
  for (const Grid* g : b.g) {
    if (g->cur != 0) return "a grid of the batch holds its state outside the first set";
    if (g->timer_mask) return "kernel timers must be off for batched steps";
  }
  return "";
}

uf_status uf_batch_autotune(uf_batch b, uf_batch_tuning* out) {
  if (!b) return fail(UF_EINVAL, "NULL batch");
  const std::string bad = batch_ready(*b);
  if (!bad.empty()) return fail(UF_EINVAL, bad);
  UF_GUARD_BEGIN
  enter_batch(*b);
  try {
    if (b->esize == 4) autotune<float>(*b);
    else autotune<double>(*b);
  } catch (...) {
    leave_batch(*b);
    throw;
  }
  leave_batch(*b);
  drop_graphs(*b);   // captured with the previous parameters
  if (out)
    for (int st = 0; st < 6; ++st) {
      out->band[st] = b->tune.band[st];
      out->blocks[st] = b->tune.blocks[st];
      out->ms[st] = b->tune.ms[st];
    }
  return UF_OK;
  UF_GUARD_END
}

uf_status uf_batch_step(uf_batch b, int32_t nsteps, uf_step_stats* stats) {
  if (!b) return fail(UF_EINVAL, "NULL batch");
  if (nsteps < 0) return fail(UF_EINVAL, "nsteps must be >= 0");
  const std::string bad = batch_ready(*b);
  if (!bad.empty()) return fail(UF_EINVAL, bad);
  UF_GUARD_BEGIN
  const int n = (int)b->g.size();
  std::vector<StepAccum> acc(n);
  for (int i = 0; i < n; ++i) UF_HIP_CHECK(hipEventRecord(b->g[i]->ev0, b->g[i]->stream));
  enter_batch(*b);
  try {
    if (b->esize == 4) batch_steps<float>(*b, nsteps, acc);
    else batch_steps<double>(*b, nsteps, acc);
  } catch (...) {
    leave_batch(*b);
    throw;
  }
  leave_batch(*b);
  for (int i = 0; i < n; ++i) UF_HIP_CHECK(hipEventRecord(b->g[i]->ev1, b->g[i]->stream));
  if (stats) {
    for (int i = 0; i < n; ++i) post_diag(*b->g[i]);
    for (int i = 0; i < n; ++i) {
      UF_HIP_CHECK(hipStreamSynchronize(b->g[i]->stream));
      float ms = 0;
      UF_HIP_CHECK(hipEventElapsedTime(&ms, b->g[i]->ev0, b->g[i]->ev1));
      fill_stats(&stats[i], acc[i], ms, *b->g[i]);
    }
  }
  for (int i = 0; i < n; ++i) {
    if (acc[i].nonfinite)
      return fail(UF_ENONFINITE, "non-finite value in the pressure solve of batch entry " + std::to_string(i));
    if (acc[i].nf_state)
      return fail(UF_ENONFINITE, "non-finite value written by the drag or k-omega stage of batch entry " +
                                     std::to_string(i));
    if (acc[i].noconv)
      return fail(UF_ENOCONV, "pressure CG reached cg_maxit in batch entry " + std::to_string(i));
  }
  return UF_OK;
  UF_GUARD_END
}

}  // extern "C"
