/*
 * uf.h -- C ABI of the MI355X (gfx950) implementation of one time step of
 * the UrbanFlow incompressible RANS solver (Liu, Rist, Pottmann, Michels,
 * "UrbanFlow: Designing Comfortable Outdoor Areas", arXiv 2204.01117).
 *
 * The library advances the mean flow (u, v, w, p) and the k-omega turbulence
 * fields on a uniform staggered (MAC) grid.  Buildings and trees enter only
 * through a per-cell porosity field (Sec. 3, unified porosity model), so the
 * pressure Poisson matrix depends on the grid and boundary kinds alone and
 * is set up once per grid.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array layouts are z fastest: element (i, j, k) of an (ex, ey, ez) array
 *    sits at (i * ey + j) * ez + k.  Cell fields have extent (nx, ny, nz);
 *    the face velocities u, v, w have (nx+1, ny, nz), (nx, ny+1, nz) and
 *    (nx, ny, nz+1).  Face u(i, j, k) lies at (i dx, (j+1/2) dy, (k+1/2) dz).
 *  - Every pointer named *_dev is a device pointer (hipMalloc'd or a torch
 *    CUDA tensor) holding values in the grid's dtype (float for UF_F32,
 *    double for UF_F64).  The library only borrows it for the duration of
 *    the call; reads and writes are enqueued on the grid's stream, so the
 *    caller must keep the memory alive until the stream reaches them.
 *  - The handle owns all of its internal device buffers.
 *  - Functions return a uf_status.  On an error the thread-local message is
 *    available from uf_last_error().  Argument errors (UF_EINVAL) are
 *    detected before anything is enqueued and leave the state unchanged.
 *  - A handle must not be used from two host threads at once.
 */
#ifndef UF_H
#define UF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct uf_grid_s* uf_grid;

typedef enum {
  UF_OK = 0,
  UF_EINVAL = 1,      /* bad argument or configuration; nothing was enqueued   */
  UF_ENOMEM = 2,      /* device allocation failed                               */
  UF_EDEVICE = 3,     /* a HIP runtime call failed                              */
  UF_ENOCONV = 4,     /* pressure CG stopped at cg_maxit; the step completed    */
  UF_ENONFINITE = 5,  /* a NaN/Inf appeared in the state; the step completed   */
  UF_ESTATE = 6,      /* call not valid in the handle's current state          */
  UF_ENOTIMPL = 7     /* entry point declared but not implemented in this version */
} uf_status;

/* Boundary kind of each domain side, sides ordered -x, +x, -y, +y, -z, +z
 * (-z is the ground).  Sec. 3 "Porosity Model vs. Solid-wall Boundary
 * Conditions": Dirichlet velocity at an inlet, zero normal derivative at an
 * outlet with zero pressure in the outlet ghost cells, no-slip at walls,
 * zero normal pressure derivative at inlets and walls.  SLIP is a
 * free-slip wall (zero normal velocity, zero tangential stress).
 * UF_BC_AUTO: a vertical side is an inlet if the wind enters through it,
 * an outlet otherwise; ground WALL, sky SLIP. */
enum { UF_BC_AUTO = -1, UF_BC_INLET = 0, UF_BC_OUTLET = 1, UF_BC_WALL = 2, UF_BC_SLIP = 3 };
enum { UF_F32 = 0, UF_F64 = 1 };
enum { UF_TURB_OFF = 0, UF_TURB_KOMEGA = 1 };
/* Pressure CG preconditioner: none, Jacobi, the first- or second-order
 * approximate inverse M^-1 = K^T K of Sec. 3 (full products, see
 * uf_config.ai_omega; AI2 takes two passes through the grid's scratch
 * vector), or a geometric multigrid V-cycle. */
enum { UF_PC_NONE = 0, UF_PC_JACOBI = 1, UF_PC_AI1 = 2, UF_PC_AI2 = 3, UF_PC_MG = 4 };
/* Inflow profile: uniform speed, the log-law of Sec. 5.1, or a table. */
enum { UF_INFLOW_UNIFORM = 0, UF_INFLOW_LOGLAW = 1, UF_INFLOW_PROFILE = 2 };
/* Stages of a step (Sec. 3 time splitting); all on by default. */
enum { UF_STAGE_ADVECT = 1, UF_STAGE_DIFFUSE = 2, UF_STAGE_DRAG = 4,
       UF_STAGE_PROJECT = 8, UF_STAGE_TURB = 16, UF_STAGE_ALL = 31 };

typedef enum { UF_U = 0, UF_V = 1, UF_W = 2, UF_P = 3, UF_K = 4, UF_OMEGA = 5,
               UF_NUT = 6, UF_PHI = 7 } uf_field;

typedef struct {
  int32_t nx, ny, nz;           /* cells per axis, each >= 1; nx, ny >= 2       */
  double dx, dy, dz;            /* cell size in metres, > 0                     */
  double dt;                    /* time step in seconds, > 0                    */
  int32_t dtype;                /* UF_F32 or UF_F64 (storage and arithmetic)    */
  int32_t bc[6];                /* side kinds; at least one side must be OUTLET */
  int32_t inflow_kind;          /* UF_INFLOW_*                                  */
  double u_ref, z_ref, z0, karman; /* log-law: u(z) = (u_fr / karman) ln(z/z0),
                                    friction speed u_fr = u_ref karman /
                                    ln(z_ref / z0); zero for z <= z0            */
  double wind_dir_deg;          /* wind direction in the horizontal plane,
                                   0 = +x, 90 = +y                              */
  const double* inflow_profile; /* host array of nz speeds (UF_INFLOW_PROFILE);
                                   copied during uf_create_grid                 */
  double nu, rho;               /* kinematic viscosity, density                 */
  int32_t turb_model;           /* UF_TURB_OFF keeps nu_t = 0                   */
  double turb_I, turb_L;        /* inlet intensity and length scale (Sec. 3);
                                   turb_L <= 0 selects 0.1 x domain height      */
  double k_min, omega_min;      /* floors of k and omega                        */
  double Cd, a, b, e;           /* drag law C_d a ((1 - phi)/(phi + e))^b       */
  int32_t precond;              /* UF_PC_*                                      */
  double ai_omega;              /* relaxation of the AI preconditioner, (0, 2)  */
  double cg_tol;                /* stop at ||r|| <= cg_tol ||b|| (criterion 0)
                                   or (M^-1 r . r) < cg_tol ||b||^2 (criterion 1,
                                   the paper's appendix A.3 test)               */
  int32_t cg_maxit;
  int32_t cg_criterion;
  int32_t stages;               /* UF_STAGE_* mask                              */
  void* stream;                 /* hipStream_t used for all work; NULL = null stream */
  /* Device allocator of every buffer the grid owns (state fields, the
   * pressure solve's vectors and partial sums, multigrid levels, the adjoint
   * workspace): alloc(bytes, alloc_ctx) returns device memory of the current
   * device usable on `stream`, or NULL (the call then fails with UF_ENOMEM);
   * free(ptr, alloc_ctx) releases it, from uf_destroy_grid after the stream
   * has been synchronised.  Set both or neither; NULL means hipMalloc and
   * hipFree.  A framework's caching allocator (PyTorch's) plugs in here, so
   * the grid's memory is pooled and accounted with the caller's tensors. */
  void* (*alloc)(size_t bytes, void* alloc_ctx);
  void (*free)(void* ptr, void* alloc_ctx);
  void* alloc_ctx;
} uf_config;

typedef struct {
  int32_t cg_iters;             /* CG iterations of the last step               */
  int32_t cg_iters_total;       /* summed over the steps of the call            */
  double cg_rel_residual;       /* ||r|| / ||b|| at exit of the last solve      */
  int32_t converged;            /* 1 if every solve of the call converged       */
  int32_t nonfinite;            /* 1 if a NaN/Inf was seen in a solve, or in the
                                   velocity the drag stage wrote or the k, omega
                                   the k-omega update wrote (see uf_step)       */
  float ms;                     /* wall time of the call on the stream          */
  int32_t cg_iters_max;         /* largest per-step CG iteration count of the call */
  /* Diagnostics of the state at the end of the call (one extra pass over the
   * grid, made only when stats are requested): */
  double max_div;               /* max over cells of |div_h u| (1/s): the
                                   projection's residual divergence             */
  double max_cfl;               /* max over cells of dt sum_d |u_d| / h_d with
                                   cell-centre velocities: the stability number
                                   of the upwind k-omega advection (Sec. 3 time
                                   step restriction)                            */
  double nut_clip_frac;         /* fraction of cells whose eddy viscosity sits
                                   at the limiter nu_max - nu (Sec. 3 viscosity
                                   limiter); 0 without the k-omega model       */
} uf_step_stats;

/* Create a grid and its state.  The initial state has the inflow profile on
 * every face, k and omega at their inlet values (Sec. 3: k = 1.5 (I U_ref)^2,
 * omega = k^(1/2) / (C_mu^(1/4) L)), p = 0, nu_t from k and omega, and
 * porosity 1 everywhere.  Errors: UF_EINVAL for a bad configuration (sizes,
 * dt <= 0, no outlet side, nu above the explicit-diffusion bound, unknown
 * enums), UF_ENOMEM, UF_EDEVICE.  *out is set only on success. */
uf_status uf_create_grid(const uf_config* cfg, uf_grid* out);

/* The side kinds a configuration resolves to, sides ordered -x, +x, -y, +y,
 * -z, +z: explicit kinds as given, UF_BC_AUTO replaced by the rule above (a
 * vertical side is an inlet when the inward normal's dot product with the
 * wind direction (cos, sin of wind_dir_deg) exceeds 1e-12, an outlet
 * otherwise; the ground a wall, the sky a slip surface).  Host only, no
 * device work.  UF_EINVAL for NULL arguments, a non-finite wind direction or
 * an unknown kind. */
uf_status uf_resolve_bc(const uf_config* cfg, int32_t out[6]);

/* Release a grid and all of its device memory (synchronises its stream). */
uf_status uf_destroy_grid(uf_grid g);

/* Set the cell porosity phi in [0, 1] (1 = air, 0 = solid; Sec. 3 unified
 * porosity model, appendix A.2 phi = 1 - V_s/V) from nx*ny*nz device
 * values, and derive the drag coefficient C_d a ((1-phi)/(phi+e))^b of each
 * cell.  Synchronises the stream to validate: UF_EINVAL (state unchanged)
 * if any value is NaN or outside [0, 1]. */
uf_status uf_set_porosity(uf_grid g, const void* phi_dev);

/* Objects as closed triangle meshes, for uf_voxelize (Sec. 3, urban model
 * resolving: the design tool hands over building and tree surfaces as
 * closed triangle meshes). */
typedef struct {
  int32_t nx, ny, nz;          /* grid cells, each >= 1; cell (i, j, k) spans
                                  [i dx, (i+1) dx) x [j dy, (j+1) dy) x
                                  [k dz, (k+1) dz), origin at the grid corner  */
  double dx, dy, dz;           /* cell size, > 0 and finite                     */
  int32_t sub;                 /* sub-samples per axis and cell, 1 .. 16        */
  int32_t nobj;                /* objects, >= 0                                 */
  const int32_t* tri_begin;    /* host, nobj + 1 offsets: object o owns the
                                  triangles tri_begin[o] .. tri_begin[o+1]-1;
                                  tri_begin[0] = 0, non-decreasing,
                                  tri_begin[nobj] = ntris                       */
  const double* phi_obj;       /* host, nobj porosities inside each object, in
                                  [0, 1] (0 = solid building, e.g. 0.5 = tree) */
  int32_t nverts, ntris;
  const double* verts_dev;     /* device, nverts x 3 coordinates (x, y, z), m   */
  const int32_t* tris_dev;     /* device, ntris x 3 vertex indices              */
} uf_mesh_set;

/* Cell porosity of mesh objects (Sec. 3, urban model resolving: a first
 * pass takes each object's axis-aligned bounding box, a second decides
 * inside or outside by the even-odd rule on a ray, whose surface crossings
 * come from the Moller-Trumbore ray/triangle test; cut cells are resolved
 * by uniform sub-division, phi = fraction of sub-samples outside).  The
 * sub-samples of cell (i, j, k) sit at ((i + (s + 1/2)/sub) dx, ...), the
 * rays run along +x, and an object with porosity phi_o gives the cell
 * 1 - f_in (1 - phi_o) with f_in its fraction of samples inside; overlapping
 * objects take the smallest value, and 1 is air.  Every cell that an
 * object's bounding box overlaps is tested.
 *
 * phi_dev: nx*ny*nz values (dtype UF_F32 or UF_F64, z fastest, the layout
 * uf_set_porosity takes), written on `stream` (a hipStream_t, NULL = null
 * stream); the call synchronises the stream and allocates temporary device
 * memory.  Inside counts are exact integers and the combination is a
 * minimum, so the result is deterministic.  Errors, before phi is written:
 * UF_EINVAL for a NULL or inconsistent argument, sizes or sub out of range,
 * phi_obj outside [0, 1], a vertex index outside [0, nverts) or a
 * non-finite coordinate.  UF_EINVAL after the fact (phi then unspecified)
 * when a sample line crosses one object's surface more than 14 times. */
uf_status uf_voxelize(const uf_mesh_set* mesh, int32_t dtype, void* phi_dev, void* stream,
                      double* cast_ms);
/* cast_ms (nullable): receives the duration of the ray-casting kernel
 * (events carried in its dispatch), 0 when no object meets the grid. */

/* Objects with smoothed faces, for design parameters that move buildings
 * by fractions of a cell (Sec. 3 motivates the cut-cell volume ratio by the
 * boundary sliding within a cell during optimisation): each object's
 * indicator is a product of logistic steps sig(t) = 1 / (1 + e^-t) of width
 * `width` across its faces, evaluated at cell centres:
 *   box       prod over axes sig((p - lo) / w) sig((hi - p) / w)
 *   cylinder  sig((R - rho) / w) sig((z - z0) / w) sig((z1 - z) / w)
 * (rho: distance from the axis; no lower step when z0 <= 0, so objects on
 * the ground stay solid down to it), and the porosity of a cell is
 * min(1, min over objects of 1 - I (1 - phi_o)). */
typedef struct {
  int32_t nx, ny, nz;          /* grid cells, each >= 1                         */
  double dx, dy, dz;           /* cell size, > 0                                */
  double width;                /* step width in metres, > 0                     */
  int32_t nboxes;              /* >= 0                                          */
  const double* boxes;         /* host, 7 per box: x0, x1, y0, y1, z0, z1, phi  */
  int32_t ncyls;               /* >= 0                                          */
  const double* cylinders;     /* host, 6 per cylinder: cx, cy, R, z0, z1, phi  */
} uf_smooth_objects;

/* Porosity of smoothed objects into phi_dev (nx*ny*nz values of dtype
 * UF_F32/UF_F64, z fastest, the layout uf_set_porosity takes), computed in
 * FP64 on `stream`; synchronises the stream.  UF_EINVAL (nothing written)
 * for NULL or inconsistent arguments, non-finite values, phi outside
 * [0, 1] or a negative radius. */
uf_status uf_smooth_porosity(const uf_smooth_objects* objects, int32_t dtype, void* phi_dev, void* stream);

/* Reverse of uf_smooth_porosity (the design-parameter chain of the
 * adjoint): given phibar_dev = dJ/dphi (device, float64, nx*ny*nz, z
 * fastest), writes dJ/d(object parameter) to grad_host: 7 per box (x0, x1,
 * y0, y1, z0, z1, phi) then 6 per cylinder (cx, cy, R, z0, z1, phi).  Each
 * cell follows the first object reaching its minimum (the branch the
 * forward took); a ground-standing object (z0 <= 0) has no z0 derivative.
 * FP64, summed in a fixed order (the same bits on every run).  Synchronises
 * `stream`.  UF_EINVAL as uf_smooth_porosity,
 * and for more than UF_MAX_GRAD_OBJECTS objects. */
enum { UF_MAX_GRAD_OBJECTS = 1024 };
uf_status uf_smooth_porosity_grad(const uf_smooth_objects* objects, const double* phibar_dev, double* grad_host,
                                  void* stream);

/* uf_smooth_porosity_grad without allocating: for callers that cannot
 * allocate device memory (code under stream or graph capture, serving loops,
 * hosts that forbid hipMalloc).  Same arguments, result and errors as
 * uf_smooth_porosity_grad (the sums may differ in the last bits: per-block
 * partials are summed on the device, with fewer blocks when many objects
 * fill the rows), for at most UF_NOALLOC_MAX_OBJECTS boxes and cylinders
 * together (UF_EINVAL beyond, nothing enqueued).  The work memory is one
 * fixed 8 MiB device array per GPU, kept by the library until the process
 * ends; every call on a GPU reuses it, so calls that overlap on one GPU
 * (other host threads, or streams not ordered with this one) race.  The
 * current device must be the stream's (UF_EINVAL otherwise).  Copies the
 * object rows from host memory on `stream` and synchronises it. */
enum { UF_NOALLOC_MAX_OBJECTS = 1024 };
uf_status uf_smooth_porosity_grad_noalloc(const uf_smooth_objects* objects, const double* phibar_dev,
                                          double* grad_host, void* stream);

/* Overwrite one state field from a device array in the layout given by
 * uf_field_extent (checkpoint restore, parity tests).  Boundary values are
 * re-imposed after the copy.  UF_PHI is the same as uf_set_porosity. */
uf_status uf_set_field(uf_grid g, int32_t field, const void* src_dev);

/* Copy one state field to a device array (asynchronous on the stream). */
uf_status uf_get_field(uf_grid g, int32_t field, void* dst_dev);

/* Extent of a field for a configuration; returns the element count, or -1
 * for an unknown field.  dims may be NULL. */
int64_t uf_field_extent(const uf_config* cfg, int32_t field, int32_t dims[3]);

/* Advance nsteps time steps: advection (MacCormack), explicit diffusion,
 * porosity drag, pressure projection, then the k-omega update (Sec. 3
 * "Discretization and Numerical Integration": terms integrated one by one,
 * turbulence after the projection).  The pressure solve starts from the
 * previous pressure, or from zero when that is the worse start (its
 * residual longer than the right-hand side).  The call returns after the last step's solve has
 * been observed to finish; later kernels may still be in flight unless
 * stats is non-NULL, which synchronises and fills it.  Returns UF_ENOCONV or
 * UF_ENONFINITE if some solve did not converge or saw a non-finite value;
 * the state has advanced in either case.  The drag and k-omega stages also
 * raise a device flag when they write a NaN/Inf; it is read with each solve's
 * status and, with stats, at the end of the call (without stats, a flag the
 * last step's k-omega update raised is reported by the next call).  The flag
 * stays set, and every uf_step returns UF_ENONFINITE, until uf_set_field or
 * uf_set_porosity overwrites the state. */
uf_status uf_step(uf_grid g, int32_t nsteps, uf_step_stats* stats);

/* Advance n independent grids by nsteps each (several cases at once: the
 * wind directions and design variants of Sec. 4 and 5, or the N + 1
 * simulations of a forward-difference gradient).  Each grid computes exactly
 * what uf_step computes for it, bit for bit; the work is enqueued by up to
 * four host threads, each owning every fourth grid, in rounds (every owned
 * grid's step up to its first pressure-CG chunk, then each one's
 * completion), so that one grid's host round trip overlaps the others'
 * kernels.  The call returns when all threads have finished.  Give each grid its own
 * stream (uf_config.stream) for the kernels to overlap.  stats, if non-NULL,
 * has n entries and synchronises like uf_step.  UF_EINVAL (nothing
 * enqueued) for NULL, n < 1, a NULL grid or a grid listed twice; UF_ENOCONV
 * or UF_ENONFINITE as uf_step, naming the first such batch entry. */
uf_status uf_step_batch(const uf_grid* grids, int32_t n, int32_t nsteps, uf_step_stats* stats);

/* A batch: n grids advanced together with one launch per stage for all of
 * them (the same cases as uf_step_batch; the paper's wind-direction and
 * design studies, Sec. 4 and 5).  Each face stage of the step (MacCormack
 * predictor and corrector, diffusion, drag, projection) and the k-omega
 * update is one kernel walking a single queue of every case's blocks.
 * Each case's pressure solve (its start from the drag output and a
 * captured number of CG iterations -- the last solve's count plus two;
 * iterations past convergence return at once) is a hipGraph of its own,
 * replayed on the case's own stream so that the cases' solves overlap; the
 * face stages before it and the projection and k-omega update after it are
 * two more hipGraphs.  Between the solves and the back half the host reads
 * every case's solve status and enqueues further iterations for a case
 * that needs them (that case's solve is then captured again, longer).  Each
 * grid computes exactly what uf_step computes for it, bit for bit.
 *
 * uf_batch_create: 1 to UF_BATCH_MAX_GRIDS grids (not owned; they must
 * outlive the batch and keep their buffers) that share one dtype, run
 * every stage of the step, all with or all without the k-omega update, and
 * have fields below 4 GiB; UF_EINVAL otherwise (nothing created).  The batch makes its own streams;
 * a call orders them after each grid's stream and the grid's stream after
 * them.  uf_batch_step: nsteps steps; the grids must hold their state as
 * full steps leave it (uf_step or uf_batch_step with every stage) and have
 * kernel timers off (UF_EINVAL otherwise); stats as uf_step_batch.
 * uf_batch_autotune: times each stage's launch for band widths of 4, 8 and
 * 16 blocks (blocks of one band of the (j, k) points walk x together) and
 * for persistent grids of 2, 4 or 8 blocks per compute unit or one block
 * per queue entry, on the sets a step overwrites (the state is only read),
 * keeps the fastest of three runs for each stage, and reports the choice
 * (stages: predictor, corrector, diffusion, drag, projection, k-omega;
 * blocks 0 = one per queue entry) when out is non-NULL.  Until it is
 * called every stage uses bands of 8 and one block per queue entry. */
#define UF_BATCH_MAX_GRIDS 64
typedef struct uf_batch_s* uf_batch;
typedef struct {
  int32_t band[6];
  int32_t blocks[6];
  float ms[6];
} uf_batch_tuning;
uf_status uf_batch_create(const uf_grid* grids, int32_t n, uf_batch* out);
uf_status uf_batch_autotune(uf_batch b, uf_batch_tuning* out);
uf_status uf_batch_step(uf_batch b, int32_t nsteps, uf_step_stats* stats);
uf_status uf_batch_destroy(uf_batch b);

/* Solve A x = b with the grid's pressure operator (A = -L_h with the
 * boundary rows described above; SPD), preconditioner and tolerance; x_dev
 * holds the initial guess on entry and the solution on exit (a guess whose
 * residual is longer than b is replaced by zero, as in uf_step's solves).  b_dev and
 * x_dev are nx*ny*nz device arrays.  The grid's state, its pressure
 * included, is left as it was (the first call allocates one cell array to
 * keep it).  Synchronises; stats may be NULL. */
uf_status uf_pressure_solve(uf_grid g, const void* b_dev, void* x_dev, uf_step_stats* stats);

/* Apply a fixed linear operator of the pressure solve to a cell array:
 * op 0 = A (the Poisson matrix), op 1 = the configured preconditioner M^-1.
 * x_dev and y_dev are nx*ny*nz device arrays and must not overlap. */
enum { UF_OP_POISSON = 0, UF_OP_PRECOND = 1 };
uf_status uf_apply_operator(uf_grid g, int32_t op, const void* x_dev, void* y_dev);

/* Design objectives (Sec. 4: the simulator returns the flow of a design and
 * an objective scores it).
 *
 * UF_OBJ_REGIONS, the target-region objective of the Nurnberg study:
 * L = sum_i (s_i - u_target)^2 with s_i the mean wind speed over the cells
 * of target region i, the speed of a cell being |u| of its cell-centre
 * velocity (the mean of its two faces per component).  Regions are boxes of
 * cell indices, half-open: i0 <= i < i1, j0 <= j < j1, k0 <= k < k1.
 *
 * UF_OBJ_PLANE, pedestrian comfort on a horizontal plane at height z_plane:
 * L = dx dy sum over columns (i, j) of phi_p [(s - s_target)^2 +
 * w_penalty max(0, s_min - s)^2], where the cell-centre velocity and the
 * porosity phi are interpolated linearly in z between the two cell centres
 * around the plane and s = sqrt(|u_p|^2 + 1e-12) (solid columns weigh 0).
 *
 * UF_OBJ_FIELD, the general form of Sec. 4: L = sum_i ||F_i(u) - F_i(u_t)||_2
 * with u_t a desired flow and F_i the cell-centre velocities of target
 * region i (the same boxes as UF_OBJ_REGIONS): per region the Euclidean norm
 * of the difference over all its cells and components. */
enum { UF_OBJ_REGIONS = 0, UF_OBJ_PLANE = 1, UF_OBJ_FIELD = 2 };
typedef struct {
  int32_t nregions;            /* UF_OBJ_REGIONS: 1 .. UF_MAX_REGIONS           */
  const int32_t* boxes;        /* host, 6 per region: i0, i1, j0, j1, k0, k1     */
  double u_target;             /* ideal mean speed (0.55 m/s in the paper)       */
  int32_t kind;                /* UF_OBJ_REGIONS or UF_OBJ_PLANE                 */
  double z_plane;              /* UF_OBJ_PLANE: height in metres, between the
                                  first and the last cell centre (nz >= 2)       */
  double s_target, s_min;      /* comfortable speed, stagnation threshold        */
  double w_penalty;            /* weight of the stagnation term, >= 0            */
  const void* u_target_dev;    /* UF_OBJ_FIELD: device, 3 * nx*ny*nz desired
                                  cell-centre velocities in the grid's dtype:
                                  the u, v, then w block, each z fastest       */
  void* dJ_dphi_accum_dev;     /* UF_OBJ_PLANE with a state gradient: NULL, or
                                  device float64 nx*ny*nz (z fastest) to which
                                  the objective's direct porosity derivative
                                  (its phi weight) is added                    */
} uf_objective_spec;
enum { UF_MAX_REGIONS = 64 };

/* Evaluates L on the current state into *J_host (synchronises the grid's
 * stream).  Speeds are summed in FP64 in a fixed order (deterministic).
 * UF_EINVAL for a NULL argument, an unknown kind, a region count out of
 * range, an empty box, a box outside the grid, a plane outside the cell
 * centres or a non-finite or negative parameter, before any work.
 * dJ_dstate_dev: NULL, or a device buffer (grid dtype) that receives dJ/du
 * for every face of the current state -- the u block ((nx+1) ny nz), then
 * the v block (nx (ny+1) nz), then the w block (nx ny (nz+1)), each z
 * fastest -- the seed of uf_adjoint_step.  Each face is half of the
 * cell-centre velocity of each adjacent cell; a cell of zero speed
 * contributes nothing to the mean-speed gradient.  Fixed boundary faces
 * get their derivative too (the reverse step ignores it).  For the plane
 * objective the two layers around the plane carry it (weights 1 - t and t
 * of the interpolation), and its direct porosity derivative goes to
 * spec->dJ_dphi_accum_dev when that is set.  The value is read back
 * synchronously; the plane gradient's kernels may still run when the call
 * returns (stream order). */
uf_status uf_objective(uf_grid g, const uf_objective_spec* spec, double* J_host, void* dJ_dstate_dev);

/* One reverse step of the discrete adjoint (gradients of a Sec. 4 design
 * objective, an extension: the paper itself differences the simulator).
 * The state the reverse carries is (u, v, w) -- plus (k, omega, nu_t) when
 * the k-omega model runs in the step (turb_model UF_TURB_KOMEGA with
 * UF_STAGE_TURB); call its field count F (3 or 6).  Given the state x^n a
 * step started from and a = dJ/dx^{n+1} for its result, writes
 * dJ/dx^n = (dx^{n+1}/dx^n)^T a and adds (dx^{n+1}/dphi)^T a into the
 * porosity gradient.  The Jacobian is the exact derivative of the discrete
 * step the library runs (its enabled stages), taken at the branch the
 * forward took at every max, min and clamp (a MacCormack value clamped to
 * its sample range follows that sample; a face stopped by the drag passes
 * nothing; a floored k or omega and a clipped nu_t pass nothing through the
 * clipped argument); the pressure solve is treated as exact, its adjoint
 * being the same projection applied to a (the step's projection is
 * symmetric), solved to cg_tol with its own warm start kept in the grid
 * between calls.  nu_t is a state field of its own: the step's diffusion
 * reads the nu_t given, and the new nu_t is the k-omega update's output.
 *   state_n_dev[F]: device, compact fields of x^n in the grid's dtype, in
 *                   the order u, v, w, k, omega, nu_t (extents as
 *                   uf_field_extent); fixed boundary faces and the inlet
 *                   ghosts of k and omega follow the boundary conditions, as
 *                   uf_set_field does.
 *   adj_np1_dev[F]: device, compact dJ/dx^{n+1}; values on fixed faces are
 *                   ignored (those faces are constants).
 *   adj_n_dev[F]:   device, compact output dJ/dx^n (zero on fixed faces);
 *                   may alias adj_np1_dev.
 *   dJ_dphi_accum_dev: NULL, or device float64 [nx*ny*nz] (z fastest) to
 *                   which the porosity derivative is added (chain through
 *                   the drag coefficient of the porosity map).
 * The grid's state, pressure and statistics are left as they were; the
 * porosity is the grid's current one, and without the k-omega update so is
 * the (then fixed) eddy viscosity.  With the model the step is recomputed
 * up to x^{n+1}, including a forward pressure solve from zero.  Adds are
 * atomic where the forward gathers, so FP32 results can differ in the last
 * bits between runs.  The first call allocates a workspace of 48 padded
 * fields.  Work is enqueued on the grid's stream; the call waits only for
 * the pressure solves' status, so the kernels after them may still run
 * when it returns (stream order).  UF_EINVAL for a NULL argument or field
 * pointer; UF_ENOCONV / UF_ENONFINITE from a pressure solve. */
uf_status uf_adjoint_step(uf_grid g, const void* const* state_n_dev, const void* const* adj_np1_dev,
                          void* const* adj_n_dev, void* dJ_dphi_accum_dev);

/* uf_adjoint_step with the state after the step given: state_np1_dev[3]
 * (device, compact u, v, w of x^{n+1} -- the result of stepping x^n, as
 * uf_get_field returns it; the caller running the reverse sweep holds it as
 * the previous call's state_n_dev).  With the k-omega update in the step
 * the turbulence reverse linearises at these fields instead of recomputing
 * them (no forward pressure solve); without it they are not read.  Passing
 * anything but the step's own result gives a wrong gradient.  Errors as
 * uf_adjoint_step, and UF_EINVAL for a NULL state_np1_dev. */
uf_status uf_adjoint_step_at(uf_grid g, const void* const* state_n_dev, const void* const* state_np1_dev,
                             const void* const* adj_np1_dev, void* const* adj_n_dev, void* dJ_dphi_accum_dev);

/* Kernel timer.  While enabled, every launch of the selected kernels carries
 * a pair of HIP events in its own dispatch (hipExtLaunchKernel start/stop
 * events: the kernel's begin and end, no separate marker packets), and the
 * elapsed times are accumulated (for the benchmark's per-kernel bandwidth
 * figures).  UF_TK_MG_COARSE covers every multigrid kernel below the finest
 * level; UF_TK_MG_UPDATE0 is the level-0 restriction that also performs the
 * CG update (the multigrid preconditioner inside the iterations),
 * UF_TK_MG_RUPD0 its marching form on large grids, which performs the
 * residual update only (x += alpha d runs on the solve's second stream and
 * is not timed), and UF_TK_MG_DOWN0 the plain restriction.  mask: bit UF_TK_* per kernel; 0 disables.  Enabling resets the
 * totals.  uf_kernel_timer_read synchronises and returns the total
 * milliseconds and the number of launches of one kernel since the timer
 * was enabled. */
enum { UF_TK_CG_AD = 0, UF_TK_CG_AXPY = 1, UF_TK_CG_PRECOND = 2, UF_TK_MG_DOWN0 = 3, UF_TK_MG_UP0 = 4,
       UF_TK_MG_COARSE = 5, UF_TK_CG_INIT = 6, UF_TK_ADVECT_FWD = 7, UF_TK_ADVECT_CORR = 8,
       UF_TK_DIFFUSE = 9, UF_TK_DRAG = 10, UF_TK_PROJECT = 11, UF_TK_TURB = 12, UF_TK_MG_UPDATE0 = 13,
       UF_TK_MG_RUPD0 = 14, UF_TK_COUNT = 15 };
uf_status uf_kernel_timer_enable(uf_grid g, uint32_t mask);
uf_status uf_kernel_timer_read(uf_grid g, int32_t kernel, double* total_ms, int64_t* launches);

/* Replace the stream used by the grid (e.g. torch's current stream). */
uf_status uf_set_stream(uf_grid g, void* stream);

/* Human-readable message of the last error on this host thread. */
const char* uf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* UF_H */
