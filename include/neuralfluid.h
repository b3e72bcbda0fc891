/*
 * neuralfluid.h -- C ABI of the MI355X (gfx950) library for one differentiable
 * Navier-Stokes step on a 3D staggered (MAC) grid with cut-cell solids.
 *
 * Method: NeuralFluid (arXiv 2405.14903), Sec. "Differentiable Navier-Stokes
 * Simulation": operator splitting into semi-Lagrangian advection
 * (Eq. advection_matrix; two-stage back-trace of App. B, Eqs. advection_1/2),
 * explicit viscosity (Eq. viscosity_matrix; App. B Eq. apply_force), and a
 * variational pressure projection with per-face fluid fractions alpha
 * (Eq. projection_matrix, Eq. u_next_matrix), solved matrix-free by
 * multigrid-preconditioned CG; plus the adjoint of each stage (Sec.
 * "Back-propagation through Time" and "Back-propagation through Geometry").
 * A constant body force (gravity) is this library's addition, used to check
 * hydrostatic balance.
 * Viscosity: U^ = (I - nu dt/dx^2 G_f^T G_f) U~ with G_f the differences of
 * each velocity component over the edges of its own face lattice (the 7-point
 * Laplacian inside; no edge leaves the lattice at a domain side, so the
 * tangential components have zero normal derivative there).  It is explicit:
 * stable for nu dt / dx^2 <= 1/6 (sim_set_dt lets a caller sub-step).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid: n = (nx, ny, nz) cells of width dx; cell (i,j,k) centre at
 * ((i+1/2)dx, (j+1/2)dx, (k+1/2)dx).  Layouts (all x fastest):
 *   cells    : i + nx*(j + ny*k)                       (nx*ny*nz values)
 *   velocity : x-faces (nx+1)*ny*nz, then y-faces nx*(ny+1)*nz, then
 *              z-faces nx*ny*(nz+1), concatenated; x-face (i,j,k) sits at
 *              (i dx, (j+1/2)dx, (k+1/2)dx) and lies between cells i-1 and i.
 * Pressure scaling: with k = dt/(rho dx), the step solves
 *   (G^T S G) P = G^T (S U^ + (I-S) U_s) / k,   W = U^ - k G P,
 *   U^{n+1} = S W + (I - S) U_s
 * where (G p)_f = p(cell on the + side) - p(cell on the - side) and a ghost
 * pressure 0 lies beyond OUTFLOW sides.  W is the fluid velocity of
 * Eq. u_next_matrix; the stored face velocity is the area average of the
 * fluid and solid (or wall / inflow) velocities over the face, so fully fluid
 * faces carry W, closed faces the solid velocity, and G^T U^{n+1} = 0.
 *
 * Memory: every float / double array argument named u_*, p_*, b, x, alpha,
 * g_* is DEVICE memory owned by the caller.  theta and ctrl are HOST double
 * arrays read at call time.  sim_stats (nullable) is a host struct in the
 * default solve mode and device-writable memory (device or pinned host) in
 * the device solve mode (sim_set_solve_mode).
 * Streams: work is enqueued on the caller's hipStream_t (0 = null stream).
 * In the default (host-checked) solve mode, calls that solve a Poisson system
 * wait on that stream for the solver's convergence checks; in the device
 * solve mode no call waits on the host, and a whole step can be captured
 * into a graph.  The final kernels of a call may still be running when it
 * returns (synchronise the stream before reading outputs).
 * Errors: arguments are validated before anything is enqueued; a negative
 * status means nothing was launched.  A positive status (host-checked mode
 * only) means the call ran to its end but a Poisson solve in it did not reach
 * the tolerance (SIM_WNOCONV) or met a NaN / Inf (SIM_WNONFINITE); the
 * outputs are then those of the last iterate.  In the device solve mode these
 * outcomes appear only in sim_stats.  No exception crosses the ABI.
 * Threading: a handle is not thread-safe; use one handle per concurrent
 * episode.  Distinct handles may be used from distinct threads and streams.
 */
#ifndef NEURALFLUID_H
#define NEURALFLUID_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sim_ctx* sim_handle;

typedef enum {
  SIM_OK = 0,
  SIM_EINVAL = -1,        /* invalid argument or descriptor               */
  SIM_ENOMEM = -2,        /* device allocation failed in sim_create       */
  SIM_EHIP = -3,          /* a HIP runtime call failed                    */
  SIM_EUNSUPPORTED = -4,  /* valid request this library does not implement */
  SIM_EBUSY = -5,         /* a pool has no free slot or budget for it now  */
  SIM_WNOCONV = 1,        /* ran; a Poisson solve stopped short of the tolerance */
  SIM_WNONFINITE = 2      /* ran; a Poisson solve met a NaN / Inf            */
} sim_status;

typedef enum { SIM_FP32 = 0, SIM_MIXED_FP16 = 1, SIM_MIXED_BF16 = 2 } sim_precision;

/* Kind of each domain side (order: x-, x+, y-, y+, z-, z+).
 * WALL: closed, no-penetration (alpha = 0, u_s = 0).  INFLOW: alpha = 0 and
 * the normal velocity is inflow_speed into the domain.  OUTFLOW: Dirichlet
 * p = 0 beyond the side (App. B, Eq. bd:dirichlet).  PERIODIC is reserved. */
typedef enum { SIM_BC_WALL = 0, SIM_BC_INFLOW = 1, SIM_BC_OUTFLOW = 2, SIM_BC_PERIODIC = 3 } sim_bc;

/* Solid description (Sec. Projection: the SDF phi and the solid velocity u_s
 * come from the geometry; phi > 0 is fluid).
 *  SIM_GEOM_NONE      : no solid (alpha = 1 except on WALL/INFLOW sides).
 *  SIM_GEOM_SPHERES   : static union of m spheres; theta = m x (cx,cy,cz,r),
 *                       n_params = 4m (m <= SIM_MAX_SPHERES); u_s = 0.
 *  SIM_GEOM_ELLIPSOID : rigid ellipsoid; theta (15) = centre c(3), semi-axes
 *                       a(3), rotation R(9, row-major, body -> world);
 *                       phi = k0 (k0 - 1)/k1 with p = R^T (x - c),
 *                       k0 = |p/a|, k1 = |p/a^2|; ctrl (6) = (v, w),
 *                       u_s(x) = v + w x (x - c).
 *  SIM_GEOM_WALL      : deformable wall on the x- side (the channel
 *                       configuration; a reading of it): displacement
 *                       d(y, z, t) = amp s(t) h(y, z), s = (1 - cos 2 pi f t)/2,
 *                       h = sum_mn a_mn B_m(y) B_n(z) a uniform cubic B-spline
 *                       over the side (knot spacing L/(M - 3), control m
 *                       centred at m - 1 spacings; M = SIM_WALL_KNOTS_Y along
 *                       y, SIM_WALL_KNOTS_Z along z); phi = x - d; the wall
 *                       moves along x: u_s = amp s'(t) h on x faces, 0 on the
 *                       others.  theta (SIM_WALL_KNOTS_Y * SIM_WALL_KNOTS_Z)
 *                       = a, y index major (a[m * SIM_WALL_KNOTS_Z + n]);
 *                       ctrl (3) = (t, f, amp), t the time of the step's
 *                       end.  The adjoint accumulates dJ/da into g_theta;
 *                       t, f and amp get no gradient (g_ctrl is untouched).
 *  SIM_GEOM_BEZIER    : static CSG scene of m parametric solids (Sec.
 *                       Geometry Representation; App. Geometry
 *                       Representation Implementation).  A cross-section is
 *                       SIM_BEZIER_SEGMENTS cubic Bezier segments around a
 *                       centre c; segment s spans the polar angles
 *                       [2 pi s/N, 2 pi (s+1)/N] and its two inner control
 *                       points lie 2 pi/(3N) inside that span at polar
 *                       distances rho[2s], rho[2s+1]; a joint is the midpoint
 *                       of the control points around it.  A solid stacks
 *                       SIM_BEZIER_KEYS key cross-sections evenly on the z
 *                       axis of its frame between z0 and z1, interpolated
 *                       linearly between keys (clamped outside [z0, z1]);
 *                       each segment is taken as its polygon through
 *                       SIM_BEZIER_SAMPLES points (t = k / samples), and the
 *                       solid's signed distance in its frame p = R^T (x - o)
 *                       is max(d(p_x, p_y), z0 - p_z, p_z - z1), d the
 *                       signed distance to the cross-section's polygon
 *                       (negative inside).  phi is the CSG of the solids'
 *                       distances, left to right: min for a union (op 0),
 *                       max for an intersection (op 1).  u_s = 0.
 *                       theta = [m, op_1 .. op_m (op_1 unused), solid_1 ..
 *                       solid_m], each solid SIM_BEZIER_SHAPE_PARAMS values:
 *                       o(3), R(9, row-major, body -> world), z0, z1 (z1 >
 *                       z0), key centres (KEYS x 2), key radii (KEYS x 2N,
 *                       key-major).  n_params = 1 + m (1 +
 *                       SIM_BEZIER_SHAPE_PARAMS), 1 <= m <= SIM_MAX_SOLIDS;
 *                       n_ctrl = 0.  theta[0] must equal m and every op be 0
 *                       or 1 (else SIM_EINVAL).  The adjoint accumulates
 *                       dJ/dtheta into g_theta (zero for m and the ops). */
typedef enum {
  SIM_GEOM_NONE = 0, SIM_GEOM_SPHERES = 1, SIM_GEOM_ELLIPSOID = 2, SIM_GEOM_WALL = 3, SIM_GEOM_BEZIER = 4
} sim_geom;

#define SIM_MAX_SPHERES 32
#define SIM_WALL_KNOTS_Y 16
#define SIM_WALL_KNOTS_Z 32
#define SIM_MAX_SOLIDS 8
#define SIM_BEZIER_SEGMENTS 4
#define SIM_BEZIER_SAMPLES 16
#define SIM_BEZIER_KEYS 3
#define SIM_BEZIER_SHAPE_PARAMS 44

typedef struct {
  int32_t n[3];           /* cells per axis                                   */
  double dx;              /* cell width                                       */
  double dt;              /* time step                                        */
  double rho;             /* density (k = dt/(rho dx))                        */
  double nu;              /* kinematic viscosity (>= 0; explicit, see below)  */
  double gravity[3];      /* body force added to every face: U^ += dt g (this
                             library's addition, for the hydrostatic check)  */
  int32_t bc[6];          /* sim_bc per side                                  */
  double inflow_speed;    /* speed on INFLOW sides                            */
  int32_t precision;      /* sim_precision of the multigrid preconditioner    */
  double tol;             /* relative residual target ||b - A x|| / ||b||     */
  int32_t max_iter;       /* CG iteration cap                                 */
  int32_t geom;           /* sim_geom                                         */
  int32_t n_params;       /* length of theta                                  */
  int32_t n_ctrl;         /* length of ctrl                                   */
} sim_desc;

typedef struct {
  int32_t iters;          /* CG iterations taken                              */
  int32_t converged;      /* 1 if the true residual (FP64) reached tol        */
  int32_t nonfinite;      /* 1 if a NaN/Inf was met in the residual           */
  int32_t pad;
  double rel_res;         /* recursive relative residual (FP64 norm)          */
  double true_rel_res;    /* ||b - A x|| / ||b|| recomputed in FP64 at the end */
} sim_stats;

/* Static description of the library build (for loaders / tests). */
const char* sim_version(void);
const char* sim_status_string(int32_t status);

/* Device bytes sim_create would allocate for desc (host only; no allocation).
 * Used for admission control.  Returns SIM_EINVAL for an invalid desc. */
int32_t sim_footprint(const sim_desc* desc, size_t* bytes);

/* Allocate all workspace for desc on the current HIP device.  Grid sizes must
 * coarsen by halving to a level of at most 4096 cells (e.g. multiples of 16).
 * PERIODIC sides return SIM_EUNSUPPORTED.  Workspace is left
 * unset; with the environment variable NF_POISON_BUFFERS=1 every buffer is
 * filled with all-ones bytes (NaN in every float format) instead, which makes
 * a read of a value no kernel wrote visible (a testing aid). */
int32_t sim_create(const sim_desc* desc, sim_handle* out);
int32_t sim_destroy(sim_handle h);

/* Sizes (in elements) of the velocity and cell arrays of this handle. */
int32_t sim_layout(sim_handle h, size_t* vel_elems, size_t* cell_elems);

/* One step n -> n+1 (Eqs. advection_matrix, viscosity_matrix, projection_matrix,
 * u_next_matrix).
 * u_n, u_n1: velocity (float, distinct).  theta: geometry at time n+1,
 * ctrl: solid velocity controls for this step (host doubles; may be NULL when
 * n_params / n_ctrl are 0).  p_n1: optional cell pressure output (NULL: kept
 * inside the handle).  The solve starts from P = 0. */
int32_t sim_step(sim_handle h, const float* u_n, const double* theta, const double* ctrl,
                 float* u_n1, float* p_n1, sim_stats* st, hipStream_t stream);

/* sim_step with the pressure already known (Eq. u_next_matrix with P given):
 * the geometry and the advection of sim_step, then the update from p_n1, the
 * pressure sim_step returned for the same u_n, theta and ctrl; no Poisson
 * solve.  The result equals sim_step's bitwise.  Back-propagation through a
 * rollout keeps each step's pressure from the first forward pass and
 * recomputes its segments with this call (one solve less per step, at the
 * cost of a cell array per step). */
int32_t sim_step_replay(sim_handle h, const float* u_n, const double* theta, const double* ctrl,
                        const float* p_n1, float* u_n1, hipStream_t stream);

/* Projection only (Eqs. projection_matrix, u_next_matrix) of a given face
 * field u_in (no advection, no body force): u_out = projected field. */
int32_t sim_project(sim_handle h, const float* u_in, const double* theta, const double* ctrl,
                    float* u_out, float* p_out, sim_stats* st, hipStream_t stream);

/* Adjoint of sim_step (Sec. Back-propagation through Time / Geometry).
 * Inputs: u_n (the step's input), p_n1 (the pressure sim_step returned for
 * it, or NULL: the forward system is solved again when shape / control
 * gradients are requested), theta, ctrl (as given to sim_step), and
 * g_u_n1 = dJ/dU^{n+1}.  Output: g_u_n = dJ/dU^n (overwritten; must alias
 * neither g_u_n1 nor u_n).  g_theta (n_params doubles) and g_ctrl (n_ctrl
 * doubles), device, are ACCUMULATED (+=) with this step's direct partials
 * dJ/dtheta and dJ/dctrl (ELLIPSOID: both; WALL, BEZIER: dJ/dtheta only;
 * NULL to skip).  The
 * adjoint pressure system (G^T S G) y = -G^T S g_u_n1 is solved with the same
 * operator (it is symmetric); st reports that solve.  Float atomics make
 * g_u_n reproducible only to rounding. */
int32_t sim_step_adjoint(sim_handle h, const float* u_n, const float* p_n1, const double* theta,
                         const double* ctrl, const float* g_u_n1, float* g_u_n, double* g_theta,
                         double* g_ctrl, sim_stats* st, hipStream_t stream);

/* Solve (G^T S G) x = b (unit scale) by MGPCG to relative residual tol (<= 0:
 * desc.tol) within max_iter (<= 0: desc.max_iter) iterations.  alpha: face
 * fractions (velocity layout) or NULL to reuse the fractions of the last
 * geometry this handle evaluated (sim_step / sim_project / sim_set_geometry).
 * x: initial guess on entry, solution on exit.  On domains without an OUTFLOW
 * side, b must sum to zero over every connected fluid region (compatible);
 * x is then defined up to a constant per region. */
int32_t poisson_solve(sim_handle h, const float* alpha, const float* b, float* x, double tol,
                      int32_t max_iter, sim_stats* st, hipStream_t stream);

/* Evaluate the geometry (phi at nodes, alpha per face) for theta / ctrl and
 * optionally copy alpha out (velocity layout, may be NULL). */
int32_t sim_set_geometry(sim_handle h, const double* theta, const double* ctrl, float* alpha_out,
                         hipStream_t stream);

/* Loss helper (the octant loss of the benchmark scenes): J = sum of u_f^2
 * over faces whose centre lies in the box [lo, hi] (physical coordinates,
 * inclusive), and g = dJ/du = 2 u on those faces, 0 elsewhere.  J: one device
 * double (overwritten, FP64 fixed-order sum); g: device floats (velocity
 * layout, overwritten).  lo / hi: host double[3]. */
int32_t sim_loss_box(sim_handle h, const float* u, const double* lo, const double* hi, double* J, float* g,
                     hipStream_t stream);

/* sim_loss_box without a handle, for callers that cannot allocate device
 * memory or must not (code under graph capture, tight serving loops,
 * harnesses that forbid allocation): it allocates nothing.  The grid is given
 * by n (cells per axis, each 1..4096, at most 2^30 cells) and dx; u, J, g, lo,
 * hi as for sim_loss_box.  Its partial sums live in one fixed device array of
 * 2048 doubles per GPU, owned by the library and held until the process
 * ends; every grid fits it (the kernel strides over the faces).  All calls on
 * one GPU share that array: calls that overlap on one GPU (distinct streams
 * or threads) race and must be serialised by the caller.  SIM_EINVAL for an
 * invalid size or pointer; nothing is enqueued then. */
int32_t sim_loss_box_noalloc(const int32_t n[3], double dx, const float* u, const double* lo, const double* hi,
                             double* J, float* g, hipStream_t stream);

/* Loss helper (the channel configuration's outflow flux): J = scale * sum
 * over the outlet faces (z faces on the z+ side) of w_f u_f, u the stored
 * face-average velocity (Eq. u_next_matrix: alpha W + (1 - alpha) u_s, the
 * flux density through the face), and g = dJ/du = scale * w on those faces,
 * 0 elsewhere.  w: device floats, nx * ny outlet weights (x fastest), or
 * NULL for 1 everywhere.  J: one device double (overwritten, FP64
 * fixed-order sum); g: device floats (velocity layout, overwritten).  The
 * time-integrated flux of a step is scale = dt dx^2. */
int32_t sim_loss_outlet(sim_handle h, const float* u, const float* w, double scale, double* J, float* g,
                        hipStream_t stream);

/* The time step of the handle's later calls (k = dt / (rho dx) follows it):
 * CFL sub-stepping splits a frame into steps of its own length. */
int32_t sim_set_dt(sim_handle h, double dt);

/* Largest |u_f| over the faces of a velocity field (device), written to the
 * host double vmax (a NaN counts as +inf); waits on the stream.  The input of
 * the CFL sub-step count. */
int32_t sim_max_speed(sim_handle h, const float* u, double* vmax, hipStream_t stream);

/* Solve control of a handle (every later Poisson solve of sim_step,
 * sim_project, sim_step_adjoint and poisson_solve).
 *  SIM_SOLVE_HOST (default): CG runs in batches; after each batch the call
 *    waits on the stream for the device-resident convergence state, then
 *    stops, continues, or restarts from the true residual.  Iteration
 *    batches are replayed from a captured graph.  sim_stats is a host struct.
 *  SIM_SOLVE_DEVICE: nothing waits on the host.  Each solve enqueues
 *    min(max_iter, budget) iterations (budget <= 0: max_iter) with an FP64
 *    true-residual check and a conditional restart behind every 8 of them;
 *    once converged, the remaining kernels exit at once on the device.  The
 *    outcome is written by a kernel into sim_stats, which must then be device
 *    memory or pinned host memory (SIM_EINVAL otherwise); the status is
 *    SIM_OK whatever the solve's outcome.  A call enqueued on a capturing
 *    stream is captured whole (wall geometry excepted: its control
 *    amplitudes are copied from pageable host memory). */
typedef enum { SIM_SOLVE_HOST = 0, SIM_SOLVE_DEVICE = 1 } sim_solve_mode;
int32_t sim_set_solve_mode(sim_handle h, int32_t mode, int32_t budget);

/* Warm-started solves (this library's addition; the paper does not say how
 * its solves start).  kinds, a combination of the bits below: with
 * SIM_WARM_PRESSURE the pressure solve of sim_step / sim_project starts from
 * the pressure of the handle's previous such solve, with SIM_WARM_ADJOINT
 * the adjoint pressure solve of sim_step_adjoint from the previous adjoint
 * solution, instead of zero.  The tolerance and the stopping test are
 * unchanged, so results agree with zero-started ones to the solver
 * tolerance, not bitwise.  Consecutive adjoint steps of a rollout have close
 * adjoint pressures (at 128^3 the adjoint solves then take 8.0 instead of 9.0
 * iterations); a step's pressure corrects that step's own advection and is
 * not close to the previous one, so SIM_WARM_PRESSURE saves nothing there.
 * Each call forgets the held pressures: the next solve of each kind starts
 * from zero, which makes a sequence of calls that begins with
 * sim_set_warm_start deterministic.  A forward re-solve inside
 * sim_step_adjoint (p_n1 NULL) starts from zero and ends the forward chain.
 * Host only; enqueues nothing.  Returns SIM_EINVAL for a NULL handle or
 * unknown bits. */
typedef enum { SIM_WARM_PRESSURE = 1, SIM_WARM_ADJOINT = 2 } sim_warm_kind;
int32_t sim_set_warm_start(sim_handle h, int32_t kinds);

/* Connected fluid regions (Sec. Projection: cells joined through faces with
 * alpha > 0).  A region that reaches no OUTFLOW face is floating: its pressure
 * is defined up to a constant and its right-hand side sums to zero over it up
 * to rounding.  With labels, every solve removes each floating region's mean
 * from the residual at its start and at each restart and measures convergence
 * on that projected residual; without them, closed domains remove one global
 * mean over the active cells.  Modes:
 *  SIM_REGIONS_AUTO (default): no labelling up front; a host-checked solve
 *    that stops short of the tolerance without a NaN / Inf labels the
 *    regions of its geometry and solves again (labels are kept until the
 *    geometry is evaluated again).  Device-mode solves never relabel.
 *  SIM_REGIONS_ALWAYS: label at every geometry evaluation.
 *  SIM_REGIONS_NEVER: never label.
 * At most 65536 regions are tracked one by one; beyond that the global mean
 * is used. */
typedef enum { SIM_REGIONS_AUTO = 0, SIM_REGIONS_ALWAYS = 1, SIM_REGIONS_NEVER = 2 } sim_regions_mode;
int32_t sim_set_regions(sim_handle h, int32_t mode);

/* Regions of the handle's current geometry (labelled now if they are not
 * yet).  region_out (device, cells, nullable): compact region id per cell in
 * cell order of each region's first cell, -1 on inactive cells.  count
 * (host): number of regions; floating (host, nullable): number of floating
 * regions, or -1 when there are more regions than tracked.  Waits on the
 * stream.  SIM_EINVAL before any geometry was evaluated. */
int32_t sim_regions(sim_handle h, int32_t* region_out, int32_t* count, int32_t* floating, hipStream_t stream);

/* Kernel timing for measurement: while enabled, the launches of one kernel
 * family are timed on the launch stream (multigrid kernels: finest level
 * only).  Single-kernel launches record their start and stop events from the
 * dispatch itself (the kernel's execution time); composite launches are
 * bracketed by event records.  sim_profile_read synchronises those events and
 * returns the summed duration (ms) and the number of launches timed, counting
 * only launches that took at least min_ms (0: all; a solver kernel enqueued
 * after convergence exits at once and can be left out this way), then clears
 * them.  kernel: one of sim_kernel, or -1 to disable.
 * SIM_K_MG_DOWN: finest-level pre-smoothing + restriction (one fused launch,
 * or the first of two when the fused kernels are disabled); SIM_K_MG_DOWN2:
 * the restriction launch of the unfused form; SIM_K_MG_UP: finest-level
 * correction + post-smoothing (fused) or the last post-smoothing launch
 * (unfused); SIM_K_MG_UP1: the first post-smoothing launch (unfused);
 * SIM_K_MG_COARSE: the one-workgroup bottom solve. */
typedef enum {
  SIM_K_GEOM_PHI = 0, SIM_K_GEOM_ALPHA, SIM_K_ADVECT, SIM_K_RHS, SIM_K_UPDATE, SIM_K_ADJ_DIV,
  SIM_K_ADJ_FACES, SIM_K_ADVECT_ADJ, SIM_K_CG_INIT, SIM_K_CG_APPLY, SIM_K_CG_UPDATE, SIM_K_CG_TRUE,
  SIM_K_MG_DOWN, SIM_K_MG_DOWN2, SIM_K_MG_UP1, SIM_K_MG_UP, SIM_K_MG_COARSE, SIM_K_VISCOSITY, SIM_K_COUNT
} sim_kernel;
int32_t sim_profile(sim_handle h, int32_t kernel);
int32_t sim_profile_read(sim_handle h, double min_ms, double* total_ms, int64_t* count);

/* Rigid ellipsoid pose dynamics (host, FP64).  theta0 (9) = centre c0(3),
 * semi-axes a(3), rotation vector r0(3); R0 = exp([r0]x).  For step n with
 * ctrl[n] = (v, w): c^{n+1} = c^n + dt v, R^{n+1} = exp([dt w]x) R^n.
 * Writes theta_steps[n*15 .. n*15+14] = (c^{n+1}, a, R^{n+1}) for n < T. */
int32_t sim_ellipsoid_poses(const double* theta0, const double* ctrl, int32_t T, double dt,
                            double* theta_steps);

/* Adjoint of sim_ellipsoid_poses: given per-step direct partials
 * g_theta_steps (T x 15) and g_ctrl_direct (T x 6), writes dJ/dtheta0 (9) and
 * the total dJ/dctrl (T x 6). */
int32_t sim_ellipsoid_poses_adjoint(const double* theta0, const double* ctrl, int32_t T, double dt,
                                    const double* g_theta_steps, const double* g_ctrl_direct,
                                    double* g_theta0, double* g_ctrl);

/* ---------------------------------------------------------------------------
 * Serving pool: many episodes at once, as a simulation server runs them.
 * A pool runs many episodes concurrently, each on a library handle and a HIP
 * stream of its own, and interleaves their work unit by unit: sim_pool_tick
 * enqueues the next unit (one step, one replayed step, one adjoint step, the
 * loss, or one projection) of every active episode that may take one, so the
 * episodes' kernels overlap on the device.  At most two units of an episode
 * are in flight at once and, when inflight_cells > 0, the units in flight
 * cover at most that many grid cells in total (one unit may always run): a
 * bound on the concurrent working set.  Admission is by HBM footprint: every
 * handle the pool holds (busy or idle), every live episode's buffer and the
 * released buffers it keeps for reuse count against budget_bytes; an episode
 * reuses a released buffer of up to twice its size and an idle handle of its
 * descriptor, and room is made by freeing kept buffers, then idle handles
 * (least recently used first).  The first episode on a grid runs its
 * solves host-checked (each waits for its convergence state) and sets that
 * grid's iteration budget, half as many again as its most iterations plus
 * two, in whole batches of 8; later episodes run in the device solve mode
 * with that budget (sim_set_solve_mode), their solver reports written on the
 * device.  A device-mode episode whose solve missed the tolerance reports
 * SIM_WNOCONV and doubles its descriptor's budget (up to max_iter); a
 * host-checked episode (the first one, or one admitted with
 * SIM_EP_HOST_CHECKED) raises the budget to its own estimate if that is
 * larger.  Adjoint episodes keep every step's pressure, replay their
 * segments from them, and warm-start their adjoint solves
 * (sim_set_warm_start).  A pool is not thread-safe; it uses the HIP device
 * current at sim_pool_create.
 * ------------------------------------------------------------------------- */
typedef struct sim_pool* sim_pool_handle;

typedef enum {
  SIM_EP_FORWARD = 0,          /* steps forward steps: u_T                                 */
  SIM_EP_FORWARD_ADJOINT = 1,  /* the same, then J = box loss of u_T (sim_loss_box) and the
                                  adjoint: dJ/du_0, per-step dJ/dtheta and dJ/dctrl        */
  SIM_EP_PROJECT = 2           /* one pressure projection of u_0 (sim_project): u_out      */
} sim_episode_kind;

/* sim_episode.flags: run every solve host-checked (each waits for its
 * convergence state), whatever budget the episode's descriptor has learned;
 * for rerunning an episode whose device-mode solve missed the tolerance. */
#define SIM_EP_HOST_CHECKED 1

typedef struct {
  sim_desc desc;          /* grid, geometry and solver settings of the episode        */
  int32_t kind;           /* sim_episode_kind                                         */
  int32_t steps;          /* >= 1 (PROJECT: 1)                                        */
  int32_t every;          /* velocity checkpoint stride of adjoint episodes (>= 1)    */
  int32_t flags;          /* 0 or SIM_EP_HOST_CHECKED                                 */
  const double* theta;    /* host, steps x desc.n_params (copied at admission)        */
  const double* ctrl;     /* host, steps x desc.n_ctrl (copied at admission)          */
  double box_lo[3];       /* loss box of adjoint episodes (sim_loss_box)              */
  double box_hi[3];
} sim_episode;

/* A pool of at most max_active concurrent episodes (1 .. 64) within
 * budget_bytes of device memory.  SIM_EINVAL for bad arguments (checked
 * before any HIP call), SIM_EHIP if a stream cannot be created. */
int32_t sim_pool_create(size_t budget_bytes, int32_t max_active, int64_t inflight_cells, sim_pool_handle* out);
/* Waits for every episode's work, then frees all handles and buffers. */
int32_t sim_pool_destroy(sim_pool_handle pool);
/* Admit an episode; u0 (device, the handle layout's velocity) is copied on
 * the episode's stream, which does not wait for other streams: u0 must be
 * complete when the call is made and unchanged until the slot's result has
 * been collected.  Returns the slot in *slot.  SIM_EBUSY: no free slot,
 * or its footprint does not fit the budget even after freeing idle handles
 * (nothing was done; try again after sim_pool_result has released work).
 * SIM_EINVAL: invalid episode (descriptor, kind, steps, every, flags, NULL
 * arrays that the geometry needs); SIM_ENOMEM / SIM_EHIP: allocation
 * failures. */
int32_t sim_pool_admit(sim_pool_handle pool, const sim_episode* ep, const float* u0, int32_t* slot);
/* Enqueue the next unit of every active episode whose work is not all
 * enqueued yet and which the in-flight bounds allow, starting from a
 * different slot each call; *pending (nullable) = the number of such
 * episodes left.  When no unit could be enqueued and units are in flight,
 * waits for the oldest of them to complete (so a caller's loop does not
 * spin).  Host-checked solves (an episode on a new grid) wait for their
 * stream.  A negative status leaves that episode failed (its result reports
 * it). */
int32_t sim_pool_tick(sim_pool_handle pool, int32_t* pending);
/* *done = 1 once all of the slot's work has completed on the device (an
 * event query, no wait), else 0. */
int32_t sim_pool_poll(sim_pool_handle pool, int32_t slot, int32_t* done);
/* Wait for the slot's work, copy its results out and release the slot (its
 * handle becomes idle).  Every output is nullable.  u_out (device): u_T, or
 * the projected field.  g_u0 (device): dJ/du_0.  g_theta (device doubles,
 * steps x n_params) and g_ctrl (steps x n_ctrl): per-step partials, as
 * sim_step_adjoint accumulates them.  J (host): the loss.  worst (host): the
 * episode's solves summarised: most iterations, converged only if all did,
 * nonfinite if any did, the largest residuals.  Returns the status of the
 * first failed unit, or a warning when a solve missed the tolerance. */
int32_t sim_pool_result(sim_pool_handle pool, int32_t slot, float* u_out, float* g_u0, double* g_theta,
                        double* g_ctrl, double* J, sim_stats* worst);

#ifdef __cplusplus
}
#endif

#endif /* NEURALFLUID_H */
