// Host-side declarations shared by the library's translation units.
#pragma once

#include "nf_internal.h"

#include <hip/hip_ext.h>

#include <vector>

namespace nf {

// Optional timing of one kernel family on the launch stream (multigrid
// kernels: the finest level only).  Single-kernel launches go through
// NF_LAUNCH, which has the dispatch itself record the start and stop events
// (hipExtLaunchKernelGGL: the kernel's own execution time, as a kernel trace
// reports it); composite launches are bracketed by event records (NF_TIMED).
struct Profiler {
  int active = -1;
  std::vector<hipEvent_t> ev;   // pairs: begin, end
  size_t used = 0;
  bool want(int id) const { return active == id; }
  bool reserve() {
    if (used + 2 <= ev.size()) return true;
    if (ev.size() >= 2 * 16384) return false;
    size_t old = ev.size();
    ev.resize(old ? 2 * old : 512);
    for (size_t q = old; q < ev.size(); ++q) (void)hipEventCreate(&ev[q]);
    return true;
  }
  // the next event pair for a launch of kernel family id (false: not timed)
  bool pair(int id, hipEvent_t& a, hipEvent_t& b) {
    if (active != id || !reserve()) return false;
    a = ev[used];
    b = ev[used + 1];
    used += 2;
    return true;
  }
  void begin(int id, hipStream_t s) {
    if (active != id || !reserve()) return;
    (void)hipEventRecord(ev[used], s);
  }
  void end(int id, hipStream_t s) {
    if (active != id || used + 2 > ev.size()) return;
    (void)hipEventRecord(ev[used + 1], s);
    used += 2;
  }
  ~Profiler() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

#define NF_TIMED(prof, id, stream, ...) \
  do {                                   \
    if (prof) (prof)->begin(id, stream); \
    __VA_ARGS__;                         \
    if (prof) (prof)->end(id, stream);   \
  } while (0)

#define NF_LAUNCH(prof, id, kernel, grid, block, shmem, stream, ...)                              \
  do {                                                                                            \
    hipEvent_t nf_e0_, nf_e1_;                                                                    \
    if ((prof) && (prof)->pair(id, nf_e0_, nf_e1_))                                               \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, nf_e0_, nf_e1_, 0, __VA_ARGS__); \
    else                                                                                          \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                       \
  } while (0)

struct Level {
  Dims d;
  void* a[3];   // face fractions (storage type of the level)
  void* invd;   // inverse diagonal
  void* r;      // restricted residual (levels >= 1)
  void* z;      // correction (levels >= 1)
  void* ta;     // smoother temporaries
  void* tb;
};

// Device solve mode: iterations between two true-residual checks (each
// check and its conditional restart costs about a dozen launches, which exit
// at once when they have nothing to do).
constexpr int kDeviceCheckEvery = 8;

// Which domain sides are OUTFLOW (Dirichlet ghost), order x-, x+, y-, y+, z-, z+.
struct Sides {
  int out[6];
};

// Connected fluid regions of the current geometry (nf_components.hip).
struct Components {
  int* parent = nullptr;     // union-find parents; then the reference cell of each cell (-1: none)
  int* id = nullptr;         // compact region id per cell (-1: inactive)
  int* blockcnt = nullptr;   // region roots per block of cells
  int* blockbase = nullptr;  // exclusive scan of blockcnt
  int* info = nullptr;       // [0] region count, [1] 1 if it is at most kMaxComponents
  int* count = nullptr;      // cells per region
  int* ground = nullptr;     // 1 if the region reaches an OUTFLOW face
  long long* sums = nullptr; // fixed-point region sums of r
  double* mean = nullptr;    // region means subtracted from r (0 on grounded regions)
  float* zroot = nullptr;    // z at each region's reference cell
  int mode = SIM_REGIONS_AUTO;
  bool valid = false;        // labels describe the current geometry
};

struct Solver {
  int nlev = 0;
  int nbottom = 0;     // first level run in the one-workgroup bottom solve (at most kBottomCells cells)
  int precision = SIM_FP32;
  int check_every = 2;
  int pcur = 0;        // which of p0 / p1 holds the current direction
  // iterations of the previous solve of each kind (sizes the first batch of
  // iterations): pressure of a step, adjoint pressure, caller's Poisson solve
  int last_iters[3] = {0, 0, 0};
  int trace = 0;       // print each convergence snapshot to stderr (NF_TRACE_SOLVER=1)
  size_t lds_bytes = 65536;  // dynamic LDS the one-workgroup bottom solve may use
  // No Dirichlet side: the operator's null space holds the constants, and the
  // residual's mean over active cells (rounding of a compatible right-hand
  // side) is removed at the start and at every restart.
  int project = 0;
  int fused = 1;       // fused tile kernels per grid level (NF_MG_FUSED=0: four passes per level)
  int bottom_lanes = 1;  // one lane per cell in the bottom solve where it fits (NF_MG_BOTTOM_LANES=0: off)
  void* rec0 = nullptr;  // finest level's packed coefficient records, 2-byte storage (null: the fused kernels read the arrays)
  Level lev[kMaxLevels];
  const float* ax = nullptr;   // fine FP32 fractions (CG operator)
  const float* ay = nullptr;
  const float* az = nullptr;
  double* x = nullptr;         // FP64 iterate
  float* r = nullptr;
  float* z = nullptr;
  float* q = nullptr;
  float* p0 = nullptr;
  float* p1 = nullptr;
  CGScalars* sc = nullptr;
  CGScalars* host_sc = nullptr;  // pinned
  double* partials = nullptr;
  double* partials_rr = nullptr;  // r . r partials of the CG update (kUpdateBlocks)
  double* partials_rz = nullptr;  // r . z partials of the V-cycle when the direction kernel totals them (4 x kRzPartsMax)
  float* scratch_a = nullptr;    // FP32 coarse fractions while building a mixed hierarchy
  float* scratch_inv = nullptr;
  size_t scratch_off[kMaxLevels] = {};
  Profiler* prof = nullptr;
  // CUDA-graph style replay of two CG iterations (captured once per handle on
  // an internal stream, launched on the caller's stream)
  int use_graph = 1;
  // solves that never wait on the host (sim_set_solve_mode): a fixed budget
  // of iterations (at most max_iter) per solve, stats written by a kernel
  int device_mode = 0;
  int budget = 0;
  Sides sides = {};
  Components comp;
  hipStream_t cap_stream = nullptr;
  hipGraph_t iter_graph[2] = {nullptr, nullptr};      // [1]: with the region shift of z
  hipGraphExec_t iter_exec[2] = {nullptr, nullptr};
};

// nf_geom.hip
void launch_phi_nodes(const Domain& D, const GeomParams& G, double* phi, hipStream_t s);
// Parametric solids: check theta (n_params values) and pack it into `host`
// (solids_buffer_doubles() doubles; the caller copies it to the device buffer
// that G.solids then names), with the per-solid adjoint boxes in G.
int pack_solids(const sim_desc& d, const double* theta, double* host, GeomParams& G);
size_t solids_buffer_doubles();
// Partial sums of the solids' parameter gradient (doubles).
size_t solids_partials_doubles();
void launch_alpha(const Domain& D, const double* phi, float* alpha, hipStream_t s);
void launch_invdiag(const Dims& d, const float* ax, const float* ay, const float* az, float* invd, hipStream_t s);
// nf_advect.hip
void launch_fill(float* p, size_t n, float v, hipStream_t s);
void launch_copy(const float* src, float* dst, size_t n, hipStream_t s);
void launch_viscosity(const Dims& d, double c, const float* in, float* out, hipStream_t s);
void launch_max_abs(size_t n, const float* u, unsigned* out_bits, hipStream_t s);
void launch_advect(const Dims& d, double dx, double dt, const double* grav, const float* u, float* out,
                   double* trace, hipStream_t s);
void launch_advect_adjoint(const Dims& d, double dx, double dt, const float* u, const double* trace,
                           const float* gout, float* gin, float* stage, hipStream_t s);
size_t advect_stage_floats(const Dims& d);
// nf_project.hip
void launch_rhs(const Domain& D, const GeomParams& G, double inv_k, const float* alpha, const float* uhat,
                float* b, hipStream_t s);
void launch_update(const Domain& D, const GeomParams& G, double kk, const float* alpha, const float* uhat,
                   const float* p, float* out, hipStream_t s);
void launch_adj_div(const Dims& d, const float* alpha, const float* g, float* rhs, hipStream_t s);
size_t adj_faces_partials(const Dims& d);
void launch_adj_faces(const Domain& D, const GeomParams& G, bool grad, double kk, const float* alpha,
                      const double* phi, const float* g, const float* y, const float* uhat, const float* p,
                      float* gu, double* partials, double* g_theta, double* g_ctrl, double* geom_scratch,
                      hipStream_t s);
size_t wall_column_doubles(const Dims& d);
void launch_loss_outlet(const Dims& d, double scale, const float* w, const float* u, double* J, float* g,
                        double* partials, hipStream_t s);
// blocks (= partial sums) of the box-loss kernel for a grid (at most kLossBlocks)
int loss_box_blocks(const Dims& d);
void launch_loss_box(const Domain& D, const double* lo, const double* hi, const float* u, double* J, float* g,
                     double* partials, hipStream_t s);
// nf_solver.hip
void solver_setup_levels(Solver& S, const float* fine_alpha, hipStream_t st);
enum SolveKind { kSolvePressure = 0, kSolveAdjoint = 1, kSolveUser = 2 };
// zero_guess: the solve starts from x = 0 whatever x holds on entry (x is
// then output only).
int solver_solve(Solver& S, SolveKind kind, const float* b, float* x, double tol, int maxit, sim_stats* stats,
                 hipStream_t st, bool zero_guess = false);
void solver_init_device(Solver& S);
// nf_components.hip
void components_label(Solver& S, hipStream_t st);
void components_project_start(Solver& S, hipStream_t st);
// iter: the per-iteration projection (skipped unless regions are tracked one by one)
void components_subtract(Solver& S, hipStream_t st, int iter = 0);
void components_shift_z(Solver& S, hipStream_t st);
void components_project_iter(Solver& S, int nrr, hipStream_t st);
void solver_release(Solver& S);

}  // namespace nf
