// Matrix-free multigrid-preconditioned CG for (G^T S G) x = b on the MAC grid.
//
// NeuralFluid solves the projection system of Eq. projection_matrix with a
// matrix-free geometric-multigrid-preconditioned CG (Sec. Time Performance
// Profiling: MGPCG with custom prolongation / restriction between a
// hierarchy of grids).  This solver:
//   * applies A x = sum over faces of alpha_f (x_c - x_nb) as a 7-point
//     stencil read straight from the face fractions (no stored matrix), in
//     difference form so that FP32 A p keeps its relative accuracy;
//   * keeps the iterate x in FP64 and the other CG vectors in FP32; every CG
//     scalar stays on the device, with FP64 dot products reduced in a fixed
//     order (per-block partials, then a one-block finishing kernel), so a
//     solve is bitwise reproducible;
//   * stops on the recursive residual, then recomputes b - A x from the FP64
//     iterate; if that true residual misses the tolerance, it replaces the
//     recursive one and CG restarts (iterative refinement, bounded);
//   * on singular systems (no Dirichlet side) removes the residual's mean over
//     active cells at the start and at every restart;
//   * preconditions with one V-cycle: level l+1 halves each axis, coarse face
//     weight = 1/2 * sum of the 2x2 fine faces it covers, restriction = mean
//     of the 8 child residuals with prolongation = 8 x injection, two
//     damped-Jacobi sweeps (omega = 6/7) before and after the correction, and
//     the levels of at most 4096 cells in one workgroup with the coarsest
//     level relaxed by up to 40 sweeps;
//   * uses the flexible (Polak-Ribiere) direction coefficient, since FP16 /
//     BF16 rounding makes the preconditioner slightly non-linear;
//   * stores the multigrid fractions, 1/diag and coarse vectors in FP32, FP16
//     or BF16 (template T); level 0's smoother iterates stay FP32.  The
//     V-cycle is linear, so its input is scaled to a fixed RMS and its output
//     scaled back, which keeps FP16 values in range.
#include "nf_internal.h"
#include "nf_solver.h"
#include "nf_tile.h"

#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cstdio>
#include <type_traits>

namespace nf {

template <typename T> __device__ inline float ld(const T* p, long i);
template <> __device__ inline float ld<float>(const float* p, long i) { return p[i]; }
template <> __device__ inline float ld<__half>(const __half* p, long i) { return __half2float(p[i]); }
template <> __device__ inline float ld<__hip_bfloat16>(const __hip_bfloat16* p, long i) {
  return __bfloat162float(p[i]);
}
template <typename T> __device__ inline T cvt(float v);
template <> __device__ inline float cvt<float>(float v) { return v; }
template <> __device__ inline __half cvt<__half>(float v) { return __float2half(v); }
template <> __device__ inline __hip_bfloat16 cvt<__hip_bfloat16>(float v) { return __float2bfloat16(v); }

__device__ inline void cdec(const Dims& d, long c, int& i, int& j, int& k) { cell_coords(d, c, i, j, k); }

// The 6 face weights of cell (i,j,k): lower / upper along x, y, z.
template <typename A>
struct Faces {
  float w[6];
  __device__ Faces() {}
  __device__ Faces(const Dims& d, const A* ax, const A* ay, const A* az, int i, int j, int k) {
    w[0] = ld(ax, d.fx(i, j, k));
    w[1] = ld(ax, d.fx(i + 1, j, k));
    w[2] = ld(ay, d.fy(i, j, k));
    w[3] = ld(ay, d.fy(i, j + 1, k));
    w[4] = ld(az, d.fz(i, j, k));
    w[5] = ld(az, d.fz(i, j, k + 1));
  }
  __device__ float diag() const { return ((w[0] + w[1]) + (w[2] + w[3])) + (w[4] + w[5]); }
};

// (A x)_c = sum over the 6 faces of alpha_f (x_c - x_nb), x_nb = 0 beyond the
// domain.  The differences are formed before the weighting: for a smooth x the
// subtraction of neighbouring values is exact in FP32, so A x keeps its
// relative accuracy (diag * x_c - sum alpha x_nb would cancel catastrophically).
template <typename A, typename F>
__device__ inline float apply_A(const Dims& d, const Faces<A>& fw, int i, int j, int k, long c, float xc, F val) {
  const long sxy = (long)d.nx * d.ny;
  float s = fw.w[0] * (xc - (i > 0 ? val(c - 1) : 0.0f));
  s += fw.w[1] * (xc - (i < d.nx - 1 ? val(c + 1) : 0.0f));
  s += fw.w[2] * (xc - (j > 0 ? val(c - d.nx) : 0.0f));
  s += fw.w[3] * (xc - (j < d.ny - 1 ? val(c + d.nx) : 0.0f));
  s += fw.w[4] * (xc - (k > 0 ? val(c - sxy) : 0.0f));
  s += fw.w[5] * (xc - (k < d.nz - 1 ? val(c + sxy) : 0.0f));
  return s;
}

// b_c - (A x)_c accumulated in FP64 from the FP64 iterate (0 on inactive cells).
__device__ inline double true_residual_at(const Dims& d, const float* ax, const float* ay, const float* az,
                                          const float* b, const double* x, int i, int j, int k, long c) {
  Faces<float> fw(d, ax, ay, az, i, j, k);
  if (!(fw.diag() > 0.0f)) return 0.0;
  const long sxy = (long)d.nx * d.ny;
  const double xc = x[c];
  double s = (double)fw.w[0] * (xc - (i > 0 ? x[c - 1] : 0.0));
  s += (double)fw.w[1] * (xc - (i < d.nx - 1 ? x[c + 1] : 0.0));
  s += (double)fw.w[2] * (xc - (j > 0 ? x[c - d.nx] : 0.0));
  s += (double)fw.w[3] * (xc - (j < d.ny - 1 ? x[c + d.nx] : 0.0));
  s += (double)fw.w[4] * (xc - (k > 0 ? x[c - sxy] : 0.0));
  s += (double)fw.w[5] * (xc - (k < d.nz - 1 ? x[c + sxy] : 0.0));
  return (double)b[c] - s;
}

__device__ inline double vscale_of(double rr, long n) { return vscale_of_rr(rr, n); }

// ---------------------------------------------------------------------------
// CG kernels (fine level: FP64 iterate, FP32 vectors).  Each reducing kernel
// writes per-block partials; a one-block k_fin_* kernel turns them into the
// device-resident scalars after the kernel boundary.
// ---------------------------------------------------------------------------

__global__ void k_x_load(long n, const float* __restrict__ xin, double* __restrict__ x) {
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) x[c] = (double)xin[c];
}

// Output of a solve: the iterate on active cells, 0 on inactive (fully solid)
// cells, which carry no unknown (the preconditioner's prolongation may leave
// values there that are never coupled to anything).
__global__ void k_x_store(Dims d, const float* __restrict__ ax, const float* __restrict__ ay,
                          const float* __restrict__ az, const double* __restrict__ x, float* __restrict__ xout) {
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)d.cells()) return;
  int i, j, k;
  cdec(d, c, i, j, k);
  Faces<float> fw(d, ax, ay, az, i, j, k);
  xout[c] = fw.diag() > 0.0f ? (float)x[c] : 0.0f;
}

// r = b - A x; partials of b.b (active cells), r.r, sum of r and the number
// of active cells.
// A bounded grid-stride grid keeps the partials few (k_fin_init totals them
// in one block).
constexpr int kInitBlocks = 1024;
__global__ __launch_bounds__(kBlock) void k_cg_init(Dims d, const float* __restrict__ ax,
                                                     const float* __restrict__ ay,
                                                     const float* __restrict__ az,
                                                     const float* __restrict__ b,
                                                     const double* __restrict__ x, float* __restrict__ r,
                                                     double* partials) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const long n = (long)d.cells();
  for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long)gridDim.x * blockDim.x) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<float> fw(d, ax, ay, az, i, j, k);
    const bool act = fw.diag() > 0.0f;
    double bc = act ? (double)b[c] : 0.0;
    double rc = true_residual_at(d, ax, ay, az, b, x, i, j, k, c);
    r[c] = (float)rc;
    v[0] += bc * bc;
    v[1] += rc * rc;
    v[2] += rc;
    v[3] += act ? 1.0 : 0.0;
  }
  block_partials<4>(v, partials);
}

// The same for a zero initial guess: r = b on active cells (1/diag > 0) and
// x = 0, without the stencil.
__global__ __launch_bounds__(kBlock) void k_cg_init_zero(long n, const float* __restrict__ invd,
                                                          const float* __restrict__ b, double* __restrict__ x,
                                                          float* __restrict__ r, double* partials) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long)gridDim.x * blockDim.x) {
    const bool act = invd[c] > 0.0f;
    const double bc = act ? (double)b[c] : 0.0;
    x[c] = 0.0;
    r[c] = (float)bc;
    v[0] += bc * bc;
    v[1] += bc * bc;
    v[2] += bc;
    v[3] += act ? 1.0 : 0.0;
  }
  block_partials<4>(v, partials);
}

// ||r - mean||^2 over active cells from r.r, sum(r) and the active count
// (or r.r when the system has a Dirichlet side).
__device__ inline double projected_rr(double rr, double sr, double na, int project) {
  if (!project || !(na > 0.0)) return rr;
  double v = rr - sr * sr / na;
  return v > 0.0 ? v : 0.0;
}

__global__ __launch_bounds__(kFinBlock) void k_fin_init(int nb, const double* partials, CGScalars* sc, double tol,
                                                         int maxit, long ncells, int project) {
  double tot[4];
  finish_partials<4>(partials, nb, tot);
  if (threadIdx.x == 0) {
    const double rr = projected_rr(tot[1], tot[2], tot[3], project);
    sc->mu = project && tot[3] > 0.0 ? tot[2] / tot[3] : 0.0;
    sc->nact = tot[3];
    sc->rr_raw = tot[1];
    sc->null_rr = 0.0;
    sc->use_comp = 0;
    sc->zmu = 0.0;
    tot[1] = rr;
    sc->bb = tot[0];
    sc->rr = tot[1];
    sc->true_rr = tot[1];
    sc->tol2bb = tol * tol * tot[0];
    sc->iters = 0;
    sc->checks = 0;
    sc->restarts = 0;
    sc->restarted = 0;
    sc->final_ = 0;
    sc->first = 1;
    sc->maxit = maxit;
    sc->nonfinite = !isfinite(tot[1]);
    sc->converged = (tot[0] == 0.0) || (tot[1] <= sc->tol2bb);
    sc->done = sc->converged || sc->nonfinite || maxit <= 0;
    sc->rho = 0.0;
    sc->rho2[0] = sc->rho2[1] = 0.0;
    sc->zmu2[0] = sc->zmu2[1] = 0.0;
    sc->beta = 0.0;
    sc->alpha = 0.0;
    sc->vscale = vscale_of(tot[1], ncells);
  }
}

// p_new = z + beta p_old (p_new = z on the first iteration); q = A p_new;
// partials of p_new . q.
__global__ __launch_bounds__(kBlock) void k_cg_dir_apply(Dims d, const float* __restrict__ ax,
                                                          const float* __restrict__ ay,
                                                          const float* __restrict__ az,
                                                          const float* __restrict__ z,
                                                          const float* __restrict__ pold,
                                                          float* __restrict__ pnew, float* __restrict__ q,
                                                          const CGScalars* sc, double* partials) {
  if (sc->done) return;
  const bool first = sc->first;
  const float beta = (float)sc->beta;
  // z minus its mean over active cells (0 unless the system is singular): the
  // V-cycle maps the constants to a large multiple of themselves, and a
  // rounding-level constant left in r would otherwise grow in p (k_fin_rz
  // forms the dots of the same projected z).  Values on inactive cells never
  // couple (all their faces are closed).
  const float zmu = (float)sc->zmu;
  long c = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  double v[1] = {0.0};
  if (c < (long)d.cells()) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<float> fw(d, ax, ay, az, i, j, k);
    auto pv = [&](long t) { return first ? z[t] - zmu : (z[t] - zmu) + beta * pold[t]; };
    float pc = pv(c);
    float qc = apply_A(d, fw, i, j, k, c, pc, pv);
    pnew[c] = pc;
    q[c] = qc;
    v[0] = (double)pc * qc;
  }
  block_partials<1>(v, partials);
}

// x += alpha p (FP64); r -= alpha q; partials of r . r (grid-stride, at most
// kUpdateBlocks blocks).  alpha = rho / (p . q) is formed by every block from
// the direction kernel's p . q partials (fixed order, so all blocks agree);
// block 0 records it, ends the first iteration and advances the count.  No
// block reads what block 0 writes.
__global__ __launch_bounds__(kBlock) void k_cg_update(long n, double* __restrict__ x, float* __restrict__ r,
                                                       const float* __restrict__ p,
                                                       const float* __restrict__ q, CGScalars* sc,
                                                       const double* pq_parts, int npq, double* rr_parts) {
  if (sc->done) return;
  __shared__ double tot_sh, alpha_sh;
  // the partials are read first, then the first cell's operands, so that
  // totalling the partials waits only for them
  constexpr int K = 4;
  double pv[K];
  const bool in_regs = npq <= K * kBlock;
  if (in_regs) partials_load<K, kBlock>(pq_parts, npq, pv);
  const long c0 = (long)blockIdx.x * blockDim.x + threadIdx.x, stride = (long)gridDim.x * blockDim.x;
  double x0 = 0.0;
  float p0 = 0.0f, r0 = 0.0f, q0 = 0.0f;
  if (c0 < n) {
    x0 = x[c0];
    p0 = p[c0];
    r0 = r[c0];
    q0 = q[c0];
  }
  double pq;
  if (in_regs) {
    pq = partials_reduce<K, kBlock>(pv, &tot_sh);
  } else {
    double tot[1];
    block_total<1, kBlock>(pq_parts, npq, tot);
    if (threadIdx.x == 0) tot_sh = tot[0];
    __syncthreads();
    pq = tot_sh;
  }
  if (threadIdx.x == 0) {
    const double a = pq != 0.0 ? sc->rho / pq : 0.0;
    alpha_sh = a;
    if (blockIdx.x == 0) {
      sc->alpha = a;
      sc->first = 0;
      sc->iters += 1;
    }
  }
  __syncthreads();
  const double a = alpha_sh;
  const float af = (float)a;
  double v[1] = {0.0};
  if (c0 < n) {
    x[c0] = x0 + a * (double)p0;
    const float rc = r0 - af * q0;
    r[c0] = rc;
    v[0] += (double)rc * rc;
  }
  for (long c = c0 + stride; c < n; c += stride) {
    x[c] += a * (double)p[c];
    const float rc = r[c] - af * q[c];
    r[c] = rc;
    v[0] += (double)rc * rc;
  }
  block_partials<1>(v, rr_parts);
}

// State after an update from rr = r . r: the V-cycle input scale and the stop
// test (converged, iteration cap, or a non-finite residual, which is sticky).
// The finest-level down kernel forms this state in every block while its
// block 0 stores it; a block that reads `done` or `nonfinite` after block 0
// stored them reads the values it computes itself.
struct RRState {
  double rr, vscale;
  int nonfinite, done;
};
__device__ inline RRState rr_state(const CGScalars* sc, double rr, long ncells) {
  RRState st;
  st.rr = rr;
  st.vscale = vscale_of(rr, ncells);
  st.nonfinite = (sc->nonfinite || !isfinite(rr)) ? 1 : 0;
  st.done = (rr <= sc->tol2bb || sc->iters >= sc->maxit || st.nonfinite) ? 1 : 0;
  return st;
}
__device__ inline void put_rr_state(CGScalars* sc, const RRState& st) {
  sc->rr = st.rr;
  sc->vscale = st.vscale;
  sc->nonfinite = st.nonfinite;
  sc->done = st.done;
}

// One-block form of the same, ahead of a V-cycle whose first kernel does not
// total the r . r partials itself.
__global__ __launch_bounds__(kFinBlock) void k_fin_rr(int nb, const double* partials, CGScalars* sc, long ncells) {
  if (sc->done) return;
  double tot[1];
  finish_partials<1>(partials, nb, tot);
  if (threadIdx.x == 0) put_rr_state(sc, rr_state(sc, tot[0], ncells));
}

// True residual from the FP64 iterate, once the recursive residual has
// converged (both kernels do nothing while CG is still iterating, so the check
// can be enqueued behind every batch of iterations).  With `allow`, a residual
// that misses the tolerance replaces r and CG restarts (k_fin_true sets
// done = 0, first = 1).
__device__ inline bool may_replace(const CGScalars* sc, int allow) {
  return allow && sc->restarts < kMaxRestarts && !sc->nonfinite && sc->iters < sc->maxit && !(sc->bb == 0.0);
}

__global__ __launch_bounds__(kBlock) void k_cg_true_residual(Dims d, const float* __restrict__ ax,
                                                              const float* __restrict__ ay,
                                                              const float* __restrict__ az,
                                                              const float* __restrict__ b,
                                                              const double* __restrict__ x, float* __restrict__ r,
                                                              int allow, const CGScalars* sc, double* partials) {
  if (!sc->done || sc->final_) return;
  const bool rep = may_replace(sc, allow);
  double v[3] = {0.0, 0.0, 0.0};
  // a bounded grid-stride grid (k_fin_true totals the partials in one block)
  for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < (long)d.cells(); c += (long)gridDim.x * blockDim.x) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<float> fw(d, ax, ay, az, i, j, k);
    double rc = true_residual_at(d, ax, ay, az, b, x, i, j, k, c);
    v[0] += rc * rc;
    v[1] += rc;
    v[2] += fw.diag() > 0.0f ? 1.0 : 0.0;
    if (rep) r[c] = (float)rc;
  }
  block_partials<3>(v, partials);
}

__global__ __launch_bounds__(kFinBlock) void k_fin_true(int nb, const double* partials, CGScalars* sc, int allow,
                                                         long ncells, int project) {
  if (!sc->done || sc->final_) return;
  const bool rep = may_replace(sc, allow);
  double tot[3];
  finish_partials<3>(partials, nb, tot);
  if (threadIdx.x == 0) {
    sc->checks += 1;
    // region by region (labels), or one global mean on closed domains
    if (sc->use_comp) {
      tot[0] = tot[0] - sc->null_rr > 0.0 ? tot[0] - sc->null_rr : 0.0;
      sc->mu = 0.0;
    } else {
      tot[0] = projected_rr(tot[0], tot[1], tot[2], project);
      sc->mu = project && tot[2] > 0.0 ? tot[1] / tot[2] : 0.0;
    }
    sc->true_rr = tot[0];
    if (!isfinite(tot[0])) sc->nonfinite = 1;
    sc->converged = !sc->nonfinite && (sc->bb == 0.0 || tot[0] <= sc->tol2bb);
    if (rep && !sc->converged && !sc->nonfinite) {
      sc->rr = tot[0];
      sc->vscale = vscale_of(tot[0], ncells);
      sc->first = 1;
      sc->done = 0;
      sc->restarts += 1;
      sc->restarted = 1;
    } else {
      sc->final_ = 1;
    }
  }
}

// Device-only solves enqueue a restart V-cycle behind every true-residual
// check; it must run only when that check restarted CG.  While CG is still
// iterating, k_hold_restart parks `done` at 2 (every solver kernel skips on a
// nonzero `done`) and k_release_restart puts it back afterwards.
__global__ void k_hold_restart(CGScalars* sc) {
  if (sc->done == 0 && !sc->restarted) sc->done = 2;
}
__global__ void k_release_restart(CGScalars* sc) {
  if (sc->done == 2) sc->done = 0;
  sc->restarted = 0;
}

// The solve's outcome into caller memory that the device can write (device
// memory or pinned host memory).
__global__ void k_write_stats(const CGScalars* sc, sim_stats* out) {
  out->iters = sc->iters;
  out->nonfinite = sc->nonfinite;
  out->converged = sc->converged && !sc->nonfinite;
  out->pad = 0;
  out->rel_res = sc->bb > 0.0 ? sqrt(sc->rr / sc->bb) : 0.0;
  out->true_rel_res = sc->bb > 0.0 ? sqrt(sc->true_rr / sc->bb) : 0.0;
}

// r -= mean on active cells (singular systems, after k_fin_init / a restart).
__global__ __launch_bounds__(kBlock) void k_sub_mean(Dims d, const float* __restrict__ ax,
                                                      const float* __restrict__ ay, const float* __restrict__ az,
                                                      float* __restrict__ r, const CGScalars* sc) {
  if (sc->done) return;
  const double mu = sc->mu;
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)d.cells()) return;
  int i, j, k;
  cdec(d, c, i, j, k);
  Faces<float> fw(d, ax, ay, az, i, j, k);
  if (fw.diag() > 0.0f) r[c] = (float)((double)r[c] - mu);
}

// k_sub_mean and k_x_store telling active cells by an FP32 1/diag (> 0)
// instead of their six face fractions.
__global__ __launch_bounds__(kBlock) void k_sub_mean_inv(long n, const float* __restrict__ invd,
                                                          float* __restrict__ r, const CGScalars* sc) {
  if (sc->done) return;
  const double mu = sc->mu;
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n && invd[c] > 0.0f) r[c] = (float)((double)r[c] - mu);
}

__global__ void k_x_store_inv(long n, const float* __restrict__ invd, const double* __restrict__ x,
                              float* __restrict__ xout) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) xout[c] = invd[c] > 0.0f ? (float)x[c] : 0.0f;
}

// rho = r . z and the flexible (Polak-Ribiere) direction coefficient
// beta = r_new . (z_new - z_old) / rho_old: the rounding of the FP16 / BF16
// V-cycle makes the preconditioner slightly non-linear, which this form
// tolerates; for an exactly linear preconditioner r_new . z_old = 0 and it
// reduces to the Fletcher-Reeves ratio.  On singular systems z is used minus
// its mean over active cells (k_cg_dir_apply subtracts zmu), and the dots are
// those of the projected vectors: r . (z - mu) = r . z - mu sum(r).
// Partials: r.z_new, r.z_old, sum(z_new), sum(r).
// The same from the totals, as state for one iteration: the previous
// iteration's rho and zmu come from the slot of the other iteration parity
// (sc->iters does not change between the V-cycle and the CG update), so a
// kernel whose block 0 stores this iteration's values may have other blocks
// reading the previous ones.
struct RZState {
  double rho, beta, mu;
  int slot;
};
__device__ inline RZState rz_state(const CGScalars* sc, const double (&tot)[4], int project) {
  RZState z;
  z.slot = sc->iters & 1;
  const int o = z.slot ^ 1;
  // with region labels z is shifted region by region instead
  z.mu = project && !sc->use_comp && sc->nact > 0.0 ? tot[2] / sc->nact : 0.0;
  z.rho = tot[0] - z.mu * tot[3];
  z.beta = 0.0;
  if (!sc->first) {
    const double rzo = tot[1] - sc->zmu2[o] * tot[3];
    z.beta = sc->rho2[o] != 0.0 ? (z.rho - rzo) / sc->rho2[o] : 0.0;
  }
  return z;
}
__device__ inline void put_rz_state(CGScalars* sc, const RZState& z) {
  sc->rho2[z.slot] = z.rho;
  sc->zmu2[z.slot] = z.mu;
  sc->rho = z.rho;
  sc->zmu = z.mu;
  if (!sc->first) sc->beta = z.beta;
}

__global__ __launch_bounds__(kFinBlock) void k_fin_rz(int nb, const double* partials, CGScalars* sc, int project) {
  if (sc->done) return;
  double tot[4];
  finish_partials<4>(partials, nb, tot);
  if (threadIdx.x == 0) put_rz_state(sc, rz_state(sc, tot, project));
}

// z *= 1 / vscale (the V-cycle ran on the scaled residual), 0 on inactive
// cells; partials of r . z, r . z_old (always 0 here: the whole V-cycle ran in
// one workgroup and overwrote z), sum(z) and sum(r).
template <typename A>
__global__ __launch_bounds__(kBlock) void k_scale_dot(long n, const A* __restrict__ invd, const float* __restrict__ r,
                                                       float* __restrict__ z, const CGScalars* sc, double* partials) {
  if (sc->done) return;
  const float inv = (float)(1.0 / sc->vscale);
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (c < n) {
    float zc = ld(invd, c) > 0.0f ? z[c] * inv : 0.0f;
    z[c] = zc;
    v[0] = (double)r[c] * (double)zc;
    v[2] = zc;
    v[3] = r[c];
  }
  block_partials<4>(v, partials);
}

// ---------------------------------------------------------------------------
// multigrid kernels on the grid levels.  A: storage of fractions / 1/diag;
// R: residual input; Z: correction storage.  At level 0 the residual is the
// FP32 CG residual, multiplied by sc->vscale on load (`s0`).
// ---------------------------------------------------------------------------

__device__ inline float level_scale(const CGScalars* sc, int lvl0) { return lvl0 ? (float)sc->vscale : 1.0f; }

// Two damped-Jacobi sweeps from z = 0:  z1 = w D^-1 r,  z2 = z1 + w D^-1 (r - A z1).
template <typename A, typename R, typename Z>
__global__ __launch_bounds__(kBlock) void k_mg_pre(Dims d, const A* __restrict__ ax, const A* __restrict__ ay,
                                                    const A* __restrict__ az, const A* __restrict__ invd,
                                                    const R* __restrict__ r, Z* __restrict__ z2,
                                                    const CGScalars* sc, int lvl0) {
  if (sc->done) return;
  const float s0 = level_scale(sc, lvl0);
  long c = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (c >= (long)d.cells()) return;
  int i, j, k;
  cdec(d, c, i, j, k);
  Faces<A> fw(d, ax, ay, az, i, j, k);
  float idc = ld(invd, c);
  auto z1 = [&](long t) { return kOmega1 * ld(invd, t) * (s0 * ld(r, t)); };
  float rc = s0 * ld(r, c);
  float z1c = kOmega1 * idc * rc;
  float Az = apply_A(d, fw, i, j, k, c, z1c, z1);
  z2[c] = cvt<Z>(z1c + kOmega2 * idc * (rc - Az));
}

// r_coarse(I,J,K) = mean over the 8 children of (r - A z).
template <typename A, typename R, typename Z, typename RC>
__global__ __launch_bounds__(kBlock) void k_mg_restrict(Dims d, Dims cd, const A* __restrict__ ax,
                                                         const A* __restrict__ ay, const A* __restrict__ az,
                                                         const R* __restrict__ r, const Z* __restrict__ z,
                                                         RC* __restrict__ rc, const CGScalars* sc, int lvl0) {
  if (sc->done) return;
  const float s0 = level_scale(sc, lvl0);
  long C = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (C >= (long)cd.cells()) return;
  int I, J, K;
  cdec(cd, C, I, J, K);
  float s = 0.0f;
  auto zv = [&](long t) { return ld(z, t); };
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    int i = 2 * I + (b & 1), j = 2 * J + ((b >> 1) & 1), k = 2 * K + (b >> 2);
    long c = d.c(i, j, k);
    Faces<A> fw(d, ax, ay, az, i, j, k);
    float Az = apply_A(d, fw, i, j, k, c, ld(z, c), zv);
    s += s0 * ld(r, c) - Az;
  }
  rc[C] = cvt<RC>(0.125f * s);
}

// z' = z_in + 8 e(parent); z_out = z' + w D^-1 (r - A z').
template <typename A, typename R, typename Z, typename E>
__global__ __launch_bounds__(kBlock) void k_mg_post1(Dims d, Dims cd, const A* __restrict__ ax,
                                                      const A* __restrict__ ay, const A* __restrict__ az,
                                                      const A* __restrict__ invd, const R* __restrict__ r,
                                                      const Z* __restrict__ zin, const E* __restrict__ e,
                                                      Z* __restrict__ zout, const CGScalars* sc, int lvl0) {
  if (sc->done) return;
  const float s0 = level_scale(sc, lvl0);
  long c = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (c >= (long)d.cells()) return;
  int i, j, k;
  cdec(d, c, i, j, k);
  Faces<A> fw(d, ax, ay, az, i, j, k);
  // z' at the cell and its 6 neighbours; the parent of a neighbour differs
  // from the cell's parent only across an even-odd boundary
  const int cnx = cd.nx, cny = cd.ny;
  const long pc = (i >> 1) + (long)cnx * ((j >> 1) + (long)cny * (k >> 1));
  const long psx = 1, psy = cnx, psz = (long)cnx * cny;
  const float ec = ld(e, pc);
  const float zc = ld(zin, c) + 8.0f * ec;
  const long sxy = (long)d.nx * d.ny;
  auto nb = [&](bool ok, long q, bool same, long pq) {
    return ok ? ld(zin, q) + 8.0f * (same ? ec : ld(e, pq)) : 0.0f;
  };
  float Az = fw.w[0] * (zc - nb(i > 0, c - 1, (i & 1), pc - psx));
  Az += fw.w[1] * (zc - nb(i < d.nx - 1, c + 1, !(i & 1), pc + psx));
  Az += fw.w[2] * (zc - nb(j > 0, c - d.nx, (j & 1), pc - psy));
  Az += fw.w[3] * (zc - nb(j < d.ny - 1, c + d.nx, !(j & 1), pc + psy));
  Az += fw.w[4] * (zc - nb(k > 0, c - sxy, (k & 1), pc - psz));
  Az += fw.w[5] * (zc - nb(k < d.nz - 1, c + sxy, !(k & 1), pc + psz));
  zout[c] = cvt<Z>(zc + kOmega1 * ld(invd, c) * (s0 * ld(r, c) - Az));
}

// z_out = z_in + w D^-1 (r - A z_in); at level 0 the output is scaled back to
// the CG residual's units and partials of r . z are written.
template <typename A, typename R, typename Z, typename O, bool LVL0>
__global__ __launch_bounds__(kBlock) void k_mg_post2(Dims d, const A* __restrict__ ax, const A* __restrict__ ay,
                                                      const A* __restrict__ az, const A* __restrict__ invd,
                                                      const R* __restrict__ r, const Z* __restrict__ zin,
                                                      O* __restrict__ zout, const CGScalars* sc, double* partials) {
  if (sc->done) return;
  const float s0 = LVL0 ? (float)sc->vscale : 1.0f;
  const float inv = LVL0 ? (float)(1.0 / sc->vscale) : 1.0f;
  const bool first = sc->first;
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (c < (long)d.cells()) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<A> fw(d, ax, ay, az, i, j, k);
    auto zv = [&](long t) { return ld(zin, t); };
    float zc = ld(zin, c);
    float rraw = ld(r, c);
    float Az = apply_A(d, fw, i, j, k, c, zc, zv);
    const float idc = ld(invd, c);
    float zo = (zc + kOmega2 * idc * (s0 * rraw - Az)) * inv;
    if (LVL0 && !(idc > 0.0f)) zo = 0.0f;   // inactive cell: no unknown
    if (LVL0 && !first) v[1] = (double)rraw * (double)ld(zout, c);   // r_new . z_old
    zout[c] = cvt<O>(zo);
    v[0] = (double)rraw * (double)zo;
    v[2] = zo;
    v[3] = rraw;
  }
  if (LVL0) block_partials<4>(v, partials);
}

// ---------------------------------------------------------------------------
// Fused grid-level kernels.  One workgroup owns a TX x TY x TZ tile of a
// level and recomputes what its neighbours own on a halo instead of waiting
// for them, so the four smoother / transfer passes of a level become two
// launches and each array is read from memory once per launch:
//   down: z1 = w D^-1 r on the tile + 2 cells, z2 = z1 + w D^-1 (r - A z1)
//         on the tile + 1 cell (stored for the way up), and the restricted
//         residual mean(r - A z2) of the tile's coarse cells;
//   up:   z' = z2 + 8 e(parent) on the tile + 2 cells, z3 = z' + w D^-1 (r - A z')
//         on the tile + 1 cell, z4 = z3 + w D^-1 (r - A z3) on the tile.
// Values beyond the domain are 0, as in apply_A.  Tile shapes, region walks
// and the buffer addressing are described in nf_tile.h.
// ---------------------------------------------------------------------------

template <class S>
__host__ __device__ inline int tiles_of(const Dims& d) {
  return tiles_x<S>(d.nx) * tiles_y<S>(d.ny) * tiles_z<S>(d.nz);
}

template <class S>
__device__ inline void tile_origin(const Dims& d, int& i0, int& j0, int& k0) {
  tile_origin_of<S>(xcd_block(blockIdx.x, gridDim.x), d.nx, d.ny, i0, j0, k0);
}

// sum over the 6 faces of w_f (v[q] - v[nb]) for a cell at local index q of a
// region with row length X and plane size XY (neighbours beyond the domain
// hold 0 in v, the Dirichlet / closed convention of apply_A)
template <typename A>
__device__ inline float apply_local(const Faces<A>& fw, const float* v, int q, int X, int XY) {
  const float c = v[q];
  float s = fw.w[0] * (c - v[q - 1]);
  s += fw.w[1] * (c - v[q + 1]);
  s += fw.w[2] * (c - v[q - X]);
  s += fw.w[3] * (c - v[q + X]);
  s += fw.w[4] * (c - v[q - XY]);
  s += fw.w[5] * (c - v[q + XY]);
  return s;
}

using Rsrc = __amdgpu_buffer_rsrc_t;


// Buffer view of an array whose base is the element (i, j, k) of a grid with
// the given row / plane lengths (elements); the base may precede the array,
// only the elements a kernel addresses must exist.
template <typename T>
__device__ inline Rsrc view(const T* p, int row, int plane, int i, int j, int k) {
  const long e = (long)i + (long)row * j + (long)plane * k;
  const uintptr_t a = (uintptr_t)p + (uintptr_t)(e * (long)sizeof(T));
  return __builtin_amdgcn_make_buffer_rsrc((void*)a, (short)0, kViewRecords, 0x00020000);
}

template <typename T> __device__ inline float vld(Rsrc r, unsigned v, unsigned s);
template <> __device__ inline float vld<float>(Rsrc r, unsigned v, unsigned s) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)v, (int)s, 0));
}
template <> __device__ inline float vld<__half>(Rsrc r, unsigned v, unsigned s) {
  return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, (int)v, (int)s, 0)));
}
template <> __device__ inline float vld<__hip_bfloat16>(Rsrc r, unsigned v, unsigned s) {
  return __bfloat162float(
      __builtin_bit_cast(__hip_bfloat16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)v, (int)s, 0)));
}
template <typename T> __device__ inline void vst(Rsrc r, unsigned v, unsigned s, float x);
template <> __device__ inline void vst<float>(Rsrc r, unsigned v, unsigned s, float x) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, (int)v, (int)s, 0);
}
template <> __device__ inline void vst<__half>(Rsrc r, unsigned v, unsigned s, float x) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2half(x)), r, (int)v, (int)s, 0);
}
template <> __device__ inline void vst<__hip_bfloat16>(Rsrc r, unsigned v, unsigned s, float x) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2bfloat16(x)), r, (int)v, (int)s,
                                        0);
}

// v rounded to the storage type T (what a later read of a stored v returns)
template <typename T>
__device__ inline float rnd(float v) {
  const T x = cvt<T>(v);
  return ld(&x, 0);
}

// Byte offset of one access: lane part v and a part s uniform over the wave.
// When the plane index varies across the wave (U false) the plane part joins
// the lane part.
struct At {
  unsigned v, s;
};
template <bool U>
__device__ inline At at(unsigned lane, unsigned plane) {
  return U ? At{lane, plane} : At{lane + plane, 0u};
}

// Extents and plane lengths (elements) of one level's arrays.
struct Lev {
  int nx, ny, nz;
  int pc;   // cells (and z faces) per plane
  int px;   // x faces per plane
  int py;   // y faces per plane
};
__device__ inline Lev level_of(const Dims& d) {
  Lev L;
  L.nx = d.nx;
  L.ny = d.ny;
  L.nz = d.nz;
  L.pc = d.nx * d.ny;
  L.px = (d.nx + 1) * d.ny;
  L.py = d.nx * (d.ny + 1);
  return L;
}

// Plane group of lane t in the +H walk (uniform over the wave where the walk
// allows it, so plane offsets stay scalar).
template <class S, int H>
__device__ inline int walk_group(int t) {
  using W = Walk<S, H>;
  if constexpr (W::P == 1) return 0;
  else if constexpr (W::kUniform) return uniform_value(t / W::PL);
  else return t / W::PL;
}

// A lane's byte offset for trip u: kNoCell when the trip's plane lies outside
// the domain (ZIN: the tile's whole +2 region is inside).
template <bool ZIN>
__device__ inline unsigned on_plane(unsigned lane, unsigned mask, int u) {
  return (ZIN || ((mask >> u) & 1u)) ? lane : kNoCell;
}

// Face views of a level at a tile (base: corner of the +2 region).
struct FaceViews {
  Rsrc ax, ay, az;
};
template <typename A>
__device__ inline FaceViews face_views(const A* ax, const A* ay, const A* az, const Lev& L, int i0, int j0, int k0) {
  return {view(ax, L.nx + 1, L.px, i0 - 2, j0 - 2, k0 - 2), view(ay, L.nx, L.py, i0 - 2, j0 - 2, k0 - 2),
          view(az, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2)};
}

// The 6 face weights of a cell in plane kr of the +2 frame, for lane offsets
// fe (x-face frame) and ce (cell frame), in bytes: x faces at fx, fx + 1;
// y faces at fy, fy + nx; z faces at fz, fz + nx ny.
template <typename A, bool U>
__device__ inline Faces<A> faces_at(const FaceViews& V, unsigned fe, unsigned ce, int kr, const Lev& L) {
  constexpr unsigned es = sizeof(A);
  const At x = at<U>(fe, (unsigned)(kr * L.px) * es);
  const At y = at<U>(ce, (unsigned)(kr * L.py) * es);
  const At z = at<U>(ce, (unsigned)(kr * L.pc) * es);
  Faces<A> f;
  f.w[0] = vld<A>(V.ax, x.v, x.s);
  f.w[1] = vld<A>(V.ax, x.v + es, x.s);
  f.w[2] = vld<A>(V.ay, y.v, y.s);
  f.w[3] = vld<A>(V.ay, y.v, y.s + (unsigned)L.nx * es);
  f.w[4] = vld<A>(V.az, z.v, z.s);
  f.w[5] = vld<A>(V.az, z.v, z.s + (unsigned)L.pc * es);
  return f;
}

// Packed coefficients of one finest-level cell with 2-byte multigrid storage
// (16 bytes, one wide load instead of seven narrow ones): the six face weights
// beta_f = alpha_f / diag in the storage type (Faces order) and 1/diag in
// FP32.  The weights lie in [0, 1] whatever the fractions, and 1/diag keeps
// its full range: the separate 2-byte arrays cap 1/diag at the largest finite
// FP16 value and hold fractions below its smallest normal with few bits, which
// a cut cell nearly inside the solid needs (diag < 1/65504 occurs every step
// of a moving body).  A sweep then reads z + w (r/diag - sum beta_f (z - z_f)).
// Built by k_pack_records from the FP32 fractions, with 1/diag also as a plain
// FP32 array right after the records (for reads of 1/diag alone, which would
// otherwise touch a whole record per value).  (FP32 storage keeps the arrays:
// its 32-byte records cost the finest kernels more in bytes than they saved
// in load instructions.)
struct alignas(16) Rec16 {
  unsigned w[4];
};
template <typename A> struct RecOf { using T = Rec16; };
template <typename A> constexpr bool kHasRecords = sizeof(A) == 2;

// Minimum waves per SIMD of a tile kernel.  A 512-lane tile puts 2 waves on
// each SIMD, so 7 waves per SIMD (65-72 VGPRs) hold 3 tiles per CU and 8
// (at most 64 VGPRs) hold 4: the 1024 finest-level tiles of a 128^3 grid then
// all fit the 256 CUs at once.  Asked only where the kernel fits 64 VGPRs
// without spilling (the FP16 finest level: k_mg_up 21.1 -> 20.7 us at 128^3);
// elsewhere the compiler's own choice stands.
template <class S, typename A>
constexpr int kTileWaves = (std::is_same<S, FineTile>::value && std::is_same<A, __half>::value) ? 8 : 1;

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <typename A> __device__ inline float dec_lo(unsigned w);
template <typename A> __device__ inline float dec_hi(unsigned w);
template <> __device__ inline float dec_lo<__half>(unsigned w) {
  return __half2float(__builtin_bit_cast(__half, (unsigned short)(w & 0xffffu)));
}
template <> __device__ inline float dec_hi<__half>(unsigned w) {
  return __half2float(__builtin_bit_cast(__half, (unsigned short)(w >> 16)));
}
template <> __device__ inline float dec_lo<__hip_bfloat16>(unsigned w) {
  return __bfloat162float(__builtin_bit_cast(__hip_bfloat16, (unsigned short)(w & 0xffffu)));
}
template <> __device__ inline float dec_hi<__hip_bfloat16>(unsigned w) {
  return __bfloat162float(__builtin_bit_cast(__hip_bfloat16, (unsigned short)(w >> 16)));
}

// Storage bits to float.  The word is taken by value: a bit cast applied
// directly to an element of a vector value compiles (with this toolchain) to a
// read of the vector's first element, whatever the element named.
__device__ inline float f32_of(unsigned w) { return __builtin_bit_cast(float, w); }

// The record of the cell in plane kr (lane offset ce in bytes): its face
// weights beta_f and 1/diag (all 0 for inactive cells and lanes outside the
// domain).
template <typename A, bool U>
__device__ inline Faces<A> rec_faces(Rsrc v, unsigned ce, int kr, const Lev& L, float& id) {
  using RT = typename RecOf<A>::T;
  const At a = at<U>(ce, (unsigned)(kr * L.pc) * (unsigned)sizeof(RT));
  Faces<A> f;
  const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(v, (int)a.v, (int)a.s, 0);
  f.w[0] = dec_lo<A>(q.x);
  f.w[1] = dec_hi<A>(q.x);
  f.w[2] = dec_lo<A>(q.y);
  f.w[3] = dec_hi<A>(q.y);
  f.w[4] = dec_lo<A>(q.z);
  f.w[5] = dec_hi<A>(q.z);
  id = f32_of(q.w);
  return f;
}

// The FP32 1/diag array that follows the records of a level of `cells` cells.
__device__ inline const float* rec_invd_array(const void* rec, long cells) {
  return (const float*)((const Rec16*)rec + cells);
}

template <typename A> __device__ inline unsigned bits_of(A v);
template <> __device__ inline unsigned bits_of<__half>(__half v) {
  return __builtin_bit_cast(unsigned short, v);
}
template <> __device__ inline unsigned bits_of<__hip_bfloat16>(__hip_bfloat16 v) {
  return __builtin_bit_cast(unsigned short, v);
}

// One record per cell of the finest level from its FP32 face fractions (1/diag
// as k_invdiag forms it).
template <typename A>
__global__ void k_pack_records(Dims d, const float* __restrict__ ax, const float* __restrict__ ay,
                               const float* __restrict__ az, typename RecOf<A>::T* __restrict__ rec,
                               float* __restrict__ invd) {
  static_assert(kHasRecords<A>, "packed records hold 2-byte storage");
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)d.cells()) return;
  int i, j, k;
  cdec(d, c, i, j, k);
  const float a[6] = {ax[d.fx(i, j, k)], ax[d.fx(i + 1, j, k)], ay[d.fy(i, j, k)],
                      ay[d.fy(i, j + 1, k)], az[d.fz(i, j, k)], az[d.fz(i, j, k + 1)]};
  const float s = a[0] + a[1] + a[2] + a[3] + a[4] + a[5];
  const float id = s > 0.0f ? 1.0f / s : 0.0f;
  unsigned b[6];
  for (int f = 0; f < 6; ++f) b[f] = bits_of<A>(cvt<A>(a[f] * id));
  typename RecOf<A>::T r;
  for (int q = 0; q < 3; ++q) r.w[q] = b[2 * q] | (b[2 * q + 1] << 16);
  r.w[3] = __builtin_bit_cast(unsigned, id);
  rec[c] = r;
  invd[c] = id;
}

// A cell-frame value of type T in plane kr (lane offset ce in bytes).
template <typename T, bool U>
__device__ inline float cell_at(Rsrc v, unsigned ce, int kr, const Lev& L) {
  const At a = at<U>(ce, (unsigned)(kr * L.pc) * (unsigned)sizeof(T));
  return vld<T>(v, a.v, a.s);
}
template <typename T, bool U>
__device__ inline void cell_put(Rsrc v, unsigned ce, int kr, const Lev& L, float x) {
  const At a = at<U>(ce, (unsigned)(kr * L.pc) * (unsigned)sizeof(T));
  vst<T>(v, a.v, a.s, x);
}

// Body of k_mg_down for one tile; ZIN: the tile's +2 region lies inside the
// domain along z (no plane checks).  PRE = 1: issue the loads of all three
// phases before the first one computes (one memory latency per launch instead
// of three; for the small coarse levels, whose launches are latency-bound and
// few tiles wide); PRE = 2: those of the first two phases.  With PRE = 0 each
// phase loads what it needs, which keeps registers low for the finest level
// (at 128^3 the finest k_mg_up took 20.7 us with PRE = 0 and 8 waves per SIMD,
// 21.5 us with PRE = 2 and 22.7 us with PRE = 1 at the occupancy their
// registers allow).
template <class S, typename A, typename R, typename Z, typename RC, int PRE, bool ZIN, bool REC>
__device__ __forceinline__ void mg_down_tile(const Dims& d, const Dims& cd, const A* ax, const A* ay, const A* az,
                                             const A* invd, const R* r, Z* z2out, RC* rc, CGScalars* sc, int lvl0,
                                             const double* rr_parts, int nrr, long ncells, int i0, int j0, int k0,
                                             float* z1s, float* z2s, double* rr_sh, const void* rec) {
  using W2 = Walk<S, 2>;
  using W1 = Walk<S, 1>;
  using W0 = Walk<S, 0>;
  constexpr int eA = sizeof(A), eR = sizeof(R), eZ = sizeof(Z);
  const Lev L = level_of(d);
  const int t = threadIdx.x;
  const FaceViews V = face_views(ax, ay, az, L, i0, j0, k0);
  const Rsrc vid = view(invd, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  const Rsrc vr = view(r, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  // packed coefficient records (REC): one view over the cell frame
  static_assert(!REC || kHasRecords<A>, "packed records hold 2-byte storage");
  using RecT = typename RecOf<A>::T;
  constexpr int kRB = (int)sizeof(RecT);
  const Rsrc VR = view((const RecT*)rec, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  const Rsrc VI = view(REC ? rec_invd_array(rec, (long)d.cells()) : (const float*)nullptr, L.nx, L.pc, i0 - 2,
                       j0 - 2, k0 - 2);
  const Rsrc vz = view(z2out, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  const Lane l2 = lane_of<S, 2>(t, walk_group<S, 2>(t), i0, j0, L.nx, L.ny);
  const Lane l1 = lane_of<S, 1>(t, walk_group<S, 1>(t), i0, j0, L.nx, L.ny);
  const Lane l0 = lane_of<S, 0>(t, walk_group<S, 0>(t), i0, j0, L.nx, L.ny);
  const unsigned m2 = ZIN ? ~0u : plane_mask(k0, l2.z, L.nz, W2::T);
  const unsigned m1 = ZIN ? ~0u : plane_mask(k0, l1.z, L.nz, W1::T);
  const unsigned m0 = ZIN ? ~0u : plane_mask(k0, l0.z, L.nz, W0::T);
  float id1[W2::T], rv1[W2::T], id2[W1::T], rv2[W1::T], id3[W0::T], rv3[W0::T];
  Faces<A> fw2[W1::T], fw3[W0::T];
  // the update's r . r partials are read before this kernel's own loads, so
  // that totalling them waits only for them
  constexpr int KR = (kUpdateBlocks + kTileThreads - 1) / kTileThreads;
  double prr[KR];
  if (nrr > 0) partials_load<KR, kTileThreads>(rr_parts, nrr, prr);
  auto load2 = [&]() {
    const unsigned fe = lane_bytes(l1.in, l1.fe, eA), ce = lane_bytes(l1.in, l1.ce, eA),
                   cr = lane_bytes(l1.in, l1.ce, eR);
#pragma unroll
    for (int u = 0; u < W1::T; ++u) {
      const int kr = l1.z + u;
      if constexpr (REC) {
        fw2[u] = rec_faces<A, W1::kUniform>(VR, on_plane<ZIN>(lane_bytes(l1.in, l1.ce, kRB), m1, u), kr, L, id2[u]);
      } else {
        fw2[u] = faces_at<A, W1::kUniform>(V, on_plane<ZIN>(fe, m1, u), on_plane<ZIN>(ce, m1, u), kr, L);
        id2[u] = cell_at<A, W1::kUniform>(vid, on_plane<ZIN>(ce, m1, u), kr, L);
      }
      rv2[u] = cell_at<R, W1::kUniform>(vr, on_plane<ZIN>(cr, m1, u), kr, L);
    }
  };
  auto load3 = [&]() {
    const unsigned fe = lane_bytes(l0.in, l0.fe, eA), ce = lane_bytes(l0.in, l0.ce, eA),
                   cr = lane_bytes(l0.in, l0.ce, eR);
#pragma unroll
    for (int u = 0; u < W0::T; ++u) {
      if constexpr (REC) {
        fw3[u] = rec_faces<A, W0::kUniform>(VR, on_plane<ZIN>(lane_bytes(l0.in, l0.ce, kRB), m0, u), l0.z + u, L, id3[u]);
      } else {
        fw3[u] = faces_at<A, W0::kUniform>(V, on_plane<ZIN>(fe, m0, u), on_plane<ZIN>(ce, m0, u), l0.z + u, L);
        id3[u] = 0.0f;
      }
      rv3[u] = cell_at<R, W0::kUniform>(vr, on_plane<ZIN>(cr, m0, u), l0.z + u, L);
    }
  };
  {
    const unsigned ce = lane_bytes(l2.in, l2.ce, eA), cr = lane_bytes(l2.in, l2.ce, eR);
#pragma unroll
    for (int u = 0; u < W2::T; ++u) {
      if constexpr (REC)
        id1[u] = cell_at<float, W2::kUniform>(VI, on_plane<ZIN>(lane_bytes(l2.in, l2.ce, 4), m2, u), l2.z + u, L);
      else
        id1[u] = cell_at<A, W2::kUniform>(vid, on_plane<ZIN>(ce, m2, u), l2.z + u, L);
      rv1[u] = cell_at<R, W2::kUniform>(vr, on_plane<ZIN>(cr, m2, u), l2.z + u, L);
    }
  }
  if (PRE != 0) load2();
  if (PRE == 1) load3();
  // with every load issued up front (the coarse levels) the solver's state is
  // read beside them rather than before them; a launch after convergence
  // still exits before it stores anything (the empty asm keeps the compiler
  // from moving the loads below the check)
  if (PRE == 1) {
    asm volatile("" ::: "memory");
    if (sc->done) return;
  }
  float s0;
  if (nrr > 0) {
    // right after the CG update (the loads above are already in flight):
    // every block totals the update's r . r partials (the same bits in each),
    // applies the stop test and scales by the new RMS; block 0 stores the
    // state for the kernels that follow
    const RRState st = rr_state(sc, partials_reduce<KR, kTileThreads>(prr, rr_sh), ncells);
    if (blockIdx.x == 0 && threadIdx.x == 0) put_rr_state(sc, st);
    if (st.done) return;
    s0 = (float)st.vscale;
  } else {
    s0 = level_scale(sc, lvl0);
  }
  if (l2.on) {
#pragma unroll
    for (int u = 0; u < W2::T; ++u) z1s[l2.q + u * W2::PL] = kOmega1 * id1[u] * (s0 * rv1[u]);
  }
  __syncthreads();
  if (PRE == 0) load2();
  if (l1.on) {
    // the tile's own cells of the +1 walk are stored for the way up
    const bool own_xy = l1.x >= 2 && l1.x < S::TX + 2 && l1.y >= 2 && l1.y < S::TY + 2;
    const unsigned oz = own_xy ? lane_bytes(l1.in, l1.ce, eZ) : kNoCell;
    const int q2 = l1.x + W2::X * l1.y + W2::PL * l1.z;
#pragma unroll
    for (int u = 0; u < W1::T; ++u) {
      const int z = l1.z + u;
      const int qq = q2 + u * W2::PL;
      const float rr = s0 * rv2[u];
      const float z2 =
          REC ? rnd<Z>(z1s[qq] + kOmega2 * (id2[u] * rr - apply_local(fw2[u], z1s, qq, W2::X, W2::PL)))
              : rnd<Z>(z1s[qq] + kOmega2 * id2[u] * (rr - apply_local(fw2[u], z1s, qq, W2::X, W2::PL)));
      cell_put<Z, W1::kUniform>(vz, (z >= 2 && z < S::TZ + 2) ? on_plane<ZIN>(oz, m1, u) : kNoCell, z, L, z2);
      z2s[l1.q + u * W1::PL] = z2;
    }
  }
  __syncthreads();
  if (PRE != 1) load3();
  if (l0.on) {
    // residual r - A z2 of the tile's cells (into the first sweep's array)
    const int q1 = (l0.x - 1) + W1::X * (l0.y - 1) + W1::PL * (l0.z - 1);
#pragma unroll
    for (int u = 0; u < W0::T; ++u) {
      const int qq = q1 + u * W1::PL;
      const float Az = apply_local(fw3[u], z2s, qq, W1::X, W1::PL);
      // records: A z2 = diag * (the weighted sum); an inactive cell has none
      z1s[l0.q + u * W0::PL] = s0 * rv3[u] - (REC ? (id3[u] > 0.0f ? Az / id3[u] : 0.0f) : Az);
    }
  }
  __syncthreads();
  // restriction: the tile's (TX/2) x (TY/2) x (TZ/2) coarse cells, one per
  // thread, each the mean of its 8 children (all inside the level: levels
  // are coarsened only while every extent is even)
  constexpr int CX = S::TX / 2, CY = S::TY / 2, CZ = S::TZ / 2;
  if (t < CX * CY * CZ) {
    const int ci = t % CX, cj = (t / CX) % CY, ck = t / (CX * CY);
    const int I = i0 / 2 + ci, J = j0 / 2 + cj, K = k0 / 2 + ck;
    if (I < cd.nx && J < cd.ny && K < cd.nz) {
      float s = 0.0f;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int li = 2 * ci + (b & 1), lj = 2 * cj + ((b >> 1) & 1), lk = 2 * ck + (b >> 2);
        s += z1s[li + S::TX * (lj + S::TY * lk)];
      }
      rc[cd.c(I, J, K)] = cvt<RC>(0.125f * s);
    }
  }
}

// REC (finest level): the coefficients come from the packed records `rec`.
template <class S, typename A, typename R, typename Z, typename RC, int PRE, bool REC = false>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(kTileWaves<S, A>))) void k_mg_down(Dims d, Dims cd, const A* __restrict__ ax,
                                                          const A* __restrict__ ay, const A* __restrict__ az,
                                                          const A* __restrict__ invd, const R* __restrict__ r,
                                                          Z* __restrict__ z2out, RC* __restrict__ rc,
                                                          CGScalars* sc, int lvl0, const double* rr_parts, int nrr,
                                                          long ncells, const void* rec = nullptr) {
  static_assert(Walk<S, 0>::N <= Walk<S, 2>::N, "the tile residual reuses the first sweep's array");
  __shared__ float z1s[Walk<S, 2>::N];   // first sweep on the +2 region; then the tile's residual
  __shared__ float z2s[Walk<S, 1>::N];
  __shared__ double rr_sh;
  if (PRE != 1 && sc->done) return;   // PRE == 1: checked after the loads
  int i0, j0, k0;
  tile_origin<S>(d, i0, j0, k0);
  if (planes_inside<S>(k0, d.nz))
    mg_down_tile<S, A, R, Z, RC, PRE, true, REC>(d, cd, ax, ay, az, invd, r, z2out, rc, sc, lvl0, rr_parts, nrr,
                                                 ncells, i0, j0, k0, z1s, z2s, &rr_sh, rec);
  else
    mg_down_tile<S, A, R, Z, RC, PRE, false, REC>(d, cd, ax, ay, az, invd, r, z2out, rc, sc, lvl0, rr_parts, nrr,
                                                  ncells, i0, j0, k0, z1s, z2s, &rr_sh, rec);
}

// Body of k_mg_up for one tile (ZIN, PRE as for mg_down_tile).
template <class S, typename A, typename R, typename Z, typename E, typename O, bool LVL0, int PRE, bool ZIN, bool REC>
__device__ __forceinline__ void mg_up_tile(const Dims& d, const Dims& cd, const A* ax, const A* ay, const A* az,
                                           const A* invd, const R* r, const Z* z2, const E* e, O* zout, float s0,
                                           float inv, bool first, int i0, int j0, int k0, float* zp, float* z3s,
                                           double (&acc)[4], const void* rec, const CGScalars* sc) {
  using W2 = Walk<S, 2>;
  using W1 = Walk<S, 1>;
  using W0 = Walk<S, 0>;
  constexpr int eA = sizeof(A), eR = sizeof(R), eZ = sizeof(Z), eE = sizeof(E), eO = sizeof(O);
  const Lev L = level_of(d);
  const int t = threadIdx.x;
  const FaceViews V = face_views(ax, ay, az, L, i0, j0, k0);
  const Rsrc vid = view(invd, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  const Rsrc vr = view(r, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  // packed coefficient records (REC): one view over the cell frame
  static_assert(!REC || kHasRecords<A>, "packed records hold 2-byte storage");
  constexpr int kRB = (int)sizeof(Rec16);
  const Rsrc VR = view((const Rec16*)rec, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  const Rsrc vz2 = view(z2, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  const Rsrc vzo = view(zout, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  const int cpc = cd.nx * cd.ny;
  // parent view base: the parent of the +2 corner (tile origins are even)
  const Rsrc ve = view(e, cd.nx, cpc, (i0 - 2) / 2, (j0 - 2) / 2, (k0 - 2) / 2);
  const Lane l2 = lane_of<S, 2>(t, walk_group<S, 2>(t), i0, j0, L.nx, L.ny);
  const Lane l1 = lane_of<S, 1>(t, walk_group<S, 1>(t), i0, j0, L.nx, L.ny);
  const Lane l0 = lane_of<S, 0>(t, walk_group<S, 0>(t), i0, j0, L.nx, L.ny);
  const unsigned m2 = ZIN ? ~0u : plane_mask(k0, l2.z, L.nz, W2::T);
  const unsigned m1 = ZIN ? ~0u : plane_mask(k0, l1.z, L.nz, W1::T);
  const unsigned m0 = ZIN ? ~0u : plane_mask(k0, l0.z, L.nz, W0::T);
  float zv[W2::T], ev[W2::T], id2[W1::T], rv2[W1::T], id3[W0::T], rv3[W0::T], zold[W0::T];
  Faces<A> fw2[W1::T], fw3[W0::T];
  auto load2 = [&]() {
    const unsigned fe = lane_bytes(l1.in, l1.fe, eA), ce = lane_bytes(l1.in, l1.ce, eA),
                   cr = lane_bytes(l1.in, l1.ce, eR);
#pragma unroll
    for (int u = 0; u < W1::T; ++u) {
      const int kr = l1.z + u;
      if constexpr (REC) {
        fw2[u] = rec_faces<A, W1::kUniform>(VR, on_plane<ZIN>(lane_bytes(l1.in, l1.ce, kRB), m1, u), kr, L, id2[u]);
      } else {
        fw2[u] = faces_at<A, W1::kUniform>(V, on_plane<ZIN>(fe, m1, u), on_plane<ZIN>(ce, m1, u), kr, L);
        id2[u] = cell_at<A, W1::kUniform>(vid, on_plane<ZIN>(ce, m1, u), kr, L);
      }
      rv2[u] = cell_at<R, W1::kUniform>(vr, on_plane<ZIN>(cr, m1, u), kr, L);
    }
  };
  auto load3 = [&]() {
    const unsigned fe = lane_bytes(l0.in, l0.fe, eA), ce = lane_bytes(l0.in, l0.ce, eA),
                   cr = lane_bytes(l0.in, l0.ce, eR), co = lane_bytes(l0.in, l0.ce, eO);
#pragma unroll
    for (int u = 0; u < W0::T; ++u) {
      const int kr = l0.z + u;
      if constexpr (REC) {
        fw3[u] = rec_faces<A, W0::kUniform>(VR, on_plane<ZIN>(lane_bytes(l0.in, l0.ce, kRB), m0, u), kr, L, id3[u]);
      } else {
        fw3[u] = faces_at<A, W0::kUniform>(V, on_plane<ZIN>(fe, m0, u), on_plane<ZIN>(ce, m0, u), kr, L);
        id3[u] = cell_at<A, W0::kUniform>(vid, on_plane<ZIN>(ce, m0, u), kr, L);
      }
      rv3[u] = cell_at<R, W0::kUniform>(vr, on_plane<ZIN>(cr, m0, u), kr, L);
      zold[u] = (LVL0 && !first) ? cell_at<O, W0::kUniform>(vzo, on_plane<ZIN>(co, m0, u), kr, L) : 0.0f;
    }
  };
  {
    const unsigned cz = lane_bytes(l2.in, l2.ce, eZ);
    // the lane's parent column in the parent view's frame
    const unsigned le = lane_bytes(l2.in, (l2.x >> 1) + cd.nx * (l2.y >> 1), eE);
#pragma unroll
    for (int u = 0; u < W2::T; ++u) {
      const int kr = l2.z + u;
      zv[u] = cell_at<Z, W2::kUniform>(vz2, on_plane<ZIN>(cz, m2, u), kr, L);
      const At a = at<W2::kUniform>(on_plane<ZIN>(le, m2, u), (unsigned)((kr >> 1) * cpc) * (unsigned)eE);
      ev[u] = vld<E>(ve, a.v, a.s);
    }
  }
  if (PRE != 0) load2();
  if (PRE == 1) load3();
  if (PRE == 1) {   // as in mg_down_tile
    asm volatile("" ::: "memory");
    if (sc->done) return;
  }
  if (l2.on) {
#pragma unroll
    for (int u = 0; u < W2::T; ++u) zp[l2.q + u * W2::PL] = zv[u] + 8.0f * ev[u];
  }
  __syncthreads();
  if (PRE == 0) load2();
  if (l1.on) {
    const int q2 = l1.x + W2::X * l1.y + W2::PL * l1.z;
#pragma unroll
    for (int u = 0; u < W1::T; ++u) {
      const int qq = q2 + u * W2::PL;
      const float Az = apply_local(fw2[u], zp, qq, W2::X, W2::PL);
      z3s[l1.q + u * W1::PL] =
          REC ? zp[qq] + kOmega1 * (id2[u] * (s0 * rv2[u]) - Az) : zp[qq] + kOmega1 * id2[u] * (s0 * rv2[u] - Az);
    }
  }
  __syncthreads();
  if (PRE != 1) load3();
  if (l0.on) {
    const int q1 = (l0.x - 1) + W1::X * (l0.y - 1) + W1::PL * (l0.z - 1);
    const unsigned co = lane_bytes(l0.in, l0.ce, eO);
#pragma unroll
    for (int u = 0; u < W0::T; ++u) {
      const int qq = q1 + u * W1::PL;
      const float Az = apply_local(fw3[u], z3s, qq, W1::X, W1::PL);
      float zo = (REC ? z3s[qq] + kOmega2 * (id3[u] * (s0 * rv3[u]) - Az)
                      : z3s[qq] + kOmega2 * id3[u] * (s0 * rv3[u] - Az)) * inv;
      if (LVL0 && !(id3[u] > 0.0f)) zo = 0.0f;   // inactive cell (and every cell outside the domain): no unknown
      cell_put<O, W0::kUniform>(vzo, on_plane<ZIN>(co, m0, u), l0.z + u, L, zo);
      if (LVL0) {
        if (!first) acc[1] += (double)rv3[u] * (double)zold[u];   // r_new . z_old
        acc[0] += (double)rv3[u] * (double)zo;
        acc[2] += (double)zo;
        acc[3] += (double)rv3[u];
      }
    }
  }
}

// REC (finest level): the coefficients come from the packed records `rec`.
template <class S, typename A, typename R, typename Z, typename E, typename O, bool LVL0, int PRE, bool REC = false>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(kTileWaves<S, A>))) void k_mg_up(Dims d, Dims cd, const A* __restrict__ ax,
                                                        const A* __restrict__ ay, const A* __restrict__ az,
                                                        const A* __restrict__ invd, const R* __restrict__ r,
                                                        const Z* __restrict__ z2, const E* __restrict__ e,
                                                        O* __restrict__ zout, const CGScalars* sc, double* partials,
                                                        const void* rec = nullptr) {
  __shared__ float zp[Walk<S, 2>::N];
  __shared__ float z3s[Walk<S, 1>::N];
  if (PRE != 1 && sc->done) return;   // PRE == 1: checked after the loads
  const float s0 = LVL0 ? (float)sc->vscale : 1.0f;
  const float inv = LVL0 ? (float)(1.0 / sc->vscale) : 1.0f;
  const bool first = sc->first;
  int i0, j0, k0;
  tile_origin<S>(d, i0, j0, k0);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (planes_inside<S>(k0, d.nz))
    mg_up_tile<S, A, R, Z, E, O, LVL0, PRE, true, REC>(d, cd, ax, ay, az, invd, r, z2, e, zout, s0, inv, first, i0, j0,
                                                       k0, zp, z3s, acc, rec, sc);
  else
    mg_up_tile<S, A, R, Z, E, O, LVL0, PRE, false, REC>(d, cd, ax, ay, az, invd, r, z2, e, zout, s0, inv, first, i0,
                                                        j0, k0, zp, z3s, acc, rec, sc);
  if (LVL0) block_partials<4, kTileThreads>(acc, partials);
}

// CG direction and operator on a tile: p = (z - zmu) + beta p_old on the tile
// + 1 cell (in LDS; written out on the tile), q = A p and p.q partials on the
// tile.  Same arithmetic as k_cg_dir_apply with one load of z and p_old per
// cell and halo.
template <class S, bool ZIN>
__device__ __forceinline__ void cg_dir_apply_tile(const Dims& d, const float* ax, const float* ay, const float* az,
                                                  const float* z, const float* pold, float* pnew, float* q,
                                                  bool first, float beta, float zmu, int i0, int j0, int k0,
                                                  float* ps, double (&acc)[1]) {
  using W1 = Walk<S, 1>;
  using W0 = Walk<S, 0>;
  const Lev L = level_of(d);
  const int t = threadIdx.x;
  const FaceViews V = face_views(ax, ay, az, L, i0, j0, k0);
  const Rsrc vz = view(z, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  const Rsrc vpo = view(pold, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  const Rsrc vpn = view(pnew, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  const Rsrc vq = view(q, L.nx, L.pc, i0 - 2, j0 - 2, k0 - 2);
  const Lane l1 = lane_of<S, 1>(t, walk_group<S, 1>(t), i0, j0, L.nx, L.ny);
  const Lane l0 = lane_of<S, 0>(t, walk_group<S, 0>(t), i0, j0, L.nx, L.ny);
  const unsigned m1 = ZIN ? ~0u : plane_mask(k0, l1.z, L.nz, W1::T);
  const unsigned m0 = ZIN ? ~0u : plane_mask(k0, l0.z, L.nz, W0::T);
  {
    const unsigned ce = lane_bytes(l1.in, l1.ce, 4);
    float zv[W1::T], pv[W1::T];
#pragma unroll
    for (int u = 0; u < W1::T; ++u) {
      zv[u] = cell_at<float, W1::kUniform>(vz, on_plane<ZIN>(ce, m1, u), l1.z + u, L);
      pv[u] = first ? 0.0f : cell_at<float, W1::kUniform>(vpo, on_plane<ZIN>(ce, m1, u), l1.z + u, L);
    }
    if (l1.on) {
      const bool own_xy = l1.x >= 2 && l1.x < S::TX + 2 && l1.y >= 2 && l1.y < S::TY + 2;
      const unsigned op = own_xy ? ce : kNoCell;
#pragma unroll
      for (int u = 0; u < W1::T; ++u) {
        const int zz = l1.z + u;
        const bool in = l1.in && (ZIN || ((m1 >> u) & 1u));
        // cells outside the domain hold 0 (z - zmu would not)
        const float pn = in ? (first ? zv[u] - zmu : (zv[u] - zmu) + beta * pv[u]) : 0.0f;
        cell_put<float, W1::kUniform>(vpn, (zz >= 2 && zz < S::TZ + 2) ? on_plane<ZIN>(op, m1, u) : kNoCell, zz, L,
                                      pn);
        ps[l1.q + u * W1::PL] = pn;
      }
    }
  }
  __syncthreads();
  Faces<float> fw[W0::T];
  const unsigned fe = lane_bytes(l0.in, l0.fe, 4), ce = lane_bytes(l0.in, l0.ce, 4);
#pragma unroll
  for (int u = 0; u < W0::T; ++u)
    fw[u] = faces_at<float, W0::kUniform>(V, on_plane<ZIN>(fe, m0, u), on_plane<ZIN>(ce, m0, u), l0.z + u, L);
  if (l0.on) {
    const int q1 = (l0.x - 1) + W1::X * (l0.y - 1) + W1::PL * (l0.z - 1);
#pragma unroll
    for (int u = 0; u < W0::T; ++u) {
      const int qq = q1 + u * W1::PL;
      const float qc = apply_local(fw[u], ps, qq, W1::X, W1::PL);
      cell_put<float, W0::kUniform>(vq, on_plane<ZIN>(ce, m0, u), l0.z + u, L, qc);
      acc[0] += (double)ps[qq] * qc;
    }
  }
}

template <class S>
__global__ __launch_bounds__(kTileThreads) void k_cg_dir_apply_tile(Dims d, const float* __restrict__ ax,
                                                                    const float* __restrict__ ay,
                                                                    const float* __restrict__ az,
                                                                    const float* __restrict__ z,
                                                                    const float* __restrict__ pold,
                                                                    float* __restrict__ pnew, float* __restrict__ q,
                                                                    CGScalars* sc, double* partials,
                                                                    const double* rz_parts, int nrz, int project) {
  __shared__ float ps[Walk<S, 1>::N];
  // nrz > 0: the V-cycle's nrz r . z partials have not been totalled yet;
  // every block totals them (the same bits in each) and forms beta and zmu;
  // block 0 stores them.  They are read first, so the total waits only for them.
  constexpr int KZ = kRzPartsMax / kTileThreads;
  double pz[4][KZ];
  if (nrz > 0) partials_load_n<4, KZ, kTileThreads>(rz_parts, nrz, pz);
  if (sc->done) return;
  const bool first = sc->first;
  float beta, zmu;
  if (nrz > 0) {
    double tot[4];
    partials_reduce_n<4, KZ, kTileThreads>(pz, tot);
    const RZState rz = rz_state(sc, tot, project);
    if (blockIdx.x == 0 && threadIdx.x == 0) put_rz_state(sc, rz);
    beta = (float)rz.beta;
    zmu = (float)rz.mu;
  } else {
    beta = (float)sc->beta;
    zmu = (float)sc->zmu;
  }
  int i0, j0, k0;
  tile_origin<S>(d, i0, j0, k0);
  double acc[1] = {0.0};
  if (planes_inside<S>(k0, d.nz))
    cg_dir_apply_tile<S, true>(d, ax, ay, az, z, pold, pnew, q, first, beta, zmu, i0, j0, k0, ps, acc);
  else
    cg_dir_apply_tile<S, false>(d, ax, ay, az, z, pold, pnew, q, first, beta, zmu, i0, j0, k0, ps, acc);
  block_partials<1, kTileThreads>(acc, partials);
}

// ---------------------------------------------------------------------------
// bottom of the V-cycle: every level with at most kCoarseMaxCells cells, in one
// workgroup with the vectors in LDS (same smoother, transfers and coarsest
// sweeps as the grid levels).
// ---------------------------------------------------------------------------

template <typename A>
struct Bottom {
  int nl;
  Dims d[kMaxLevels];
  const A* ax[kMaxLevels];
  const A* ay[kMaxLevels];
  const A* az[kMaxLevels];
  const A* invd[kMaxLevels];
  int off[kMaxLevels];    // LDS offset (floats) of level l's three vectors r, z, t
  int coff[kMaxLevels];   // LDS offset of the level's staged fractions and 1/diag (FP32), -1: read from memory
  int cg;                 // > 0: the coarsest level is solved by at most cg Jacobi-preconditioned CG iterations
  int red_off;            // with cg: LDS offset (floats, even) of one double per wave for its workgroup totals
};

// Coefficients of one level, from LDS (P = float) or from memory (P = storage type).
template <typename P>
struct Coef {
  const P* ax;
  const P* ay;
  const P* az;
  const P* invd;
};

// Two more damped-Jacobi sweeps on z (through t), each followed by a barrier.
template <typename P>
__device__ inline void bottom_sweep_pair(const Dims& d, const Coef<P>& K, const float* r, float* z, float* t) {
  const int n = (int)d.cells(), T = blockDim.x;
  for (int c = threadIdx.x; c < n; c += T) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<P> fw(d, K.ax, K.ay, K.az, i, j, k);
    t[c] = z[c] + kOmega * ld(K.invd, c) * (r[c] - apply_A(d, fw, i, j, k, c, z[c], [&](long q) { return z[q]; }));
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += T) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<P> fw(d, K.ax, K.ay, K.az, i, j, k);
    z[c] = t[c] + kOmega * ld(K.invd, c) * (r[c] - apply_A(d, fw, i, j, k, c, t[c], [&](long q) { return t[q]; }));
  }
  __syncthreads();
}

// z = kBottomSweeps damped-Jacobi sweeps from 0 (t holds the first); then the
// restricted residual mean over the 8 children of (r - A z) into rc.
template <typename P>
__device__ inline void bottom_down(const Dims& d, const Dims& cd, const Coef<P>& K, const float* r, float* z, float* t,
                                   float* rc) {
  const int n = (int)d.cells(), T = blockDim.x;
  // the first sweep from 0 (t = w D^-1 r) is formed on the fly at each cell
  // and its neighbours, so the two sweeps need one barrier
  auto t1 = [&](long q) { return kOmega * ld(K.invd, q) * r[q]; };
  for (int c = threadIdx.x; c < n; c += T) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<P> fw(d, K.ax, K.ay, K.az, i, j, k);
    const float tc = t1(c);
    float Az = apply_A(d, fw, i, j, k, c, tc, t1);
    z[c] = tc + kOmega * ld(K.invd, c) * (r[c] - Az);
  }
  __syncthreads();
  for (int s = 2; s < kBottomSweeps; s += 2) bottom_sweep_pair(d, K, r, z, t);
  for (int C = threadIdx.x; C < (int)cd.cells(); C += T) {
    int I, J, K_;
    cdec(cd, C, I, J, K_);
    float s = 0.0f;
    for (int b = 0; b < 8; ++b) {
      int i = 2 * I + (b & 1), j = 2 * J + ((b >> 1) & 1), k = 2 * K_ + (b >> 2);
      int c = d.c(i, j, k);
      Faces<P> fw(d, K.ax, K.ay, K.az, i, j, k);
      s += r[c] - apply_A(d, fw, i, j, k, c, z[c], [&](long q) { return z[q]; });
    }
    rc[C] = 0.125f * s;
  }
  __syncthreads();
}

// Coarsest level: min(kCoarseSweepsMax, 2 * extent^2) damped-Jacobi sweeps
// from 0.  When every cell has its own thread, the cell's coefficients stay in
// registers across the sweeps.
template <typename P>
__device__ inline void bottom_coarsest(const Dims& d, const Coef<P>& K, const float* r, float* z, float* t) {
  const int n = (int)d.cells(), T = blockDim.x;
  const int ext = max(d.nx, max(d.ny, d.nz));
  const int sweeps = min(kCoarseSweepsMax, 2 * ext * ext);
  for (int c = threadIdx.x; c < n; c += T) z[c] = 0.0f;
  __syncthreads();
  float *src = z, *dst = t;
  if (n <= 64) {
    // one wavefront does all the sweeps: LDS operations of one wavefront are
    // performed in order, so only the compiler needs a barrier between sweeps
    if (threadIdx.x < 64) {
      const int c = threadIdx.x;
      const bool on = c < n;
      int i = 0, j = 0, k = 0;
      if (on) cdec(d, c, i, j, k);
      Faces<P> fw(d, K.ax, K.ay, K.az, on ? i : 0, on ? j : 0, on ? k : 0);
      const float idc = on ? ld(K.invd, c) : 0.0f;
      const float rc = on ? r[c] : 0.0f;
      for (int s = 0; s < sweeps; ++s) {
        if (on) {
          const float* sp = src;
          float Az = apply_A(d, fw, i, j, k, c, sp[c], [&](long q) { return sp[q]; });
          dst[c] = sp[c] + kOmega * idc * (rc - Az);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        float* tmp = src;
        src = dst;
        dst = tmp;
      }
    } else {
      if (sweeps & 1) {
        float* tmp = src;
        src = dst;
        dst = tmp;
      }
    }
    __syncthreads();
  } else if (n <= T) {
    const int c = threadIdx.x;
    const bool on = c < n;
    int i = 0, j = 0, k = 0;
    if (on) cdec(d, c, i, j, k);
    Faces<P> fw(d, K.ax, K.ay, K.az, on ? i : 0, on ? j : 0, on ? k : 0);
    const float idc = on ? ld(K.invd, c) : 0.0f;
    const float rc = on ? r[c] : 0.0f;
    for (int s = 0; s < sweeps; ++s) {
      if (on) {
        const float* sp = src;
        float Az = apply_A(d, fw, i, j, k, c, sp[c], [&](long q) { return sp[q]; });
        dst[c] = sp[c] + kOmega * idc * (rc - Az);
      }
      __syncthreads();
      float* tmp = src;
      src = dst;
      dst = tmp;
    }
  } else {
    for (int s = 0; s < sweeps; ++s) {
      for (int c = threadIdx.x; c < n; c += T) {
        int i, j, k;
        cdec(d, c, i, j, k);
        Faces<P> fw(d, K.ax, K.ay, K.az, i, j, k);
        const float* sp = src;
        float Az = apply_A(d, fw, i, j, k, c, sp[c], [&](long q) { return sp[q]; });
        dst[c] = sp[c] + kOmega * ld(K.invd, c) * (r[c] - Az);
      }
      __syncthreads();
      float* tmp = src;
      src = dst;
      dst = tmp;
    }
  }
  if (src != z) {
    for (int c = threadIdx.x; c < n; c += T) z[c] = src[c];
    __syncthreads();
  }
}

// Sum of v over the workgroup in a fixed order, returned to every thread
// (red: one double per wave; two barriers, so red can be reused at once).
__device__ inline double block_allsum(double v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
  v = wave_sum(v);
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < nw; ++q) s += red[q];
  __syncthreads();
  return s;
}

// Coarsest level of a grid whose thinnest extent stopped the coarsening
// early (e.g. 2 x 32 x 64 under a 32 x 512 x 1024 slab): its smooth modes
// span tens of cells, which Jacobi sweeps barely reach, so it gets a
// Jacobi-preconditioned CG from z = 0 instead, for at most `maxit`
// iterations or until r . D^-1 r falls by 1e-8.  Only for grounded systems
// (an OUTFLOW side), whose coarse operator is definite.  r is overwritten
// (it is the residual); t holds the direction.  The outer CG is the flexible
// form, so a preconditioner that depends on its input this way is allowed.
// Every branch depends on workgroup totals only, so all threads take it.
template <typename P>
__device__ inline void bottom_coarsest_cg(const Dims& d, const Coef<P>& K, float* r, float* z, float* p, int maxit,
                                          double* red) {
  const int n = (int)d.cells(), T = blockDim.x;
  double part = 0.0;
  for (int c = threadIdx.x; c < n; c += T) {
    const float sc = ld(K.invd, c) * r[c];
    z[c] = 0.0f;
    p[c] = sc;
    part += (double)r[c] * (double)sc;
  }
  double rho = block_allsum(part, red);
  const double stop = 1e-8 * rho;
  for (int it = 0; it < maxit && rho > stop; ++it) {
    part = 0.0;
    for (int c = threadIdx.x; c < n; c += T) {
      int i, j, k;
      cdec(d, c, i, j, k);
      Faces<P> fw(d, K.ax, K.ay, K.az, i, j, k);
      const float Ap = apply_A(d, fw, i, j, k, c, p[c], [&](long q) { return p[q]; });
      part += (double)p[c] * (double)Ap;
    }
    const double pAp = block_allsum(part, red);
    if (!(pAp > 0.0)) break;
    const float alpha = (float)(rho / pAp);
    part = 0.0;
    for (int c = threadIdx.x; c < n; c += T) {
      int i, j, k;
      cdec(d, c, i, j, k);
      Faces<P> fw(d, K.ax, K.ay, K.az, i, j, k);
      const float Ap = apply_A(d, fw, i, j, k, c, p[c], [&](long q) { return p[q]; });
      z[c] += alpha * p[c];
      const float rc = r[c] - alpha * Ap;
      r[c] = rc;
      part += (double)rc * (double)(ld(K.invd, c) * rc);
    }
    const double rho_new = block_allsum(part, red);
    const float beta = (float)(rho_new / rho);
    rho = rho_new;
    for (int c = threadIdx.x; c < n; c += T) p[c] = ld(K.invd, c) * r[c] + beta * p[c];
    __syncthreads();
  }
}

// z' = z + 8 e(parent); t = z' + w D^-1 (r - A z'); z = t + w D^-1 (r - A t).
template <typename P>
__device__ inline void bottom_up(const Dims& d, const Dims& cd, const Coef<P>& K, const float* r, float* z, float* t,
                                 const float* e) {
  const int n = (int)d.cells(), T = blockDim.x;
  auto zp = [&](long q) {
    int ti, tj, tk;
    cdec(d, q, ti, tj, tk);
    return z[q] + 8.0f * e[(ti >> 1) + cd.nx * ((tj >> 1) + cd.ny * (tk >> 1))];
  };
  for (int c = threadIdx.x; c < n; c += T) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<P> fw(d, K.ax, K.ay, K.az, i, j, k);
    float zc = zp(c);
    t[c] = zc + kOmega * ld(K.invd, c) * (r[c] - apply_A(d, fw, i, j, k, c, zc, zp));
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += T) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<P> fw(d, K.ax, K.ay, K.az, i, j, k);
    z[c] = t[c] + kOmega * ld(K.invd, c) * (r[c] - apply_A(d, fw, i, j, k, c, t[c], [&](long q) { return t[q]; }));
  }
  __syncthreads();
  for (int s = 2; s < kBottomSweeps; s += 2) bottom_sweep_pair(d, K, r, z, t);
}

template <typename A, typename R, typename Z>
__global__ __launch_bounds__(1024) void k_mg_bottom(Bottom<A> B, const R* __restrict__ rin, Z* __restrict__ zout,
                                                     const CGScalars* sc, int lvl0) {
  if (sc->done) return;
  extern __shared__ float lds[];
  const float s0 = level_scale(sc, lvl0);
  const int T = blockDim.x;
  auto R_ = [&](int l) { return lds + B.off[l]; };
  auto Z_ = [&](int l) { return lds + B.off[l] + (int)B.d[l].cells(); };
  auto T_ = [&](int l) { return lds + B.off[l] + 2 * (int)B.d[l].cells(); };
  auto staged = [&](int l) {
    const float* p = lds + B.coff[l];
    const int fx = (int)B.d[l].nfx(), fy = (int)B.d[l].nfy(), fz = (int)B.d[l].nfz();
    return Coef<float>{p, p + fx, p + fx + fy, p + fx + fy + fz};
  };
  auto global = [&](int l) { return Coef<A>{B.ax[l], B.ay[l], B.az[l], B.invd[l]}; };
  // stage the coefficients that fit, converted to FP32
  for (int l = 0; l < B.nl; ++l) {
    if (B.coff[l] < 0) continue;
    float* dst = lds + B.coff[l];
    const int fx = (int)B.d[l].nfx(), fy = (int)B.d[l].nfy(), fz = (int)B.d[l].nfz(), n = (int)B.d[l].cells();
    for (int q = threadIdx.x; q < fx; q += T) dst[q] = ld(B.ax[l], q);
    for (int q = threadIdx.x; q < fy; q += T) dst[fx + q] = ld(B.ay[l], q);
    for (int q = threadIdx.x; q < fz; q += T) dst[fx + fy + q] = ld(B.az[l], q);
    for (int q = threadIdx.x; q < n; q += T) dst[fx + fy + fz + q] = ld(B.invd[l], q);
  }
  {
    const int n = (int)B.d[0].cells();
    float* r0 = R_(0);
    for (int c = threadIdx.x; c < n; c += T) r0[c] = s0 * ld(rin, c);
  }
  __syncthreads();
  const int L = B.nl;
  for (int l = 0; l < L - 1; ++l) {
    if (B.coff[l] >= 0)
      bottom_down(B.d[l], B.d[l + 1], staged(l), R_(l), Z_(l), T_(l), R_(l + 1));
    else
      bottom_down(B.d[l], B.d[l + 1], global(l), R_(l), Z_(l), T_(l), R_(l + 1));
  }
  if (B.cg > 0) {
    // the totals' slots live in the dynamic LDS (the kernel has no static LDS:
    // its dynamic limit is set to the device's whole per-workgroup LDS)
    double* red = (double*)(lds + B.red_off);
    if (B.coff[L - 1] >= 0)
      bottom_coarsest_cg(B.d[L - 1], staged(L - 1), R_(L - 1), Z_(L - 1), T_(L - 1), B.cg, red);
    else
      bottom_coarsest_cg(B.d[L - 1], global(L - 1), R_(L - 1), Z_(L - 1), T_(L - 1), B.cg, red);
    __syncthreads();
  } else if (B.coff[L - 1] >= 0)
    bottom_coarsest(B.d[L - 1], staged(L - 1), R_(L - 1), Z_(L - 1), T_(L - 1));
  else
    bottom_coarsest(B.d[L - 1], global(L - 1), R_(L - 1), Z_(L - 1), T_(L - 1));
  for (int l = L - 2; l >= 0; --l) {
    if (B.coff[l] >= 0)
      bottom_up(B.d[l], B.d[l + 1], staged(l), R_(l), Z_(l), T_(l), Z_(l + 1));
    else
      bottom_up(B.d[l], B.d[l + 1], global(l), R_(l), Z_(l), T_(l), Z_(l + 1));
  }
  {
    const int n = (int)B.d[0].cells();
    const float* z0 = Z_(0);
    for (int c = threadIdx.x; c < n; c += T) zout[c] = cvt<Z>(z0[c]);
  }
}

// ---------------------------------------------------------------------------
// bottom with one lane per cell: every bottom level has at most as many cells
// as the workgroup has lanes, and there are at most kBottomLaneLevels levels.
// Each lane keeps its cell's fractions, 1/diag, residual and down iterate in
// registers for the whole bottom; only the iterates go through LDS.  Lanes are
// numbered children first (bottom_cell), so a restriction sums 8 consecutive
// lanes by cross-lane exchanges instead of one lane walking 8 children.  Same
// sweeps, transfers and coarsest sweeps as k_mg_bottom.
// ---------------------------------------------------------------------------

template <typename A>
struct LaneCell {
  bool on;        // the lane has a cell on this level
  int i, j, k;    // the cell
  int c;          // its index (x fastest)
  int pc;         // index of its parent on the next coarser level
  Faces<A> fw;    // its face fractions
  float idg;      // its 1 / diag
  float pidg;     // 1 / diag of the parent
};

template <typename A>
__device__ inline float lane_sweep(const Dims& d, const LaneCell<A>& q, float r, float xc, const float* src) {
  const float Ax = apply_A(d, q.fw, q.i, q.j, q.k, q.c, xc, [&](long p) { return src[p]; });
  return xc + kOmega * q.idg * (r - Ax);
}

// Coarsest level l of the bottom from 0: returns the buffer holding the result
// and leaves the lane's own value in x.
template <typename A>
__device__ inline const float* lane_coarsest(const Dims& d, const LaneCell<A>& q, float r, float* Zb, float* Tb,
                                             float& x) {
  const int n = (int)d.cells();
  const int ext = max(d.nx, max(d.ny, d.nz));
  const int sweeps = min(kCoarseSweepsMax, 2 * ext * ext);
  // sweep s writes Zb when s is even, Tb when odd; the first starts from 0
  x = q.on ? kOmega * q.idg * r : 0.0f;
  if (q.on) Zb[q.c] = x;
  if (n <= 64) {
    // the cells sit on lanes 0 .. n-1 of the first wavefront, whose LDS
    // operations are performed in order: only the compiler needs a barrier
    if (threadIdx.x < 64) {
      for (int s = 1; s < sweeps; ++s) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const float* src = (s & 1) ? Zb : Tb;
        float* dst = (s & 1) ? Tb : Zb;
        if (q.on) {
          x = lane_sweep(d, q, r, x, src);
          dst[q.c] = x;
        }
      }
    }
  } else {
    for (int s = 1; s < sweeps; ++s) {
      __syncthreads();
      const float* src = (s & 1) ? Zb : Tb;
      float* dst = (s & 1) ? Tb : Zb;
      if (q.on) {
        x = lane_sweep(d, q, r, x, src);
        dst[q.c] = x;
      }
    }
  }
  __syncthreads();
  return ((sweeps - 1) & 1) ? Tb : Zb;
}

template <typename A, typename R, typename Z>
__global__ __launch_bounds__(1024) void k_mg_bottom_lanes(Bottom<A> B, const R* __restrict__ rin,
                                                          Z* __restrict__ zout, const CGScalars* sc, int lvl0) {
  extern __shared__ float lds[];
  const int t = threadIdx.x, L = B.nl;
  const float s0 = level_scale(sc, lvl0);
  auto R_ = [&](int l) { return lds + B.off[l]; };
  auto Z_ = [&](int l) { return lds + B.off[l] + (int)B.d[l].cells(); };
  auto T_ = [&](int l) { return lds + B.off[l] + 2 * (int)B.d[l].cells(); };
  const Dims dc = B.d[L - 1];
  // every lane's cell and coefficients on every level, and the residual of
  // the finest, in one batch of loads
  LaneCell<A> o[kBottomLaneLevels];
  float rv[kBottomLaneLevels], zv[kBottomLaneLevels];
#pragma unroll
  for (int l = 0; l < kBottomLaneLevels; ++l) {
    LaneCell<A>& q = o[l];
    q.i = q.j = q.k = 0;
    q.on = l < L && bottom_cell(t, l, L, dc.nx, dc.ny, dc.nz, q.i, q.j, q.k);
    q.c = q.pc = 0;
    q.idg = q.pidg = 0.0f;
    for (int f = 0; f < 6; ++f) q.fw.w[f] = 0.0f;
    rv[l] = zv[l] = 0.0f;
    if (q.on) {
      const Dims d = B.d[l];
      q.c = d.c(q.i, q.j, q.k);
      q.fw = Faces<A>(d, B.ax[l], B.ay[l], B.az[l], q.i, q.j, q.k);
      q.idg = ld(B.invd[l], q.c);
      if (l + 1 < L) {
        q.pc = B.d[l + 1].c(q.i >> 1, q.j >> 1, q.k >> 1);
        q.pidg = ld(B.invd[l + 1], q.pc);
      }
    }
  }
  if (o[0].on) rv[0] = s0 * ld(rin, o[0].c);
  // the solver's state is read beside the batch above, not before it; a
  // launch after convergence still exits before it writes anything (the
  // empty asm keeps the compiler from moving the loads below the check)
  asm volatile("" ::: "memory");
  if (sc->done) return;

  // down: kBottomSweeps sweeps from 0 on every level but the coarsest, then
  // the residual's mean over the 8 children into the parent, with the
  // parent's first sweep from 0 (w D^-1 r) beside it
#pragma unroll
  for (int l = 0; l + 1 < kBottomLaneLevels; ++l) {
    if (l + 1 >= L) break;
    const Dims d = B.d[l];
    const LaneCell<A>& q = o[l];
    float* Zb = Z_(l);
    float* Tb = T_(l);
    float t1;
    if (l == 0) {
      t1 = kOmega * q.idg * rv[0];
      if (q.on) Tb[q.c] = t1;
      __syncthreads();
    } else {
      rv[l] = q.on ? R_(l)[q.c] : 0.0f;
      t1 = q.on ? Tb[q.c] : 0.0f;
    }
    float z = q.on ? lane_sweep(d, q, rv[l], t1, Tb) : 0.0f;
    if (q.on) Zb[q.c] = z;
    __syncthreads();
    for (int s = 2; s < kBottomSweeps; s += 2) {
      const float tt = q.on ? lane_sweep(d, q, rv[l], z, Zb) : 0.0f;
      if (q.on) Tb[q.c] = tt;
      __syncthreads();
      z = q.on ? lane_sweep(d, q, rv[l], tt, Tb) : 0.0f;
      if (q.on) Zb[q.c] = z;
      __syncthreads();
    }
    zv[l] = z;
    float res = q.on ? rv[l] - apply_A(d, q.fw, q.i, q.j, q.k, q.c, z, [&](long p) { return Zb[p]; }) : 0.0f;
    res += __shfl_xor(res, 1);
    res += __shfl_xor(res, 2);
    res += __shfl_xor(res, 4);
    if (q.on && (t & 7) == 0) {
      const float rc = 0.125f * res;
      R_(l + 1)[q.pc] = rc;
      T_(l + 1)[q.pc] = kOmega * q.pidg * rc;
    }
    __syncthreads();
  }

  // coarsest
  const float* e = nullptr;
#pragma unroll
  for (int l = 0; l < kBottomLaneLevels; ++l) {
    if (l != L - 1) continue;
    const float r = l == 0 ? rv[0] : (o[l].on ? R_(l)[o[l].c] : 0.0f);
    float x;
    e = lane_coarsest(B.d[l], o[l], r, Z_(l), T_(l), x);
    zv[l] = x;
  }

  // up: z' = z + 8 e(parent), then kBottomSweeps sweeps
#pragma unroll
  for (int l = kBottomLaneLevels - 2; l >= 0; --l) {
    if (l + 1 >= L) continue;
    const Dims d = B.d[l];
    const LaneCell<A>& q = o[l];
    float* Zb = Z_(l);
    float* Tb = T_(l);
    float z = q.on ? zv[l] + 8.0f * e[q.pc] : 0.0f;
    if (q.on) Zb[q.c] = z;   // the down iterate of this level is not read again
    __syncthreads();
    for (int s = 0; s < kBottomSweeps; s += 2) {
      const float tt = q.on ? lane_sweep(d, q, rv[l], z, Zb) : 0.0f;
      if (q.on) Tb[q.c] = tt;
      __syncthreads();
      z = q.on ? lane_sweep(d, q, rv[l], tt, Tb) : 0.0f;
      if (q.on) Zb[q.c] = z;
      if (l > 0 || s + 2 < kBottomSweeps) __syncthreads();
    }
    zv[l] = z;
    e = Zb;
  }
  if (o[0].on) zout[o[0].c] = cvt<Z>(zv[0]);
}

template <typename T>
__global__ void k_cast(long n, const float* __restrict__ src, T* __restrict__ dst, float cap) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = cvt<T>(fminf(src[i], cap));
}

// One coarse level of the hierarchy in one launch, one thread per coarse
// cell.  A coarse face is kCoarseAlphaScale times the sum of the 2 x 2 fine
// faces it covers; the thread forms its cell's six (a face shared with a
// neighbour gets the same bits from both threads: same arithmetic, same
// order), stores the ones it owns (its lower faces, and the upper faces of
// the domain's last cells) in FP32 (the next level coarsens them) and, when T
// is a 2-byte type, in T as well, and stores 1 / diag (1 / the sum of the six,
// 0 for an inactive cell, capped at `cap`) in T.  The same values, bit for
// bit, as coarsening the faces in one launch and forming 1 / diag from the
// stored faces in another.
template <typename T>
__device__ inline void store_face(float v, float* __restrict__ c32, T* __restrict__ cT, long f) {
  c32[f] = v;
  if constexpr (!std::is_same<T, float>::value) cT[f] = cvt<T>(fminf(v, 3e38f));
}

template <typename T>
__global__ void k_coarse_level(Dims fd, Dims cd, const float* __restrict__ fax, const float* __restrict__ fay,
                               const float* __restrict__ faz, float* __restrict__ cax, float* __restrict__ cay,
                               float* __restrict__ caz, T* __restrict__ tax, T* __restrict__ tay, T* __restrict__ taz,
                               T* __restrict__ invd, float cap) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)cd.cells()) return;
  const int I = (int)(c % cd.nx);
  const long t = c / cd.nx;
  const int J = (int)(t % cd.ny);
  const int K = (int)(t / cd.ny);
  // coarse faces of the three components at coarse face coordinates
  auto fxv = [&](int a, int b, int e) {
    const int i = 2 * a, j = 2 * b, k = 2 * e;
    const float s = fax[fd.fx(i, j, k)] + fax[fd.fx(i, j + 1, k)] + fax[fd.fx(i, j, k + 1)] + fax[fd.fx(i, j + 1, k + 1)];
    return kCoarseAlphaScale * s;
  };
  auto fyv = [&](int a, int b, int e) {
    const int i = 2 * a, j = 2 * b, k = 2 * e;
    const float s = fay[fd.fy(i, j, k)] + fay[fd.fy(i + 1, j, k)] + fay[fd.fy(i, j, k + 1)] + fay[fd.fy(i + 1, j, k + 1)];
    return kCoarseAlphaScale * s;
  };
  auto fzv = [&](int a, int b, int e) {
    const int i = 2 * a, j = 2 * b, k = 2 * e;
    const float s = faz[fd.fz(i, j, k)] + faz[fd.fz(i + 1, j, k)] + faz[fd.fz(i, j + 1, k)] + faz[fd.fz(i + 1, j + 1, k)];
    return kCoarseAlphaScale * s;
  };
  const float x0 = fxv(I, J, K), x1 = fxv(I + 1, J, K);
  const float y0 = fyv(I, J, K), y1 = fyv(I, J + 1, K);
  const float z0 = fzv(I, J, K), z1 = fzv(I, J, K + 1);
  store_face<T>(x0, cax, tax, cd.fx(I, J, K));
  if (I == cd.nx - 1) store_face<T>(x1, cax, tax, cd.fx(I + 1, J, K));
  store_face<T>(y0, cay, tay, cd.fy(I, J, K));
  if (J == cd.ny - 1) store_face<T>(y1, cay, tay, cd.fy(I, J + 1, K));
  store_face<T>(z0, caz, taz, cd.fz(I, J, K));
  if (K == cd.nz - 1) store_face<T>(z1, caz, taz, cd.fz(I, J, K + 1));
  const float s = x0 + x1 + y0 + y1 + z0 + z1;
  const float v = s > 0.0f ? 1.0f / s : 0.0f;
  invd[c] = cvt<T>(fminf(v, cap));
}

static inline unsigned nblocks(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------

// Whether the direction kernel totals the V-cycle's r . z partials itself
// (fused grid levels above the bottom, at most kRzPartsMax finest tiles);
// otherwise k_fin_rz does, at the end of the V-cycle.
static bool rz_in_direction(const Solver& S) {
  return S.fused && S.nbottom > 0 && tiles_of<FineTile>(S.lev[0].d) <= kRzPartsMax;
}

// nrr > 0: the V-cycle follows a CG update whose nrr r . r partials have not
// been totalled yet (the finest fused down kernel does it, else k_fin_rr).
template <typename T>
static void vcycle(const Solver& S, const float* r0, float* z0, hipStream_t st, int nrr) {
  const int L = S.nlev;
  const int G = S.nbottom;  // levels 0 .. G-1 run as grid kernels, G .. L-1 in one workgroup
  CGScalars* sc = S.sc;
  auto A = [&](int l) { return (const T*)S.lev[l].a[0]; };
  auto Ay = [&](int l) { return (const T*)S.lev[l].a[1]; };
  auto Az = [&](int l) { return (const T*)S.lev[l].a[2]; };
  auto ID = [&](int l) { return (const T*)S.lev[l].invd; };
  const long n0 = (long)S.lev[0].d.cells();
  Bottom<T> B;
  B.nl = L - G;
  {
    // grounded systems whose coarsest level stayed large: CG there (at most
    // twice its largest extent in iterations)
    const Dims& dc = S.lev[L - 1].d;
    const int ext = std::max(dc.nx, std::max(dc.ny, dc.nz));
    B.cg = (!S.project && dc.cells() > (size_t)kBottomCells) ? std::min(2 * ext, 256) : 0;
  }
  B.red_off = 0;
  int off = 0;
  for (int q = 0; q < B.nl; ++q) {
    const int l = G + q;
    B.d[q] = S.lev[l].d;
    B.ax[q] = A(l);
    B.ay[q] = Ay(l);
    B.az[q] = Az(l);
    B.invd[q] = ID(l);
    B.off[q] = off;
    B.coff[q] = -1;
    off += 3 * (int)S.lev[l].d.cells();
  }
  const size_t lds_lanes = (size_t)off * sizeof(float);
  if (B.cg > 0) {
    B.red_off = (off + 1) & ~1;                 // 8-byte aligned (the dynamic LDS base is)
    off = B.red_off + 2 * (1024 / 64);          // one double per wave of the largest workgroup
  }
  // stage coefficients in LDS from the coarsest level up, while they fit
  for (int q = B.nl - 1; q >= 0; --q) {
    const Dims& d = S.lev[G + q].d;
    const int need = (int)(d.nfx() + d.nfy() + d.nfz() + d.cells());
    if ((size_t)(off + need) * sizeof(float) > S.lds_bytes) break;
    B.coff[q] = off;
    off += need;
  }
  const size_t lds = (size_t)off * sizeof(float);
  const int bthreads = S.lev[G].d.cells() >= 1024 ? 1024 : (int)((S.lev[G].d.cells() + 63) / 64 * 64);
  // one lane per cell when the finest bottom level fits the workgroup
  const bool lanes = S.bottom_lanes && S.lev[G].d.cells() <= 1024 && B.nl <= kBottomLaneLevels;
  auto bottom = [&](auto kernel, auto lanes_kernel, auto rin, auto zout, int lvl0) {
    if (lanes)
      NF_LAUNCH(S.prof, SIM_K_MG_COARSE, lanes_kernel, dim3(1), dim3(bthreads), lds_lanes, st, B, rin, zout, sc, lvl0);
    else
      NF_LAUNCH(S.prof, SIM_K_MG_COARSE, kernel, dim3(1), dim3(bthreads), lds, st, B, rin, zout, sc, lvl0);
  };
  if (nrr > 0 && !(S.fused && G > 0))
    hipLaunchKernelGGL(k_fin_rr, dim3(1), dim3(kFinBlock), 0, st, nrr, S.partials_rr, sc, n0);
  if (G == 0) {
    bottom(k_mg_bottom<T, float, float>, k_mg_bottom_lanes<T, float, float>, r0, z0, 1);
    hipLaunchKernelGGL(k_scale_dot<T>, dim3(nblocks(n0)), dim3(kBlock), 0, st, n0, ID(0), r0, z0, sc, S.partials);
    hipLaunchKernelGGL(k_fin_rz, dim3(1), dim3(kFinBlock), 0, st, (int)nblocks(n0), S.partials, sc, S.project);
    return;
  }
  if (S.fused) {
    // coarse levels of at least kWideTileCells cells use 16 x 8 x 8 tiles (half
    // the workgroups and less halo per cell), smaller ones 8 x 8 x 8 (enough
    // workgroups to spread their latency-bound launches)
    auto wide = [](const Dims& d) { return d.cells() >= (size_t)kWideTileCells; };
    for (int l = 0; l < G; ++l) {
      const Dims& d = S.lev[l].d;
      const Dims& cd = S.lev[l + 1].d;
      T* rc = (T*)S.lev[l + 1].r;
      if (l == 0) {
        bool done = false;
        if constexpr (kHasRecords<T>) {
          if (S.rec0) {
            NF_LAUNCH(S.prof, SIM_K_MG_DOWN, (k_mg_down<FineTile, T, float, float, T, 0, true>),
                      dim3(tiles_of<FineTile>(d)), dim3(kTileThreads), 0, st, d, cd, A(0), Ay(0), Az(0), ID(0), r0,
                      (float*)S.lev[0].ta, rc, sc, 1, S.partials_rr, nrr, n0, (const void*)S.rec0);
            done = true;
          }
        }
        if (!done)
          NF_LAUNCH(S.prof, SIM_K_MG_DOWN, (k_mg_down<FineTile, T, float, float, T, false>), dim3(tiles_of<FineTile>(d)),
                    dim3(kTileThreads), 0, st, d, cd, A(0), Ay(0), Az(0), ID(0), r0, (float*)S.lev[0].ta, rc, sc, 1,
                    S.partials_rr, nrr, n0, nullptr);
      } else if (wide(d)) {
        hipLaunchKernelGGL((k_mg_down<CoarseTileH, T, T, T, T, true>), dim3(tiles_of<CoarseTileH>(d)), dim3(kTileThreads), 0, st, d, cd,
                           A(l), Ay(l), Az(l), ID(l), (const T*)S.lev[l].r, (T*)S.lev[l].ta, rc, sc, 0, nullptr, 0, 0L);
      } else {
        hipLaunchKernelGGL((k_mg_down<CoarseTile, T, T, T, T, true>), dim3(tiles_of<CoarseTile>(d)), dim3(kTileThreads), 0, st, d, cd,
                           A(l), Ay(l), Az(l), ID(l), (const T*)S.lev[l].r, (T*)S.lev[l].ta, rc, sc, 0, nullptr, 0, 0L);
      }
    }
    bottom(k_mg_bottom<T, T, T>, k_mg_bottom_lanes<T, T, T>, (const T*)S.lev[G].r, (T*)S.lev[G].z, 0);
    for (int l = G - 1; l >= 0; --l) {
      const Dims& d = S.lev[l].d;
      const Dims& cd = S.lev[l + 1].d;
      const T* e = (const T*)S.lev[l + 1].z;
      if (l == 0) {
        const bool merged = rz_in_direction(S);
        bool done = false;
        if constexpr (kHasRecords<T>) {
          if (S.rec0) {
            NF_LAUNCH(S.prof, SIM_K_MG_UP, (k_mg_up<FineTile, T, float, float, T, float, true, 0, true>),
                      dim3(tiles_of<FineTile>(d)), dim3(kTileThreads), 0, st, d, cd, A(0), Ay(0), Az(0), ID(0), r0,
                      (const float*)S.lev[0].ta, e, z0, sc, merged ? S.partials_rz : S.partials, (const void*)S.rec0);
            done = true;
          }
        }
        if (!done)
          NF_LAUNCH(S.prof, SIM_K_MG_UP, (k_mg_up<FineTile, T, float, float, T, float, true, false>),
                    dim3(tiles_of<FineTile>(d)), dim3(kTileThreads), 0, st, d, cd, A(0), Ay(0), Az(0), ID(0), r0,
                    (const float*)S.lev[0].ta, e, z0, sc, merged ? S.partials_rz : S.partials, nullptr);
        if (!merged)
          hipLaunchKernelGGL(k_fin_rz, dim3(1), dim3(kFinBlock), 0, st, (int)tiles_of<FineTile>(d), S.partials, sc, S.project);
      } else if (wide(d)) {
        hipLaunchKernelGGL((k_mg_up<CoarseTileH, T, T, T, T, T, false, true>), dim3(tiles_of<CoarseTileH>(d)), dim3(kTileThreads), 0, st,
                           d, cd, A(l), Ay(l), Az(l), ID(l), (const T*)S.lev[l].r, (const T*)S.lev[l].ta, e, (T*)S.lev[l].z, sc,
                           S.partials);
      } else {
        hipLaunchKernelGGL((k_mg_up<CoarseTile, T, T, T, T, T, false, true>), dim3(tiles_of<CoarseTile>(d)), dim3(kTileThreads), 0, st,
                           d, cd, A(l), Ay(l), Az(l), ID(l), (const T*)S.lev[l].r, (const T*)S.lev[l].ta, e, (T*)S.lev[l].z, sc,
                           S.partials);
      }
    }
    return;
  }
  for (int l = 0; l < G; ++l) {
    const Dims& d = S.lev[l].d;
    const Dims& cd = S.lev[l + 1].d;
    T* ta = (T*)S.lev[l].ta;
    T* rc = (T*)S.lev[l + 1].r;
    if (l == 0) {
      float* ta0 = (float*)S.lev[0].ta;
      NF_LAUNCH(S.prof, SIM_K_MG_DOWN, (k_mg_pre<T, float, float>), dim3(nblocks(d.cells())), dim3(kBlock), 0, st, d,
                                  A(0), Ay(0), Az(0), ID(0), r0, ta0, sc, 1);
      NF_LAUNCH(S.prof, SIM_K_MG_DOWN2, (k_mg_restrict<T, float, float, T>), dim3(nblocks(cd.cells())), dim3(kBlock), 0,
                                  st, d, cd, A(0), Ay(0), Az(0), r0, (const float*)ta0, rc, sc, 1);
    } else {
      const T* rl = (const T*)S.lev[l].r;
      hipLaunchKernelGGL((k_mg_pre<T, T, T>), dim3(nblocks(d.cells())), dim3(kBlock), 0, st, d, A(l), Ay(l),
                         Az(l), ID(l), rl, ta, sc, 0);
      hipLaunchKernelGGL((k_mg_restrict<T, T, T, T>), dim3(nblocks(cd.cells())), dim3(kBlock), 0, st, d, cd, A(l),
                         Ay(l), Az(l), rl, (const T*)ta, rc, sc, 0);
    }
  }
  bottom(k_mg_bottom<T, T, T>, k_mg_bottom_lanes<T, T, T>, (const T*)S.lev[G].r, (T*)S.lev[G].z, 0);
  for (int l = G - 1; l >= 0; --l) {
    const Dims& d = S.lev[l].d;
    const Dims& cd = S.lev[l + 1].d;
    const T* ta = (const T*)S.lev[l].ta;
    T* tb = (T*)S.lev[l].tb;
    const T* e = (const T*)S.lev[l + 1].z;
    if (l == 0) {
      const float* ta0 = (const float*)S.lev[0].ta;
      float* tb0 = (float*)S.lev[0].tb;
      NF_LAUNCH(S.prof, SIM_K_MG_UP1, (k_mg_post1<T, float, float, T>), dim3(nblocks(d.cells())), dim3(kBlock), 0, st, d,
                                  cd, A(0), Ay(0), Az(0), ID(0), r0, ta0, e, tb0, sc, 1);
      NF_LAUNCH(S.prof, SIM_K_MG_UP, (k_mg_post2<T, float, float, float, true>), dim3(nblocks(d.cells())), dim3(kBlock),
                                  0, st, d, A(0), Ay(0), Az(0), ID(0), r0, (const float*)tb0, z0, sc, S.partials);
      hipLaunchKernelGGL(k_fin_rz, dim3(1), dim3(kFinBlock), 0, st, (int)nblocks(d.cells()), S.partials, sc,
                         S.project);
    } else {
      const T* rl = (const T*)S.lev[l].r;
      hipLaunchKernelGGL((k_mg_post1<T, T, T, T>), dim3(nblocks(d.cells())), dim3(kBlock), 0, st, d, cd, A(l),
                         Ay(l), Az(l), ID(l), rl, ta, e, tb, sc, 0);
      hipLaunchKernelGGL((k_mg_post2<T, T, T, T, false>), dim3(nblocks(d.cells())), dim3(kBlock), 0, st, d, A(l),
                         Ay(l), Az(l), ID(l), rl, (const T*)tb, (T*)S.lev[l].z, sc, S.partials);
    }
  }
}

static void vcycle_dispatch(const Solver& S, const float* r0, float* z0, hipStream_t st, int nrr = 0) {
  if (S.precision == SIM_MIXED_FP16)
    vcycle<__half>(S, r0, z0, st, nrr);
  else if (S.precision == SIM_MIXED_BF16)
    vcycle<__hip_bfloat16>(S, r0, z0, st, nrr);
  else
    vcycle<float>(S, r0, z0, st, nrr);
}

template <typename T>
static void cast_level(const Dims& d, const float* lx, const float* ly, const float* lz, const float* inv,
                       const Level& L, float invcap, hipStream_t st) {
  hipLaunchKernelGGL(k_cast<T>, dim3(nblocks(d.nfx())), dim3(kBlock), 0, st, (long)d.nfx(), lx, (T*)L.a[0], 3e38f);
  hipLaunchKernelGGL(k_cast<T>, dim3(nblocks(d.nfy())), dim3(kBlock), 0, st, (long)d.nfy(), ly, (T*)L.a[1], 3e38f);
  hipLaunchKernelGGL(k_cast<T>, dim3(nblocks(d.nfz())), dim3(kBlock), 0, st, (long)d.nfz(), lz, (T*)L.a[2], 3e38f);
  hipLaunchKernelGGL(k_cast<T>, dim3(nblocks(d.cells())), dim3(kBlock), 0, st, (long)d.cells(), inv, (T*)L.invd,
                     invcap);
}

// The finest level's packed coefficient records, from its FP32 fractions.
template <typename T>
static void pack_records(const Solver& S, const float* fx, const float* fy, const float* fz, hipStream_t st) {
  if (!S.rec0) return;
  const Level& L = S.lev[0];
  hipLaunchKernelGGL(k_pack_records<T>, dim3(nblocks(L.d.cells())), dim3(kBlock), 0, st, L.d, fx, fy, fz,
                     (typename RecOf<T>::T*)S.rec0, (float*)((Rec16*)S.rec0 + L.d.cells()));
}

// Multigrid copies of the fine fractions and inverse diagonals.
void solver_setup_levels(Solver& S, const float* fine_alpha, hipStream_t st) {
  const Dims& d0 = S.lev[0].d;
  const float* fx = fine_alpha;
  const float* fy = fx + d0.nfx();
  const float* fz = fy + d0.nfy();
  S.ax = fx;
  S.ay = fy;
  S.az = fz;
  // connected-region labels belong to one geometry
  S.comp.valid = false;
  if (S.comp.mode == SIM_REGIONS_ALWAYS) components_label(S, st);
  if (S.precision == SIM_FP32) {
    S.lev[0].a[0] = (void*)fx;
    S.lev[0].a[1] = (void*)fy;
    S.lev[0].a[2] = (void*)fz;
    launch_invdiag(d0, fx, fy, fz, (float*)S.lev[0].invd, st);
    for (int l = 1; l < S.nlev; ++l) {
      const Dims& fd = S.lev[l - 1].d;
      const Dims& cd = S.lev[l].d;
      float* cx = (float*)S.lev[l].a[0];
      float* cy = (float*)S.lev[l].a[1];
      float* cz = (float*)S.lev[l].a[2];
      hipLaunchKernelGGL(k_coarse_level<float>, dim3(nblocks(cd.cells())), dim3(kBlock), 0, st, fd, cd,
                         (const float*)S.lev[l - 1].a[0], (const float*)S.lev[l - 1].a[1],
                         (const float*)S.lev[l - 1].a[2], cx, cy, cz, cx, cy, cz, (float*)S.lev[l].invd, 3e38f);
    }
    return;
  }
  // mixed: build each level in FP32 scratch, then store it in T
  for (int l = 0; l < S.nlev; ++l) {
    // FP16: level 0 only needs 1/diag to stay finite (its iterates are FP32);
    // coarser levels store their iterates in FP16 and keep the tighter cap
    const float cap = S.precision != SIM_MIXED_FP16 ? 3e38f : (l == 0 ? kHalfMax : kHalfInvDiagMax);
    const Dims& d = S.lev[l].d;
    if (l > 0) {
      // coarse levels: one launch storing the FP32 faces and the copies in
      // the storage type (instead of coarsening, 1 / diag and a cast per array)
      const Dims& fd = S.lev[l - 1].d;
      float* cx = S.scratch_a + S.scratch_off[l];
      float* cy = cx + d.nfx();
      float* cz = cy + d.nfy();
      const float* px = l == 1 ? fx : S.scratch_a + S.scratch_off[l - 1];
      const float* py = l == 1 ? fy : px + fd.nfx();
      const float* pz = l == 1 ? fz : py + fd.nfy();
      const Level& L = S.lev[l];
      if (S.precision == SIM_MIXED_FP16)
        hipLaunchKernelGGL(k_coarse_level<__half>, dim3(nblocks(d.cells())), dim3(kBlock), 0, st, fd, d, px, py, pz,
                           cx, cy, cz, (__half*)L.a[0], (__half*)L.a[1], (__half*)L.a[2], (__half*)L.invd, cap);
      else
        hipLaunchKernelGGL(k_coarse_level<__hip_bfloat16>, dim3(nblocks(d.cells())), dim3(kBlock), 0, st, fd, d, px,
                           py, pz, cx, cy, cz, (__hip_bfloat16*)L.a[0], (__hip_bfloat16*)L.a[1],
                           (__hip_bfloat16*)L.a[2], (__hip_bfloat16*)L.invd, cap);
      continue;
    }
    const float *lx = fx, *ly = fy, *lz = fz;
    // the fused V-cycle reads level 0's coefficients from the packed records
    // (below): its 2-byte arrays would go unread
    if (l == 0 && S.fused && S.rec0) continue;
    launch_invdiag(d, lx, ly, lz, S.scratch_inv, st);
    if (S.precision == SIM_MIXED_FP16)
      cast_level<__half>(d, lx, ly, lz, S.scratch_inv, S.lev[l], cap, st);
    else
      cast_level<__hip_bfloat16>(d, lx, ly, lz, S.scratch_inv, S.lev[l], cap, st);
  }
  if (S.precision == SIM_MIXED_FP16)
    pack_records<__half>(S, fx, fy, fz, st);
  else
    pack_records<__hip_bfloat16>(S, fx, fy, fz, st);
}

// The V-cycle's output, then (with region labels) its region-by-region shift.
static void precondition(Solver& S, hipStream_t st, int nrr = 0) {
  vcycle_dispatch(S, S.r, S.z, st, nrr);
  if (S.comp.valid) components_shift_z(S, st);
}

static void enqueue_iterations(Solver& S, double* x, int count, hipStream_t st) {
  const Dims& d = S.lev[0].d;
  const long n = (long)d.cells();
  for (int c = 0; c < count; ++c) {
    float* pold = S.pcur ? S.p1 : S.p0;
    float* pnew = S.pcur ? S.p0 : S.p1;
    const int nb = (int)nblocks(n);
    int npq = nb;
    if (S.fused) {
      npq = tiles_of<FineTile>(d);
      const int nrz = rz_in_direction(S) ? npq : 0;
      NF_LAUNCH(S.prof, SIM_K_CG_APPLY, k_cg_dir_apply_tile<FineTile>, dim3(npq), dim3(kTileThreads), 0, st, d, S.ax,
                S.ay, S.az, S.z, pold, pnew, S.q, S.sc, S.partials, S.partials_rz, nrz, S.project);
    } else {
      NF_LAUNCH(S.prof, SIM_K_CG_APPLY, k_cg_dir_apply, dim3(nb), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, S.z, pold,
                                  pnew, S.q, S.sc, S.partials);
    }
    const int nu = nb < kUpdateBlocks ? nb : kUpdateBlocks;
    NF_LAUNCH(S.prof, SIM_K_CG_UPDATE, k_cg_update, dim3(nu), dim3(kBlock), 0, st, n, x, S.r, pnew, S.q, S.sc,
              S.partials, npq, S.partials_rr);
    // with region labels the updated residual is projected region by region
    // (its FP32 rounding otherwise leaves region sums that the shifted z would
    // weight with the V-cycle's large region constants in r . z)
    if (S.comp.valid) components_project_iter(S, nu, st);
    precondition(S, st, nu);
    S.pcur ^= 1;
  }
}

// Capture two iterations (starting with p0 as the current direction) into a
// graph; replaying it leaves the direction parity unchanged.  One graph per
// form of the iteration (with or without the region shift of z).
static bool capture_pair(Solver& S, double* x) {
  const int v = S.comp.valid ? 1 : 0;
  if (S.iter_exec[v]) return true;
  if (!S.cap_stream && hipStreamCreateWithFlags(&S.cap_stream, hipStreamNonBlocking) != hipSuccess) return false;
  if (hipStreamBeginCapture(S.cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return false;
  const int saved = S.pcur;
  S.pcur = 0;
  Profiler* prof = S.prof;
  S.prof = nullptr;
  enqueue_iterations(S, x, 2, S.cap_stream);
  S.prof = prof;
  S.pcur = saved;
  if (hipStreamEndCapture(S.cap_stream, &S.iter_graph[v]) != hipSuccess) return false;
  if (hipGraphInstantiate(&S.iter_exec[v], S.iter_graph[v], nullptr, nullptr, 0) != hipSuccess) {
    S.iter_exec[v] = nullptr;
    return false;
  }
  return true;
}

// Run `count` CG iterations (count is rounded up to an even number when the
// captured pair is replayed; surplus iterations after convergence are skipped
// on the device).  Returns the number enqueued.
static int cg_iterations(Solver& S, double* x, int count, hipStream_t st) {
  const bool timing = S.prof && S.prof->active >= 0;
  if (S.use_graph && !timing && S.pcur == 0 && capture_pair(S, x)) {
    const int pairs = (count + 1) / 2;
    for (int q = 0; q < pairs; ++q) (void)hipGraphLaunch(S.iter_exec[S.comp.valid ? 1 : 0], st);
    return 2 * pairs;
  }
  enqueue_iterations(S, x, count, st);
  return count;
}

// Dynamic LDS available to the one-workgroup bottom solve on the current device.
void solver_init_device(Solver& S) {
  int dev = 0, v = 0;
  S.lds_bytes = 65536;
  if (hipGetDevice(&dev) != hipSuccess) return;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) return;
  const void* fns[6] = {(const void*)k_mg_bottom<float, float, float>,
                        (const void*)k_mg_bottom<__half, float, float>,
                        (const void*)k_mg_bottom<__hip_bfloat16, float, float>,
                        (const void*)k_mg_bottom<float, float, float>,
                        (const void*)k_mg_bottom<__half, __half, __half>,
                        (const void*)k_mg_bottom<__hip_bfloat16, __hip_bfloat16, __hip_bfloat16>};
  for (const void* f : fns)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess) {
      (void)hipGetLastError();   // keep the default limit and leave no error behind
      return;
    }
  S.lds_bytes = (size_t)v;
}

void solver_release(Solver& S) {
  for (int v = 0; v < 2; ++v) {
    if (S.iter_exec[v]) (void)hipGraphExecDestroy(S.iter_exec[v]);
    if (S.iter_graph[v]) (void)hipGraphDestroy(S.iter_graph[v]);
    S.iter_exec[v] = nullptr;
    S.iter_graph[v] = nullptr;
  }
  if (S.cap_stream) (void)hipStreamDestroy(S.cap_stream);
  S.cap_stream = nullptr;
}

static int snapshot(Solver& S, hipStream_t st) {
  if (hipMemcpyAsync(S.host_sc, S.sc, sizeof(CGScalars), hipMemcpyDeviceToHost, st) != hipSuccess) return SIM_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SIM_EHIP;
  if (S.trace) {
    const CGScalars& h = *S.host_sc;
    fprintf(stderr, "[nf-solver] iters %d done %d conv %d first %d rel %.3e true %.3e vscale %.3e\n", h.iters, h.done,
            h.converged, h.first, h.bb > 0 ? sqrt(h.rr / h.bb) : 0.0, h.bb > 0 ? sqrt(h.true_rr / h.bb) : 0.0,
            h.vscale);
  }
  return SIM_OK;
}

// Solves that never wait on the host: a fixed budget of iterations with a
// true-residual check (and a conditional restart) behind every chunk; every
// kernel enqueued after convergence exits at once on the device.
// The finest level's 1/diag in FP32 (0 on inactive cells), or NULL where the
// level keeps it only in 2-byte storage.
static const float* fine_invd32(const Solver& S) {
  if (S.precision == SIM_FP32) return (const float*)S.lev[0].invd;
  if (S.rec0) return (const float*)((const Rec16*)S.rec0 + S.lev[0].d.cells());
  return nullptr;
}

// r -= its mean over the active cells (closed domains without region labels).
static void sub_mean(Solver& S, hipStream_t st) {
  const Dims& d = S.lev[0].d;
  const long n = (long)d.cells();
  if (const float* id = fine_invd32(S))
    hipLaunchKernelGGL(k_sub_mean_inv, dim3(nblocks(n)), dim3(kBlock), 0, st, n, id, S.r, S.sc);
  else
    hipLaunchKernelGGL(k_sub_mean, dim3(nblocks(n)), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, S.r, S.sc);
}

// The solve's output: the iterate on active cells, 0 elsewhere.
static void x_store(Solver& S, const double* x, float* xout, hipStream_t st) {
  const Dims& d = S.lev[0].d;
  const long n = (long)d.cells();
  if (const float* id = fine_invd32(S))
    hipLaunchKernelGGL(k_x_store_inv, dim3(nblocks(n)), dim3(kBlock), 0, st, n, id, x, xout);
  else
    hipLaunchKernelGGL(k_x_store, dim3(nblocks(n)), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, x, xout);
}

static void solve_on_device(Solver& S, const float* b, double* x, int budget, hipStream_t st) {
  const Dims& d = S.lev[0].d;
  const long n = (long)d.cells();
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) cap = hipStreamCaptureStatusNone;
  // the captured iteration pair is not replayed inside a caller's capture
  const bool graphs = cap == hipStreamCaptureStatusNone;
  const int chunk = kDeviceCheckEvery;
  for (int left = budget; left > 0;) {
    const int c = left < chunk ? left : chunk;
    if (graphs)
      left -= cg_iterations(S, x, c, st);
    else {
      enqueue_iterations(S, x, c, st);
      left -= c;
    }
    const int nbt = (int)std::min<size_t>(nblocks(n), kInitBlocks);
    hipLaunchKernelGGL(k_cg_true_residual, dim3(nbt), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, b, x, S.r, 1, S.sc,
                       S.partials);
    hipLaunchKernelGGL(k_fin_true, dim3(1), dim3(kFinBlock), 0, st, nbt, S.partials, S.sc, 1, n, S.project);
    if (left <= 0) break;
    hipLaunchKernelGGL(k_hold_restart, dim3(1), dim3(1), 0, st, S.sc);
    if (S.comp.valid)
      components_subtract(S, st);
    else if (S.project)
      sub_mean(S, st);
    precondition(S, st);
    hipLaunchKernelGGL(k_release_restart, dim3(1), dim3(1), 0, st, S.sc);
  }
}

int solver_solve(Solver& S, SolveKind kind, const float* b, float* xio, double tol, int maxit, sim_stats* stats,
                 hipStream_t st, bool zero_guess) {
  const Dims& d = S.lev[0].d;
  const long n = (long)d.cells();
  CGScalars* sc = S.sc;
  double* x = S.x;
  if (S.device_mode && S.budget > 0 && S.budget < maxit) maxit = S.budget;
  const float* invd32 = zero_guess ? fine_invd32(S) : nullptr;
  if (zero_guess && !invd32) {
    // no FP32 1/diag to find the active cells by: start from an explicit zero
    launch_fill(xio, (size_t)n, 0.0f, st);
    zero_guess = false;
  }
  if (zero_guess) {
    const int nb = (int)std::min<size_t>(nblocks(n), kInitBlocks);
    NF_LAUNCH(S.prof, SIM_K_CG_INIT, k_cg_init_zero, dim3(nb), dim3(kBlock), 0, st, n, invd32, b, x, S.r,
              S.partials);
    hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(kFinBlock), 0, st, nb, S.partials, sc, tol, maxit, n, S.project);
  } else {
    hipLaunchKernelGGL(k_x_load, dim3(nblocks(n)), dim3(kBlock), 0, st, n, xio, x);
    const int nb = (int)std::min<size_t>(nblocks(n), kInitBlocks);
    NF_LAUNCH(S.prof, SIM_K_CG_INIT, k_cg_init, dim3(nb), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, b, x, S.r,
              S.partials);
    hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(kFinBlock), 0, st, nb, S.partials, sc, tol, maxit, n, S.project);
  }
  if (S.comp.valid)
    components_project_start(S, st);
  else if (S.project)
    sub_mean(S, st);
  precondition(S, st);
  S.pcur = 0;
  if (S.device_mode) {
    solve_on_device(S, b, x, maxit, st);
    x_store(S, x, xio, st);
    if (stats) hipLaunchKernelGGL(k_write_stats, dim3(1), dim3(1), 0, st, sc, stats);
    return SIM_OK;
  }
  // Each round enqueues a batch of iterations and the (conditional) true-
  // residual check behind it, then synchronises once.  The first batch is
  // sized from the previous solve of this handle, so a typical solve needs a
  // single round; iterations enqueued after convergence exit at once on the
  // device.  Every round runs iterations or uses up one of a bounded number of
  // restarts, and the round count is capped, so the loop terminates.
  int batch = S.last_iters[kind] > 0 ? S.last_iters[kind] : 2;
  const int chunk = S.check_every > 0 ? S.check_every : 2;
  int restarts = 0, checks_seen = 0, rounds = 0;
  for (;;) {
    const int allow = restarts < kMaxRestarts ? 1 : 0;
    (void)cg_iterations(S, x, batch, st);
    const int nbt = (int)std::min<size_t>(nblocks(n), kInitBlocks);
    NF_LAUNCH(S.prof, SIM_K_CG_TRUE, k_cg_true_residual, dim3(nbt), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, b, x,
              S.r, allow, sc, S.partials);
    hipLaunchKernelGGL(k_fin_true, dim3(1), dim3(kFinBlock), 0, st, nbt, S.partials, sc, allow, n, S.project);
    int r = snapshot(S, st);
    if (r != SIM_OK) return r;
    batch = chunk;
    const CGScalars& h = *S.host_sc;
    if (h.nonfinite) break;
    if (++rounds > maxit + 2 * kMaxRestarts + 8) break;
    if (h.checks == checks_seen) continue;   // still iterating
    checks_seen = h.checks;
    if (h.converged || !allow || h.iters >= maxit || h.done) break;
    // the check restarted CG from the true residual
    ++restarts;
    hipLaunchKernelGGL(k_release_restart, dim3(1), dim3(1), 0, st, sc);
    if (S.comp.valid)
      components_subtract(S, st);
    else if (S.project)
      sub_mean(S, st);
    precondition(S, st);
  }
  {
    // A solve that stalls short of the tolerance without a NaN / Inf on a
    // geometry whose connected regions are not labelled yet: label them and
    // solve again with the residual projected region by region (a floating
    // region's rounding-level incompatibility would otherwise hold the
    // residual up).  The initial guess is still in xio.
    const CGScalars& h = *S.host_sc;
    if (!h.converged && !h.nonfinite && !S.comp.valid && S.comp.mode == SIM_REGIONS_AUTO) {
      components_label(S, st);
      return solver_solve(S, kind, b, xio, tol, maxit, stats, st, zero_guess);
    }
  }
  S.last_iters[kind] = S.host_sc->iters;
  x_store(S, x, xio, st);
  const CGScalars& h = *S.host_sc;
  if (stats) {
    stats->iters = h.iters;
    stats->nonfinite = h.nonfinite;
    stats->converged = h.converged && !h.nonfinite;
    stats->pad = 0;
    stats->rel_res = h.bb > 0.0 ? sqrt(h.rr / h.bb) : 0.0;
    stats->true_rel_res = h.bb > 0.0 ? sqrt(h.true_rr / h.bb) : 0.0;
  }
  if (h.nonfinite) return SIM_WNONFINITE;
  if (!h.converged) return SIM_WNOCONV;
  return SIM_OK;
}

}  // namespace nf
