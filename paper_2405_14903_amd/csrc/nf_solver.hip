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
//     damped-Jacobi sweeps (omega = 0.8) before and after the correction, and
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

#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstdio>

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

__device__ inline void cdec(const Dims& d, long c, int& i, int& j, int& k) {
  const unsigned cu = (unsigned)c, nx = (unsigned)d.nx, ny = (unsigned)d.ny;
  const unsigned t = cu / nx;
  i = (int)(cu - t * nx);
  k = (int)(t / ny);
  j = (int)(t - (unsigned)k * ny);
}

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

__device__ inline double vscale_of(double rr, long n) {
  double rms = sqrt(rr / (double)n);
  return rms > 0.0 && isfinite(rms) ? kVcycleRms / rms : 1.0;
}

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
__global__ __launch_bounds__(kBlock) void k_cg_init(Dims d, const float* __restrict__ ax,
                                                     const float* __restrict__ ay,
                                                     const float* __restrict__ az,
                                                     const float* __restrict__ b,
                                                     const double* __restrict__ x, float* __restrict__ r,
                                                     double* partials) {
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (c < (long)d.cells()) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<float> fw(d, ax, ay, az, i, j, k);
    const bool act = fw.diag() > 0.0f;
    double bc = act ? (double)b[c] : 0.0;
    double rc = true_residual_at(d, ax, ay, az, b, x, i, j, k, c);
    r[c] = (float)rc;
    v[0] = bc * bc;
    v[1] = rc * rc;
    v[2] = rc;
    v[3] = act ? 1.0 : 0.0;
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
    sc->zmu = 0.0;
    tot[1] = rr;
    sc->bb = tot[0];
    sc->rr = tot[1];
    sc->true_rr = tot[1];
    sc->tol2bb = tol * tol * tot[0];
    sc->iters = 0;
    sc->checks = 0;
    sc->first = 1;
    sc->maxit = maxit;
    sc->nonfinite = !isfinite(tot[1]);
    sc->converged = (tot[0] == 0.0) || (tot[1] <= sc->tol2bb);
    sc->done = sc->converged || sc->nonfinite || maxit <= 0;
    sc->rho = 0.0;
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

__global__ __launch_bounds__(kFinBlock) void k_fin_pq(int nb, const double* partials, CGScalars* sc) {
  if (sc->done) return;
  double tot[1];
  finish_partials<1>(partials, nb, tot);
  if (threadIdx.x == 0) {
    sc->alpha = tot[0] != 0.0 ? sc->rho / tot[0] : 0.0;
    sc->first = 0;
  }
}

// x += alpha p (FP64); r -= alpha q; partials of r . r.
__global__ __launch_bounds__(kBlock) void k_cg_update(long n, double* __restrict__ x, float* __restrict__ r,
                                                       const float* __restrict__ p,
                                                       const float* __restrict__ q, const CGScalars* sc,
                                                       double* partials) {
  if (sc->done) return;
  const double a = sc->alpha;
  const float af = (float)a;
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double v[1] = {0.0};
  if (c < n) {
    x[c] += a * (double)p[c];
    float rc = r[c] - af * q[c];
    r[c] = rc;
    v[0] = (double)rc * rc;
  }
  block_partials<1>(v, partials);
}

__global__ __launch_bounds__(kFinBlock) void k_fin_rr(int nb, const double* partials, CGScalars* sc, long ncells) {
  if (sc->done) return;
  double tot[1];
  finish_partials<1>(partials, nb, tot);
  if (threadIdx.x == 0) {
    sc->rr = tot[0];
    sc->iters += 1;
    sc->vscale = vscale_of(tot[0], ncells);
    if (!isfinite(tot[0])) sc->nonfinite = 1;
    if (tot[0] <= sc->tol2bb || sc->iters >= sc->maxit || sc->nonfinite) sc->done = 1;
  }
}

// True residual from the FP64 iterate, once the recursive residual has
// converged (both kernels do nothing while CG is still iterating, so the check
// can be enqueued behind every batch of iterations).  With `allow`, a residual
// that misses the tolerance replaces r and CG restarts (k_fin_true sets
// done = 0, first = 1).
__device__ inline bool may_replace(const CGScalars* sc, int allow) {
  return allow && !sc->nonfinite && sc->iters < sc->maxit && !(sc->bb == 0.0);
}

__global__ __launch_bounds__(kBlock) void k_cg_true_residual(Dims d, const float* __restrict__ ax,
                                                              const float* __restrict__ ay,
                                                              const float* __restrict__ az,
                                                              const float* __restrict__ b,
                                                              const double* __restrict__ x, float* __restrict__ r,
                                                              int allow, const CGScalars* sc, double* partials) {
  if (!sc->done) return;
  const bool rep = may_replace(sc, allow);
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (c < (long)d.cells()) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<float> fw(d, ax, ay, az, i, j, k);
    double rc = true_residual_at(d, ax, ay, az, b, x, i, j, k, c);
    v[0] = rc * rc;
    v[1] = rc;
    v[2] = fw.diag() > 0.0f ? 1.0 : 0.0;
    if (rep) r[c] = (float)rc;
  }
  block_partials<3>(v, partials);
}

__global__ __launch_bounds__(kFinBlock) void k_fin_true(int nb, const double* partials, CGScalars* sc, int allow,
                                                         long ncells, int project) {
  if (!sc->done) return;
  const bool rep = may_replace(sc, allow);
  double tot[3];
  finish_partials<3>(partials, nb, tot);
  if (threadIdx.x == 0) {
    sc->checks += 1;
    tot[0] = projected_rr(tot[0], tot[1], tot[2], project);
    sc->mu = project && tot[2] > 0.0 ? tot[1] / tot[2] : 0.0;
    sc->true_rr = tot[0];
    if (!isfinite(tot[0])) sc->nonfinite = 1;
    sc->converged = !sc->nonfinite && (sc->bb == 0.0 || tot[0] <= sc->tol2bb);
    if (rep && !sc->converged && !sc->nonfinite) {
      sc->rr = tot[0];
      sc->vscale = vscale_of(tot[0], ncells);
      sc->first = 1;
      sc->done = 0;
    }
  }
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

// rho = r . z and the flexible (Polak-Ribiere) direction coefficient
// beta = r_new . (z_new - z_old) / rho_old: the rounding of the FP16 / BF16
// V-cycle makes the preconditioner slightly non-linear, which this form
// tolerates; for an exactly linear preconditioner r_new . z_old = 0 and it
// reduces to the Fletcher-Reeves ratio.  On singular systems z is used minus
// its mean over active cells (k_cg_dir_apply subtracts zmu), and the dots are
// those of the projected vectors: r . (z - mu) = r . z - mu sum(r).
// Partials: r.z_new, r.z_old, sum(z_new), sum(r).
__global__ __launch_bounds__(kFinBlock) void k_fin_rz(int nb, const double* partials, CGScalars* sc, int project) {
  if (sc->done) return;
  double tot[4];
  finish_partials<4>(partials, nb, tot);
  if (threadIdx.x == 0) {
    const double mu = project && sc->nact > 0.0 ? tot[2] / sc->nact : 0.0;
    const double rz = tot[0] - mu * tot[3];
    if (sc->first) {
      sc->rho = rz;
    } else {
      const double rzo = tot[1] - sc->zmu * tot[3];
      sc->beta = sc->rho != 0.0 ? (rz - rzo) / sc->rho : 0.0;
      sc->rho = rz;
    }
    sc->zmu = mu;
  }
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
  auto z1 = [&](long t) { return kOmega * ld(invd, t) * (s0 * ld(r, t)); };
  float rc = s0 * ld(r, c);
  float z1c = kOmega * idc * rc;
  float Az = apply_A(d, fw, i, j, k, c, z1c, z1);
  z2[c] = cvt<Z>(z1c + kOmega * idc * (rc - Az));
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
  zout[c] = cvt<Z>(zc + kOmega * ld(invd, c) * (s0 * ld(r, c) - Az));
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
    float zo = (zc + kOmega * idc * (s0 * rraw - Az)) * inv;
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
// Values beyond the domain are 0, as in apply_A.
// ---------------------------------------------------------------------------

// Tile shapes: the finest level uses long x rows (efficient halo reuse), the
// coarse levels small cubes (their launches are latency-bound: less serial
// work per thread and more workgroups).
template <int TX_, int TY_, int TZ_>
struct TileShape {
  static constexpr int TX = TX_, TY = TY_, TZ = TZ_;
};
using FineTile = TileShape<32, 8, 8>;
using CoarseTile = TileShape<8, 8, 8>;
constexpr int kTileThreads = 512;   // 8 waves per tile: more loads in flight per CU
// Loops over a region have a compile-time trip count, so they unroll fully
// and every thread issues all of its loads before the first one is used.
constexpr int trips(int n) { return (n + kTileThreads - 1) / kTileThreads; }
template <class S, int H>
struct Halo {
  static constexpr int X = S::TX + 2 * H, Y = S::TY + 2 * H, Z = S::TZ + 2 * H, N = X * Y * Z;
};

template <class S>
__host__ __device__ inline int tiles_of(const Dims& d) {
  return ((d.nx + S::TX - 1) / S::TX) * ((d.ny + S::TY - 1) / S::TY) * ((d.nz + S::TZ - 1) / S::TZ);
}

template <class S>
__device__ inline void tile_origin(const Dims& d, int& i0, int& j0, int& k0) {
  const int tx = (d.nx + S::TX - 1) / S::TX, ty = (d.ny + S::TY - 1) / S::TY;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  i0 = (b % tx) * S::TX;
  j0 = ((b / tx) % ty) * S::TY;
  k0 = (b / (tx * ty)) * S::TZ;
}

__device__ inline bool in_dom(const Dims& d, int i, int j, int k) {
  return i >= 0 && j >= 0 && k >= 0 && i < d.nx && j < d.ny && k < d.nz;
}

// sum over the 6 faces of w_f (v[q] - v[nb]) for a cell at local index q of a
// halo region with row length X and plane size XY (neighbours beyond the
// domain hold 0 in v, the Dirichlet / closed convention of apply_A)
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

// Each phase first issues every load of the thread's cells (out-of-domain
// cells load element 0, which always exists, and are masked afterwards), then
// computes: a thread keeps all its loads in flight at once.
struct RegionCell {
  int q, i, j, k;
  bool ok;   // q inside the region and (i, j, k) inside the domain
};

template <class S, int H>
__device__ inline RegionCell region_cell(const Dims& d, int i0, int j0, int k0, int u) {
  using R = Halo<S, H>;
  RegionCell rc;
  rc.q = threadIdx.x + u * kTileThreads;
  const int q = rc.q < R::N ? rc.q : 0;
  const int li = q % R::X, lj = (q / R::X) % R::Y, lk = q / (R::X * R::Y);
  rc.i = i0 + li - H;
  rc.j = j0 + lj - H;
  rc.k = k0 + lk - H;
  rc.ok = rc.q < R::N && in_dom(d, rc.i, rc.j, rc.k);
  if (!rc.ok) rc.i = rc.j = rc.k = 0;
  return rc;
}

// local index in the +2 region of a cell at local index q of the +1 region
template <class S>
__device__ inline int up1to2(int q) {
  using H1 = Halo<S, 1>;
  using H2 = Halo<S, 2>;
  const int li = q % H1::X, lj = (q / H1::X) % H1::Y, lk = q / (H1::X * H1::Y);
  return (li + 1) + H2::X * ((lj + 1) + H2::Y * (lk + 1));
}

// PRE: issue the loads of all three phases before the first one computes (one
// memory latency per launch instead of three; for the small coarse levels,
// whose launches are latency-bound and few tiles wide).  Without PRE each
// phase loads what it needs, which keeps registers low for the finest level.
template <class S, typename A, typename R, typename Z, typename RC, bool PRE>
__global__ __launch_bounds__(kTileThreads) void k_mg_down(Dims d, Dims cd, const A* __restrict__ ax,
                                                          const A* __restrict__ ay, const A* __restrict__ az,
                                                          const A* __restrict__ invd, const R* __restrict__ r,
                                                          Z* __restrict__ z2out, RC* __restrict__ rc,
                                                          const CGScalars* sc, int lvl0) {
  if (sc->done) return;
  using H2 = Halo<S, 2>;
  using H1 = Halo<S, 1>;
  __shared__ float z1s[H2::N];
  __shared__ float rs[H1::N];
  __shared__ float z2s[H1::N];
  const float s0 = level_scale(sc, lvl0);
  int i0, j0, k0;
  tile_origin<S>(d, i0, j0, k0);
  constexpr int T1 = trips(H2::N), T2 = trips(H1::N);
  RegionCell c1[T1], c2[T2];
  float id1[T1], rv1[T1], id2[T2], rv2[T2];
  Faces<A> fw2[T2], fw3[8];
  // restriction: the tile's (S::TX/2) x (S::TY/2) x (S::TZ/2) coarse cells, one per thread
  const int t = threadIdx.x;
  const int ci = t % (S::TX / 2), cj = (t / (S::TX / 2)) % (S::TY / 2), ck = t / ((S::TX / 2) * (S::TY / 2));
  const int I = i0 / 2 + ci, J = j0 / 2 + cj, K = k0 / 2 + ck;
  const bool rok = t < (S::TX / 2) * (S::TY / 2) * (S::TZ / 2) && I < cd.nx && J < cd.ny && K < cd.nz;
  auto load2 = [&]() {
#pragma unroll
    for (int u = 0; u < T2; ++u) {
      c2[u] = region_cell<S, 1>(d, i0, j0, k0, u);
      const long c = d.c(c2[u].i, c2[u].j, c2[u].k);
      fw2[u] = Faces<A>(d, ax, ay, az, c2[u].i, c2[u].j, c2[u].k);
      id2[u] = ld(invd, c);
      rv2[u] = ld(r, c);
    }
  };
  auto load3 = [&]() {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = rok ? 2 * I + (b & 1) : 0, j = rok ? 2 * J + ((b >> 1) & 1) : 0, k = rok ? 2 * K + (b >> 2) : 0;
      fw3[b] = Faces<A>(d, ax, ay, az, i, j, k);
    }
  };
#pragma unroll
  for (int u = 0; u < T1; ++u) {
    c1[u] = region_cell<S, 2>(d, i0, j0, k0, u);
    const long c = d.c(c1[u].i, c1[u].j, c1[u].k);
    id1[u] = ld(invd, c);
    rv1[u] = ld(r, c);
  }
  if (PRE) {
    load2();
    load3();
  }
#pragma unroll
  for (int u = 0; u < T1; ++u)
    if (c1[u].q < H2::N) z1s[c1[u].q] = c1[u].ok ? kOmega * id1[u] * (s0 * rv1[u]) : 0.0f;
  __syncthreads();
  if (!PRE) load2();
#pragma unroll
  for (int u = 0; u < T2; ++u) {
    const int q = c2[u].q;
    if (q >= H1::N) continue;
    float z2 = 0.0f, rr = 0.0f;
    if (c2[u].ok) {
      const int q2 = up1to2<S>(q);
      rr = s0 * rv2[u];
      const Z zs = cvt<Z>(z1s[q2] + kOmega * id2[u] * (rr - apply_local(fw2[u], z1s, q2, H2::X, H2::X * H2::Y)));
      z2 = ld(&zs, 0);
      const int li = q % H1::X, lj = (q / H1::X) % H1::Y, lk = q / (H1::X * H1::Y);
      if (li >= 1 && li <= S::TX && lj >= 1 && lj <= S::TY && lk >= 1 && lk <= S::TZ)
        z2out[d.c(c2[u].i, c2[u].j, c2[u].k)] = zs;
    }
    z2s[q] = z2;
    rs[q] = rr;
  }
  __syncthreads();
  if (!PRE) load3();
  if (rok) {
    float s = 0.0f;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int li = 2 * ci + (b & 1), lj = 2 * cj + ((b >> 1) & 1), lk = 2 * ck + (b >> 2);
      const int q1 = (li + 1) + H1::X * ((lj + 1) + H1::Y * (lk + 1));
      s += rs[q1] - apply_local(fw3[b], z2s, q1, H1::X, H1::X * H1::Y);
    }
    rc[cd.c(I, J, K)] = cvt<RC>(0.125f * s);
  }
}

template <class S, typename A, typename R, typename Z, typename E, typename O, bool LVL0, bool PRE>
__global__ __launch_bounds__(kTileThreads) void k_mg_up(Dims d, Dims cd, const A* __restrict__ ax,
                                                        const A* __restrict__ ay, const A* __restrict__ az,
                                                        const A* __restrict__ invd, const R* __restrict__ r,
                                                        const Z* __restrict__ z2, const E* __restrict__ e,
                                                        O* __restrict__ zout, const CGScalars* sc, double* partials) {
  if (sc->done) return;
  using H2 = Halo<S, 2>;
  using H1 = Halo<S, 1>;
  __shared__ float zp[H2::N];
  __shared__ float z3s[H1::N];
  const float s0 = LVL0 ? (float)sc->vscale : 1.0f;
  const float inv = LVL0 ? (float)(1.0 / sc->vscale) : 1.0f;
  const bool first = sc->first;
  int i0, j0, k0;
  tile_origin<S>(d, i0, j0, k0);
  constexpr int T1 = trips(H2::N), T2 = trips(H1::N), T3 = trips(S::TX * S::TY * S::TZ);
  RegionCell c1[T1], c2[T2];
  float zv[T1], ev[T1], id2[T2], rv2[T2], id3[T3], rv3[T3], zold[T3];
  Faces<A> fw2[T2], fw3[T3];
  bool ok3[T3];
  int cl3[T3];
  auto load2 = [&]() {
#pragma unroll
    for (int u = 0; u < T2; ++u) {
      c2[u] = region_cell<S, 1>(d, i0, j0, k0, u);
      const long c = d.c(c2[u].i, c2[u].j, c2[u].k);
      fw2[u] = Faces<A>(d, ax, ay, az, c2[u].i, c2[u].j, c2[u].k);
      id2[u] = ld(invd, c);
      rv2[u] = ld(r, c);
    }
  };
  auto load3 = [&]() {
#pragma unroll
    for (int u = 0; u < T3; ++u) {
      const int q = threadIdx.x + u * kTileThreads;
      const int li = q % S::TX, lj = (q / S::TX) % S::TY, lk = q / (S::TX * S::TY);
      int i = i0 + li, j = j0 + lj, k = k0 + lk;
      ok3[u] = in_dom(d, i, j, k);
      if (!ok3[u]) i = j = k = 0;
      cl3[u] = (li + 1) + H1::X * ((lj + 1) + H1::Y * (lk + 1));
      const long c = d.c(i, j, k);
      fw3[u] = Faces<A>(d, ax, ay, az, i, j, k);
      id3[u] = ld(invd, c);
      rv3[u] = ld(r, c);
      zold[u] = (LVL0 && !first) ? ld(zout, c) : 0.0f;
    }
  };
#pragma unroll
  for (int u = 0; u < T1; ++u) {
    c1[u] = region_cell<S, 2>(d, i0, j0, k0, u);
    zv[u] = ld(z2, d.c(c1[u].i, c1[u].j, c1[u].k));
    ev[u] = ld(e, cd.c(c1[u].i >> 1, c1[u].j >> 1, c1[u].k >> 1));
  }
  if (PRE) {
    load2();
    load3();
  }
#pragma unroll
  for (int u = 0; u < T1; ++u)
    if (c1[u].q < H2::N) zp[c1[u].q] = c1[u].ok ? zv[u] + 8.0f * ev[u] : 0.0f;
  __syncthreads();
  if (!PRE) load2();
#pragma unroll
  for (int u = 0; u < T2; ++u) {
    const int q = c2[u].q;
    if (q >= H1::N) continue;
    float v = 0.0f;
    if (c2[u].ok) {
      const int q2 = up1to2<S>(q);
      v = zp[q2] + kOmega * id2[u] * (s0 * rv2[u] - apply_local(fw2[u], zp, q2, H2::X, H2::X * H2::Y));
    }
    z3s[q] = v;
  }
  __syncthreads();
  if (!PRE) load3();
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < T3; ++u) {
    if (!ok3[u]) continue;
    const int q = threadIdx.x + u * kTileThreads;
    const int li = q % S::TX, lj = (q / S::TX) % S::TY, lk = q / (S::TX * S::TY);
    const long c = d.c(i0 + li, j0 + lj, k0 + lk);
    const int q1 = cl3[u];
    float zo = (z3s[q1] + kOmega * id3[u] * (s0 * rv3[u] - apply_local(fw3[u], z3s, q1, H1::X, H1::X * H1::Y))) * inv;
    if (LVL0 && !(id3[u] > 0.0f)) zo = 0.0f;   // inactive cell: no unknown
    if (LVL0 && !first) acc[1] += (double)rv3[u] * (double)zold[u];   // r_new . z_old
    zout[c] = cvt<O>(zo);
    if (LVL0) {
      acc[0] += (double)rv3[u] * (double)zo;
      acc[2] += (double)zo;
      acc[3] += (double)rv3[u];
    }
  }
  if (LVL0) block_partials<4, kTileThreads>(acc, partials);
}

// CG direction and operator on a tile: p = (z - zmu) + beta p_old on the tile
// + 1 cell (in LDS; written out on the tile), q = A p and p.q partials on the
// tile.  Same arithmetic as k_cg_dir_apply with one load of z and p_old per
// cell and halo.
template <class S>
__global__ __launch_bounds__(kTileThreads) void k_cg_dir_apply_tile(Dims d, const float* __restrict__ ax,
                                                                    const float* __restrict__ ay,
                                                                    const float* __restrict__ az,
                                                                    const float* __restrict__ z,
                                                                    const float* __restrict__ pold,
                                                                    float* __restrict__ pnew, float* __restrict__ q,
                                                                    const CGScalars* sc, double* partials) {
  if (sc->done) return;
  using H1 = Halo<S, 1>;
  __shared__ float ps[H1::N];
  const bool first = sc->first;
  const float beta = (float)sc->beta;
  const float zmu = (float)sc->zmu;
  int i0, j0, k0;
  tile_origin<S>(d, i0, j0, k0);
  {
    constexpr int T = trips(H1::N);
    RegionCell cell[T];
    float zv[T], pv[T];
#pragma unroll
    for (int u = 0; u < T; ++u) {
      cell[u] = region_cell<S, 1>(d, i0, j0, k0, u);
      const long c = d.c(cell[u].i, cell[u].j, cell[u].k);
      zv[u] = z[c];
      pv[u] = first ? 0.0f : pold[c];
    }
#pragma unroll
    for (int u = 0; u < T; ++u) {
      const int qq = cell[u].q;
      if (qq >= H1::N) continue;
      float p = 0.0f;
      if (cell[u].ok) {
        p = first ? zv[u] - zmu : (zv[u] - zmu) + beta * pv[u];
        const int li = qq % H1::X, lj = (qq / H1::X) % H1::Y, lk = qq / (H1::X * H1::Y);
        if (li >= 1 && li <= S::TX && lj >= 1 && lj <= S::TY && lk >= 1 && lk <= S::TZ)
          pnew[d.c(cell[u].i, cell[u].j, cell[u].k)] = p;
      }
      ps[qq] = p;
    }
  }
  __syncthreads();
  double acc[1] = {0.0};
  {
    constexpr int T = trips(S::TX * S::TY * S::TZ);
    bool ok[T];
    int cl[T];
    long cc[T];
    Faces<float> fw[T];
#pragma unroll
    for (int u = 0; u < T; ++u) {
      const int qq = threadIdx.x + u * kTileThreads;
      const int li = qq % S::TX, lj = (qq / S::TX) % S::TY, lk = qq / (S::TX * S::TY);
      int i = i0 + li, j = j0 + lj, k = k0 + lk;
      ok[u] = in_dom(d, i, j, k);
      if (!ok[u]) i = j = k = 0;
      cl[u] = (li + 1) + H1::X * ((lj + 1) + H1::Y * (lk + 1));
      cc[u] = d.c(i, j, k);
      fw[u] = Faces<float>(d, ax, ay, az, i, j, k);
    }
#pragma unroll
    for (int u = 0; u < T; ++u) {
      if (!ok[u]) continue;
      const float qc = apply_local(fw[u], ps, cl[u], H1::X, H1::X * H1::Y);
      q[cc[u]] = qc;
      acc[0] += (double)ps[cl[u]] * qc;
    }
  }
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
};

// Coefficients of one level, from LDS (P = float) or from memory (P = storage type).
template <typename P>
struct Coef {
  const P* ax;
  const P* ay;
  const P* az;
  const P* invd;
};

// z = two damped-Jacobi sweeps from 0 (t holds the first); then the restricted
// residual mean over the 8 children of (r - A z) into rc.
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
  if (B.coff[L - 1] >= 0)
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

template <typename T>
__global__ void k_cast(long n, const float* __restrict__ src, T* __restrict__ dst, float cap) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = cvt<T>(fminf(src[i], cap));
}

static inline unsigned nblocks(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------

template <typename T>
static void vcycle(const Solver& S, const float* r0, float* z0, hipStream_t st) {
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
  if (G == 0) {
    NF_LAUNCH(S.prof, SIM_K_MG_COARSE, (k_mg_bottom<T, float, float>), dim3(1), dim3(bthreads), lds, st, B, r0, z0, sc, 1);
    hipLaunchKernelGGL(k_scale_dot<T>, dim3(nblocks(n0)), dim3(kBlock), 0, st, n0, ID(0), r0, z0, sc, S.partials);
    hipLaunchKernelGGL(k_fin_rz, dim3(1), dim3(kFinBlock), 0, st, (int)nblocks(n0), S.partials, sc, S.project);
    return;
  }
  if (S.fused) {
    auto tiles = [](const Dims& d, bool fine) {
      return (unsigned)(fine ? tiles_of<FineTile>(d) : tiles_of<CoarseTile>(d));
    };
    for (int l = 0; l < G; ++l) {
      const Dims& d = S.lev[l].d;
      const Dims& cd = S.lev[l + 1].d;
      T* rc = (T*)S.lev[l + 1].r;
      if (l == 0) {
        NF_LAUNCH(S.prof, SIM_K_MG_DOWN, (k_mg_down<FineTile, T, float, float, T, false>), dim3(tiles(d, true)), dim3(kTileThreads), 0, st,
                  d, cd, A(0), Ay(0), Az(0), ID(0), r0, (float*)S.lev[0].ta, rc, sc, 1);
      } else {
        hipLaunchKernelGGL((k_mg_down<CoarseTile, T, T, T, T, true>), dim3(tiles(d, false)), dim3(kTileThreads), 0, st, d, cd, A(l), Ay(l), Az(l),
                           ID(l), (const T*)S.lev[l].r, (T*)S.lev[l].ta, rc, sc, 0);
      }
    }
    NF_LAUNCH(S.prof, SIM_K_MG_COARSE, (k_mg_bottom<T, T, T>), dim3(1), dim3(bthreads), lds, st, B, (const T*)S.lev[G].r,
                                (T*)S.lev[G].z, sc, 0);
    for (int l = G - 1; l >= 0; --l) {
      const Dims& d = S.lev[l].d;
      const Dims& cd = S.lev[l + 1].d;
      const T* e = (const T*)S.lev[l + 1].z;
      if (l == 0) {
        NF_LAUNCH(S.prof, SIM_K_MG_UP, (k_mg_up<FineTile, T, float, float, T, float, true, false>), dim3(tiles(d, true)), dim3(kTileThreads),
                  0, st, d, cd, A(0), Ay(0), Az(0), ID(0), r0, (const float*)S.lev[0].ta, e, z0, sc, S.partials);
        hipLaunchKernelGGL(k_fin_rz, dim3(1), dim3(kFinBlock), 0, st, (int)tiles(d, true), S.partials, sc, S.project);
      } else {
        hipLaunchKernelGGL((k_mg_up<CoarseTile, T, T, T, T, T, false, true>), dim3(tiles(d, false)), dim3(kTileThreads), 0, st, d, cd, A(l), Ay(l),
                           Az(l), ID(l), (const T*)S.lev[l].r, (const T*)S.lev[l].ta, e, (T*)S.lev[l].z, sc,
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
  NF_LAUNCH(S.prof, SIM_K_MG_COARSE, (k_mg_bottom<T, T, T>), dim3(1), dim3(bthreads), lds, st, B, (const T*)S.lev[G].r,
                              (T*)S.lev[G].z, sc, 0);
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

static void vcycle_dispatch(const Solver& S, const float* r0, float* z0, hipStream_t st) {
  if (S.precision == SIM_MIXED_FP16)
    vcycle<__half>(S, r0, z0, st);
  else if (S.precision == SIM_MIXED_BF16)
    vcycle<__hip_bfloat16>(S, r0, z0, st);
  else
    vcycle<float>(S, r0, z0, st);
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

// Multigrid copies of the fine fractions and inverse diagonals.
void solver_setup_levels(Solver& S, const float* fine_alpha, hipStream_t st) {
  const Dims& d0 = S.lev[0].d;
  const float* fx = fine_alpha;
  const float* fy = fx + d0.nfx();
  const float* fz = fy + d0.nfy();
  S.ax = fx;
  S.ay = fy;
  S.az = fz;
  if (S.precision == SIM_FP32) {
    S.lev[0].a[0] = (void*)fx;
    S.lev[0].a[1] = (void*)fy;
    S.lev[0].a[2] = (void*)fz;
    launch_invdiag(d0, fx, fy, fz, (float*)S.lev[0].invd, st);
    for (int l = 1; l < S.nlev; ++l) {
      const Dims& fd = S.lev[l - 1].d;
      const Dims& cd = S.lev[l].d;
      launch_coarsen_alpha(fd, cd, (const float*)S.lev[l - 1].a[0], (const float*)S.lev[l - 1].a[1],
                           (const float*)S.lev[l - 1].a[2], (float*)S.lev[l].a[0], (float*)S.lev[l].a[1],
                           (float*)S.lev[l].a[2], st);
      launch_invdiag(cd, (const float*)S.lev[l].a[0], (const float*)S.lev[l].a[1], (const float*)S.lev[l].a[2],
                     (float*)S.lev[l].invd, st);
    }
    return;
  }
  // mixed: build each level in FP32 scratch, then store it in T
  for (int l = 0; l < S.nlev; ++l) {
    // FP16: level 0 only needs 1/diag to stay finite (its iterates are FP32);
    // coarser levels store their iterates in FP16 and keep the tighter cap
    const float cap = S.precision != SIM_MIXED_FP16 ? 3e38f : (l == 0 ? kHalfMax : kHalfInvDiagMax);
    const Dims& d = S.lev[l].d;
    const float *lx, *ly, *lz;
    if (l == 0) {
      lx = fx;
      ly = fy;
      lz = fz;
    } else {
      const Dims& fd = S.lev[l - 1].d;
      float* cx = S.scratch_a + S.scratch_off[l];
      float* cy = cx + d.nfx();
      float* cz = cy + d.nfy();
      const float *px, *py, *pz;
      if (l == 1) {
        px = fx;
        py = fy;
        pz = fz;
      } else {
        px = S.scratch_a + S.scratch_off[l - 1];
        py = px + fd.nfx();
        pz = py + fd.nfy();
      }
      launch_coarsen_alpha(fd, d, px, py, pz, cx, cy, cz, st);
      lx = cx;
      ly = cy;
      lz = cz;
    }
    launch_invdiag(d, lx, ly, lz, S.scratch_inv, st);
    if (S.precision == SIM_MIXED_FP16)
      cast_level<__half>(d, lx, ly, lz, S.scratch_inv, S.lev[l], cap, st);
    else
      cast_level<__hip_bfloat16>(d, lx, ly, lz, S.scratch_inv, S.lev[l], cap, st);
  }
}

static void enqueue_iterations(Solver& S, double* x, int count, hipStream_t st) {
  const Dims& d = S.lev[0].d;
  const long n = (long)d.cells();
  for (int c = 0; c < count; ++c) {
    float* pold = S.pcur ? S.p1 : S.p0;
    float* pnew = S.pcur ? S.p0 : S.p1;
    const int nb = (int)nblocks(n);
    if (S.fused) {
      const int nt = tiles_of<FineTile>(d);
      NF_LAUNCH(S.prof, SIM_K_CG_APPLY, k_cg_dir_apply_tile<FineTile>, dim3(nt), dim3(kTileThreads), 0, st, d, S.ax, S.ay,
                S.az, S.z, pold, pnew, S.q, S.sc, S.partials);
      hipLaunchKernelGGL(k_fin_pq, dim3(1), dim3(kFinBlock), 0, st, nt, S.partials, S.sc);
    } else {
      NF_LAUNCH(S.prof, SIM_K_CG_APPLY, k_cg_dir_apply, dim3(nb), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, S.z, pold,
                                  pnew, S.q, S.sc, S.partials);
      hipLaunchKernelGGL(k_fin_pq, dim3(1), dim3(kFinBlock), 0, st, nb, S.partials, S.sc);
    }
    NF_LAUNCH(S.prof, SIM_K_CG_UPDATE, k_cg_update, dim3(nb), dim3(kBlock), 0, st, n, x, S.r, pnew, S.q, S.sc,
              S.partials);
    hipLaunchKernelGGL(k_fin_rr, dim3(1), dim3(kFinBlock), 0, st, nb, S.partials, S.sc, n);
    vcycle_dispatch(S, S.r, S.z, st);
    S.pcur ^= 1;
  }
}

// Capture two iterations (starting with p0 as the current direction) into a
// graph; replaying it leaves the direction parity unchanged.
static bool capture_pair(Solver& S, double* x) {
  if (S.iter_exec) return true;
  if (!S.cap_stream && hipStreamCreateWithFlags(&S.cap_stream, hipStreamNonBlocking) != hipSuccess) return false;
  if (hipStreamBeginCapture(S.cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return false;
  const int saved = S.pcur;
  S.pcur = 0;
  Profiler* prof = S.prof;
  S.prof = nullptr;
  enqueue_iterations(S, x, 2, S.cap_stream);
  S.prof = prof;
  S.pcur = saved;
  if (hipStreamEndCapture(S.cap_stream, &S.iter_graph) != hipSuccess) return false;
  if (hipGraphInstantiate(&S.iter_exec, S.iter_graph, nullptr, nullptr, 0) != hipSuccess) {
    S.iter_exec = nullptr;
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
    for (int q = 0; q < pairs; ++q) (void)hipGraphLaunch(S.iter_exec, st);
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
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess) return;
  S.lds_bytes = (size_t)v;
}

void solver_release(Solver& S) {
  if (S.iter_exec) (void)hipGraphExecDestroy(S.iter_exec);
  if (S.iter_graph) (void)hipGraphDestroy(S.iter_graph);
  if (S.cap_stream) (void)hipStreamDestroy(S.cap_stream);
  S.iter_exec = nullptr;
  S.iter_graph = nullptr;
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

int solver_solve(Solver& S, SolveKind kind, const float* b, float* xio, double tol, int maxit, sim_stats* stats,
                 hipStream_t st) {
  const Dims& d = S.lev[0].d;
  const long n = (long)d.cells();
  CGScalars* sc = S.sc;
  double* x = S.x;
  hipLaunchKernelGGL(k_x_load, dim3(nblocks(n)), dim3(kBlock), 0, st, n, xio, x);
  NF_LAUNCH(S.prof, SIM_K_CG_INIT, k_cg_init, dim3(nblocks(n)), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, b, x, S.r,
                              S.partials);
  hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(kFinBlock), 0, st, (int)nblocks(n), S.partials, sc, tol, maxit, n,
                     S.project);
  if (S.project)
    hipLaunchKernelGGL(k_sub_mean, dim3(nblocks(n)), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, S.r, sc);
  vcycle_dispatch(S, S.r, S.z, st);
  S.pcur = 0;
  // Each round enqueues a batch of iterations and the (conditional) true-
  // residual check behind it, then synchronises once.  The first batch is
  // sized from the previous solve of this handle, so a typical solve needs a
  // single round; iterations enqueued after convergence exit at once on the
  // device.  Every round runs iterations or uses up one of a bounded number of
  // restarts, and the round count is capped, so the loop terminates.
  const int kMaxRestarts = 8;
  int batch = S.last_iters[kind] > 0 ? S.last_iters[kind] : 2;
  const int chunk = S.check_every > 0 ? S.check_every : 2;
  int restarts = 0, checks_seen = 0, rounds = 0;
  for (;;) {
    const int allow = restarts < kMaxRestarts ? 1 : 0;
    (void)cg_iterations(S, x, batch, st);
    NF_LAUNCH(S.prof, SIM_K_CG_TRUE, k_cg_true_residual, dim3(nblocks(n)), dim3(kBlock), 0, st, d, S.ax, S.ay,
              S.az, b, x, S.r, allow, sc, S.partials);
    hipLaunchKernelGGL(k_fin_true, dim3(1), dim3(kFinBlock), 0, st, (int)nblocks(n), S.partials, sc, allow, n,
                       S.project);
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
    if (S.project)
      hipLaunchKernelGGL(k_sub_mean, dim3(nblocks(n)), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, S.r, sc);
    vcycle_dispatch(S, S.r, S.z, st);
  }
  S.last_iters[kind] = S.host_sc->iters;
  hipLaunchKernelGGL(k_x_store, dim3(nblocks(n)), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, x, xio);
  if (stats) {
    const CGScalars& h = *S.host_sc;
    stats->iters = h.iters;
    stats->nonfinite = h.nonfinite;
    stats->converged = h.converged && !h.nonfinite;
    stats->pad = 0;
    stats->rel_res = h.bb > 0.0 ? sqrt(h.rr / h.bb) : 0.0;
    stats->true_rel_res = h.bb > 0.0 ? sqrt(h.true_rr / h.bb) : 0.0;
  }
  return SIM_OK;
}

}  // namespace nf
