// Matrix-free multigrid-preconditioned CG for (G^T S G) x = b on the MAC grid.
//
// NeuralFluid solves the projection system of Eq. projection_matrix with a
// matrix-free geometric-multigrid-preconditioned CG (Sec. Time Performance
// Profiling: MGPCG with custom prolongation / restriction between a
// hierarchy of grids).  This solver:
//   * applies A x = sum over faces of alpha_f (x_c - x_nb) as a 7-point
//     stencil read straight from the face fractions (no stored matrix);
//   * keeps the iterate x in FP64 and the other CG vectors in FP32; every CG
//     scalar stays on the device, with FP64 dot products reduced in a fixed
//     order (per-block partials summed by the last block to finish), so a
//     solve is bitwise reproducible;
//   * stops on the recursive residual, then recomputes b - A x from the FP64
//     iterate; if that true residual misses the tolerance, the true residual
//     replaces the recursive one and CG restarts (iterative refinement);
//   * preconditions with one V-cycle: level l+1 halves each axis, coarse face
//     weight = 1/2 * sum of the 2x2 fine faces it covers, restriction = mean
//     of the 8 child residuals with prolongation = 8 x injection (together the
//     transpose pair), two damped-Jacobi sweeps (omega = 0.8) before and after
//     the correction, and 40 Jacobi sweeps on the coarsest level (<= 4096
//     cells) in one workgroup.  Every piece is a fixed linear symmetric map,
//     so the preconditioner is symmetric and plain CG applies;
//   * stores the multigrid arrays in FP32, FP16 or BF16 (template T).  The
//     V-cycle is linear, so its input is scaled to a fixed RMS and its output
//     scaled back, which keeps FP16 values in range; 1/diag is capped in FP16.
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
  i = (int)(c % d.nx);
  long t = c / d.nx;
  j = (int)(t % d.ny);
  k = (int)(t / d.ny);
}

// The 6 face weights of cell (i,j,k): lower / upper along x, y, z.
template <typename A>
struct Faces {
  float w[6];
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

__global__ void k_x_store(long n, const double* __restrict__ x, float* __restrict__ xout) {
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) xout[c] = (float)x[c];
}

// r = b - A x; partials of b.b (active cells) and r.r.
__global__ __launch_bounds__(kBlock) void k_cg_init(Dims d, const float* __restrict__ ax,
                                                     const float* __restrict__ ay,
                                                     const float* __restrict__ az,
                                                     const float* __restrict__ b,
                                                     const double* __restrict__ x, float* __restrict__ r,
                                                     double* partials) {
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (c < (long)d.cells()) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<float> fw(d, ax, ay, az, i, j, k);
    double bc = fw.diag() > 0.0f ? (double)b[c] : 0.0;
    double rc = true_residual_at(d, ax, ay, az, b, x, i, j, k, c);
    r[c] = (float)rc;
    v[0] = bc * bc;
    v[1] = rc * rc;
  }
  block_partials<2>(v, partials);
}

__global__ __launch_bounds__(kFinBlock) void k_fin_init(int nb, const double* partials, CGScalars* sc, double tol,
                                                         int maxit, long ncells) {
  double tot[2];
  finish_partials<2>(partials, nb, tot);
  if (threadIdx.x == 0) {
    sc->bb = tot[0];
    sc->rr = tot[1];
    sc->true_rr = tot[1];
    sc->tol2bb = tol * tol * tot[0];
    sc->iters = 0;
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
  long c = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  double v[1] = {0.0};
  if (c < (long)d.cells()) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<float> fw(d, ax, ay, az, i, j, k);
    auto pv = [&](long t) { return first ? z[t] : z[t] + beta * pold[t]; };
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

// True residual from the FP64 iterate.  With `allow`, a residual that misses
// the tolerance replaces r and CG restarts (k_fin_true sets done = 0, first = 1).
__device__ inline bool may_replace(const CGScalars* sc, int allow) {
  return allow && !sc->nonfinite && sc->iters < sc->maxit && !(sc->bb == 0.0);
}

__global__ __launch_bounds__(kBlock) void k_cg_true_residual(Dims d, const float* __restrict__ ax,
                                                              const float* __restrict__ ay,
                                                              const float* __restrict__ az,
                                                              const float* __restrict__ b,
                                                              const double* __restrict__ x, float* __restrict__ r,
                                                              int allow, const CGScalars* sc, double* partials) {
  const bool rep = may_replace(sc, allow);
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double v[1] = {0.0};
  if (c < (long)d.cells()) {
    int i, j, k;
    cdec(d, c, i, j, k);
    double rc = true_residual_at(d, ax, ay, az, b, x, i, j, k, c);
    v[0] = rc * rc;
    if (rep) r[c] = (float)rc;
  }
  block_partials<1>(v, partials);
}

__global__ __launch_bounds__(kFinBlock) void k_fin_true(int nb, const double* partials, CGScalars* sc, int allow,
                                                         long ncells) {
  const bool rep = may_replace(sc, allow);
  double tot[1];
  finish_partials<1>(partials, nb, tot);
  if (threadIdx.x == 0) {
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

// rho = r . z and the flexible (Polak-Ribiere) direction coefficient
// beta = r_new . (z_new - z_old) / rho_old: the rounding of the FP16 / BF16
// V-cycle makes the preconditioner slightly non-linear, which this form
// tolerates; for an exactly linear preconditioner r_new . z_old = 0 and it
// reduces to the Fletcher-Reeves ratio.
__global__ __launch_bounds__(kFinBlock) void k_fin_rz(int nb, const double* partials, CGScalars* sc) {
  if (sc->done) return;
  double tot[2];
  finish_partials<2>(partials, nb, tot);
  if (threadIdx.x == 0) {
    if (sc->first) {
      sc->rho = tot[0];
    } else {
      sc->beta = sc->rho != 0.0 ? (tot[0] - tot[1]) / sc->rho : 0.0;
      sc->rho = tot[0];
    }
  }
}

// z *= 1 / vscale (the V-cycle ran on the scaled residual); partials of r . z.
__global__ __launch_bounds__(kBlock) void k_scale_dot(long n, const float* __restrict__ r, float* __restrict__ z,
                                                       const CGScalars* sc, double* partials) {
  if (sc->done) return;
  const float inv = (float)(1.0 / sc->vscale);
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (c < n) {
    float zc = z[c] * inv;
    z[c] = zc;
    v[0] = (double)r[c] * (double)zc;
  }
  block_partials<2>(v, partials);
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
  const int cnx = cd.nx, cny = cd.ny;
  auto zp = [&](long t) {
    int ti = (int)(t % d.nx);
    long tt = t / d.nx;
    int tj = (int)(tt % d.ny), tk = (int)(tt / d.ny);
    return ld(zin, t) + 8.0f * ld(e, (ti >> 1) + (long)cnx * ((tj >> 1) + (long)cny * (tk >> 1)));
  };
  float zc = zp(c);
  float Az = apply_A(d, fw, i, j, k, c, zc, zp);
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
  double v[2] = {0.0, 0.0};
  if (c < (long)d.cells()) {
    int i, j, k;
    cdec(d, c, i, j, k);
    Faces<A> fw(d, ax, ay, az, i, j, k);
    auto zv = [&](long t) { return ld(zin, t); };
    float zc = ld(zin, c);
    float rraw = ld(r, c);
    float Az = apply_A(d, fw, i, j, k, c, zc, zv);
    float zo = (zc + kOmega * ld(invd, c) * (s0 * rraw - Az)) * inv;
    if (LVL0 && !first) v[1] = (double)rraw * (double)ld(zout, c);   // r_new . z_old
    zout[c] = cvt<O>(zo);
    v[0] = (double)rraw * (double)zo;
  }
  if (LVL0) block_partials<2>(v, partials);
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
  int off[kMaxLevels];   // LDS offset (floats) of level l's three vectors r, z, t
};

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
  {
    const int n = (int)B.d[0].cells();
    float* r0 = R_(0);
    for (int c = threadIdx.x; c < n; c += T) r0[c] = s0 * ld(rin, c);
  }
  __syncthreads();
  // down
  for (int l = 0; l < B.nl; ++l) {
    const Dims& d = B.d[l];
    const int n = (int)d.cells();
    float *r = R_(l), *z = Z_(l), *t = T_(l);
    if (l == B.nl - 1) {
      for (int c = threadIdx.x; c < n; c += T) z[c] = 0.0f;
      __syncthreads();
      float *src = z, *dst = t;
      for (int s = 0; s < kCoarseSweeps; ++s) {
        for (int c = threadIdx.x; c < n; c += T) {
          int i, j, k;
          cdec(d, c, i, j, k);
          Faces<A> fw(d, B.ax[l], B.ay[l], B.az[l], i, j, k);
          float Az = apply_A(d, fw, i, j, k, c, src[c], [&](long q) { return src[q]; });
          dst[c] = src[c] + kOmega * ld(B.invd[l], c) * (r[c] - Az);
        }
        __syncthreads();
        float* tmp = src;
        src = dst;
        dst = tmp;
      }
      if (src != z) {
        for (int c = threadIdx.x; c < n; c += T) z[c] = src[c];
        __syncthreads();
      }
      break;
    }
    for (int c = threadIdx.x; c < n; c += T) t[c] = kOmega * ld(B.invd[l], c) * r[c];
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += T) {
      int i, j, k;
      cdec(d, c, i, j, k);
      Faces<A> fw(d, B.ax[l], B.ay[l], B.az[l], i, j, k);
      float Az = apply_A(d, fw, i, j, k, c, t[c], [&](long q) { return t[q]; });
      z[c] = t[c] + kOmega * ld(B.invd[l], c) * (r[c] - Az);
    }
    __syncthreads();
    const Dims& cd = B.d[l + 1];
    float* rc = R_(l + 1);
    for (int C = threadIdx.x; C < (int)cd.cells(); C += T) {
      int I, J, K;
      cdec(cd, C, I, J, K);
      float s = 0.0f;
      for (int b = 0; b < 8; ++b) {
        int i = 2 * I + (b & 1), j = 2 * J + ((b >> 1) & 1), k = 2 * K + (b >> 2);
        int c = d.c(i, j, k);
        Faces<A> fw(d, B.ax[l], B.ay[l], B.az[l], i, j, k);
        s += r[c] - apply_A(d, fw, i, j, k, c, z[c], [&](long q) { return z[q]; });
      }
      rc[C] = 0.125f * s;
    }
    __syncthreads();
  }
  // up
  for (int l = B.nl - 2; l >= 0; --l) {
    const Dims& d = B.d[l];
    const Dims& cd = B.d[l + 1];
    const int n = (int)d.cells();
    float *r = R_(l), *z = Z_(l), *t = T_(l);
    const float* e = Z_(l + 1);
    auto zp = [&](long q) {
      int ti = (int)(q % d.nx);
      long tt = q / d.nx;
      int tj = (int)(tt % d.ny), tk = (int)(tt / d.ny);
      return z[q] + 8.0f * e[(ti >> 1) + cd.nx * ((tj >> 1) + cd.ny * (tk >> 1))];
    };
    for (int c = threadIdx.x; c < n; c += T) {
      int i, j, k;
      cdec(d, c, i, j, k);
      Faces<A> fw(d, B.ax[l], B.ay[l], B.az[l], i, j, k);
      float zc = zp(c);
      t[c] = zc + kOmega * ld(B.invd[l], c) * (r[c] - apply_A(d, fw, i, j, k, c, zc, zp));
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += T) {
      int i, j, k;
      cdec(d, c, i, j, k);
      Faces<A> fw(d, B.ax[l], B.ay[l], B.az[l], i, j, k);
      z[c] = t[c] + kOmega * ld(B.invd[l], c) * (r[c] - apply_A(d, fw, i, j, k, c, t[c], [&](long q) { return t[q]; }));
    }
    __syncthreads();
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
    off += 3 * (int)S.lev[l].d.cells();
  }
  const size_t lds = (size_t)off * sizeof(float);
  const int bthreads = S.lev[G].d.cells() >= 1024 ? 1024 : (int)((S.lev[G].d.cells() + 63) / 64 * 64);
  if (G == 0) {
    NF_TIMED(S.prof, SIM_K_MG_COARSE, st,
             hipLaunchKernelGGL((k_mg_bottom<T, float, float>), dim3(1), dim3(bthreads), lds, st, B, r0, z0, sc, 1));
    hipLaunchKernelGGL(k_scale_dot, dim3(nblocks(n0)), dim3(kBlock), 0, st, n0, r0, z0, sc, S.partials);
    hipLaunchKernelGGL(k_fin_rz, dim3(1), dim3(kFinBlock), 0, st, (int)nblocks(n0), S.partials, sc);
    return;
  }
  for (int l = 0; l < G; ++l) {
    const Dims& d = S.lev[l].d;
    const Dims& cd = S.lev[l + 1].d;
    T* ta = (T*)S.lev[l].ta;
    T* rc = (T*)S.lev[l + 1].r;
    if (l == 0) {
      NF_TIMED(S.prof, SIM_K_MG_PRE, st,
               hipLaunchKernelGGL((k_mg_pre<T, float, T>), dim3(nblocks(d.cells())), dim3(kBlock), 0, st, d, A(0),
                                  Ay(0), Az(0), ID(0), r0, ta, sc, 1));
      NF_TIMED(S.prof, SIM_K_MG_RESTRICT, st,
               hipLaunchKernelGGL((k_mg_restrict<T, float, T, T>), dim3(nblocks(cd.cells())), dim3(kBlock), 0, st, d,
                                  cd, A(0), Ay(0), Az(0), r0, (const T*)ta, rc, sc, 1));
    } else {
      const T* rl = (const T*)S.lev[l].r;
      hipLaunchKernelGGL((k_mg_pre<T, T, T>), dim3(nblocks(d.cells())), dim3(kBlock), 0, st, d, A(l), Ay(l),
                         Az(l), ID(l), rl, ta, sc, 0);
      hipLaunchKernelGGL((k_mg_restrict<T, T, T, T>), dim3(nblocks(cd.cells())), dim3(kBlock), 0, st, d, cd, A(l),
                         Ay(l), Az(l), rl, (const T*)ta, rc, sc, 0);
    }
  }
  NF_TIMED(S.prof, SIM_K_MG_COARSE, st,
           hipLaunchKernelGGL((k_mg_bottom<T, T, T>), dim3(1), dim3(bthreads), lds, st, B, (const T*)S.lev[G].r,
                              (T*)S.lev[G].z, sc, 0));
  for (int l = G - 1; l >= 0; --l) {
    const Dims& d = S.lev[l].d;
    const Dims& cd = S.lev[l + 1].d;
    const T* ta = (const T*)S.lev[l].ta;
    T* tb = (T*)S.lev[l].tb;
    const T* e = (const T*)S.lev[l + 1].z;
    if (l == 0) {
      NF_TIMED(S.prof, SIM_K_MG_POST1, st,
               hipLaunchKernelGGL((k_mg_post1<T, float, T, T>), dim3(nblocks(d.cells())), dim3(kBlock), 0, st, d, cd,
                                  A(0), Ay(0), Az(0), ID(0), r0, ta, e, tb, sc, 1));
      NF_TIMED(S.prof, SIM_K_MG_POST2, st,
               hipLaunchKernelGGL((k_mg_post2<T, float, T, float, true>), dim3(nblocks(d.cells())), dim3(kBlock), 0, st,
                                  d, A(0), Ay(0), Az(0), ID(0), r0, (const T*)tb, z0, sc, S.partials));
      hipLaunchKernelGGL(k_fin_rz, dim3(1), dim3(kFinBlock), 0, st, (int)nblocks(d.cells()), S.partials, sc);
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
  const float cap = S.precision == SIM_MIXED_FP16 ? kHalfInvDiagMax : 3e38f;
  for (int l = 0; l < S.nlev; ++l) {
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

static void cg_iterations(Solver& S, double* x, int count, hipStream_t st) {
  const Dims& d = S.lev[0].d;
  const long n = (long)d.cells();
  for (int c = 0; c < count; ++c) {
    float* pold = S.pcur ? S.p1 : S.p0;
    float* pnew = S.pcur ? S.p0 : S.p1;
    const int nb = (int)nblocks(n);
    NF_TIMED(S.prof, SIM_K_CG_APPLY, st,
             hipLaunchKernelGGL(k_cg_dir_apply, dim3(nb), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, S.z, pold,
                                pnew, S.q, S.sc, S.partials));
    hipLaunchKernelGGL(k_fin_pq, dim3(1), dim3(kFinBlock), 0, st, nb, S.partials, S.sc);
    NF_TIMED(S.prof, SIM_K_CG_UPDATE, st,
             hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(kBlock), 0, st, n, x, S.r, pnew, S.q, S.sc,
                                S.partials));
    hipLaunchKernelGGL(k_fin_rr, dim3(1), dim3(kFinBlock), 0, st, nb, S.partials, S.sc, n);
    vcycle_dispatch(S, S.r, S.z, st);
    S.pcur ^= 1;
  }
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

int solver_solve(Solver& S, const float* b, float* xio, double tol, int maxit, sim_stats* stats, hipStream_t st) {
  const Dims& d = S.lev[0].d;
  const long n = (long)d.cells();
  CGScalars* sc = S.sc;
  double* x = S.x;
  hipLaunchKernelGGL(k_x_load, dim3(nblocks(n)), dim3(kBlock), 0, st, n, xio, x);
  NF_TIMED(S.prof, SIM_K_CG_INIT, st,
           hipLaunchKernelGGL(k_cg_init, dim3(nblocks(n)), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, b, x, S.r,
                              S.partials));
  hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(kFinBlock), 0, st, (int)nblocks(n), S.partials, sc, tol, maxit, n);
  vcycle_dispatch(S, S.r, S.z, st);
  S.pcur = 0;
  // First batch sized from the previous solve of this handle, then small
  // batches.  Every pass of the loop either runs iterations on the device or
  // uses up one of a bounded number of restarts, so the loop terminates.
  const int kMaxRestarts = 8;
  int batch = S.last_iters > 1 ? S.last_iters - 1 : 2;
  const int chunk = S.check_every > 0 ? S.check_every : 2;
  int restarts = 0;
  int r = snapshot(S, st);
  if (r != SIM_OK) return r;
  for (;;) {
    const int it_dev = S.host_sc->iters;
    const int cnt = S.host_sc->done ? 0 : (batch < maxit - it_dev ? batch : maxit - it_dev);
    if (cnt > 0) {
      cg_iterations(S, x, cnt, st);
      r = snapshot(S, st);
      if (r != SIM_OK) return r;
    }
    batch = chunk;
    const CGScalars& h = *S.host_sc;
    if (h.nonfinite) break;
    if (h.done || h.iters >= maxit || cnt <= 0) {
      // true residual from the FP64 iterate; restart from it if needed
      const int allow = restarts < kMaxRestarts && h.iters < maxit ? 1 : 0;
      NF_TIMED(S.prof, SIM_K_CG_TRUE, st,
               hipLaunchKernelGGL(k_cg_true_residual, dim3(nblocks(n)), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, b,
                                  x, S.r, allow, sc, S.partials));
      hipLaunchKernelGGL(k_fin_true, dim3(1), dim3(kFinBlock), 0, st, (int)nblocks(n), S.partials, sc, allow, n);
      r = snapshot(S, st);
      if (r != SIM_OK) return r;
      if (S.host_sc->converged || S.host_sc->nonfinite || !allow) break;
      ++restarts;
      vcycle_dispatch(S, S.r, S.z, st);
    }
  }
  S.last_iters = S.host_sc->iters;
  hipLaunchKernelGGL(k_x_store, dim3(nblocks(n)), dim3(kBlock), 0, st, n, x, xio);
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
