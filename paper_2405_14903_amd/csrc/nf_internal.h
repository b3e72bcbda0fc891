// Internal types and device helpers of the gfx950 MAC-grid library.
// Layouts are those documented in neuralfluid.h (x fastest, velocity =
// x-faces | y-faces | z-faces).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "neuralfluid.h"

namespace nf {

constexpr int kBlock = 256;          // 4 waves of 64 lanes
constexpr int kMaxLevels = 12;
constexpr int kCoarseMaxCells = 4096;   // largest coarsest level (it must fit one workgroup's LDS)
constexpr int kBottomCells = 512;       // levels of at most this many cells run in the one-workgroup bottom solve
constexpr int kPreSweeps = 2;        // damped-Jacobi sweeps before / after coarse correction
constexpr int kBottomSweeps = 4;     // the same on the levels of the one-workgroup bottom solve (even)
constexpr float kOmega = 6.0f / 7.0f;   // damped-Jacobi weight: the smoothing optimum for the 7-point stencil in 3D
// The two sweeps per side of the grid levels use two weights instead: the
// reciprocals of the roots of the degree-2 Chebyshev polynomial on [2/5, 2].
// The eigenvalues of D^-1 A lie in (0, 2]; the modes a grid twice as coarse
// cannot represent have them in [1/3, 2], and of the intervals [a, 2] tried
// (a = 1/6, 1/4, 1/3, 2/5, 1/2) a = 2/5 took the fewest CG iterations.  Two
// such sweeps shrink [2/5, 2] by at most 1 / T_2(3/2) = 0.29 and [1/3, 2] by
// 0.39, against 0.51 for two sweeps with kOmega; the sweeps commute, so the
// V-cycle stays symmetric, and |1 - w1 l| |1 - w2 l| < 1 on (0, 2].
constexpr float kOmega1 = 0.566352f;   // 1 / (6/5 + (4/5) cos(pi/4))
constexpr float kOmega2 = 1.576505f;   // 1 / (6/5 - (4/5) cos(pi/4))
constexpr int kCoarseSweepsMax = 40;   // coarsest level: min(40, 2 * (largest extent)^2) sweeps
constexpr float kCoarseAlphaScale = 0.5f;   // coarse face = 0.5 * sum of the 4 fine faces
constexpr double kVcycleRms = 1.0 / 64.0;   // RMS of the (scaled) residual entering the V-cycle
constexpr float kHalfInvDiagMax = 1024.0f;  // cap of 1/diag in FP16 storage
constexpr float kHalfMax = 65504.0f;         // largest finite FP16 value

// Division of any 32-bit n by a fixed d (1 <= d < 2^32) by multiplication:
// with M = floor((2^64 - 1) / d) + 1 = ceil(2^64 / d), floor(n / d) is the
// high 64 bits of M n (Lemire, Kaser and Kurz, Faster remainder by direct
// computation, 2019: the error term is below n / 2^64 < 1 / d).  d = 1 has
// no 64-bit M and is stored as 0.
__host__ __device__ inline unsigned long long div_magic(int d) {
  return d > 1 ? ~0ull / (unsigned long long)d + 1ull : 0ull;
}
__device__ inline unsigned div_fast(unsigned n, unsigned long long M) {
  return M ? (unsigned)__umul64hi(M, (unsigned long long)n) : n;
}

struct Dims {
  int nx, ny, nz;
  // division multipliers (div_magic) of nx, nx + 1, ny and ny + 1, for the
  // cell, face and node decodes
  unsigned long long mnx, mnx1, mny, mny1;
  Dims() = default;
  __host__ __device__ Dims(int x, int y, int z)
      : nx(x), ny(y), nz(z), mnx(div_magic(x)), mnx1(div_magic(x + 1)), mny(div_magic(y)), mny1(div_magic(y + 1)) {}
  __host__ __device__ size_t cells() const { return (size_t)nx * ny * nz; }
  __host__ __device__ size_t nfx() const { return (size_t)(nx + 1) * ny * nz; }
  __host__ __device__ size_t nfy() const { return (size_t)nx * (ny + 1) * nz; }
  __host__ __device__ size_t nfz() const { return (size_t)nx * ny * (nz + 1); }
  __host__ __device__ size_t faces() const { return nfx() + nfy() + nfz(); }
  __host__ __device__ size_t nodes() const { return (size_t)(nx + 1) * (ny + 1) * (nz + 1); }
  __host__ __device__ int c(int i, int j, int k) const { return i + nx * (j + ny * k); }
  __host__ __device__ int fx(int i, int j, int k) const { return i + (nx + 1) * (j + ny * k); }
  __host__ __device__ int fy(int i, int j, int k) const { return i + nx * (j + (ny + 1) * k); }
  __host__ __device__ int fz(int i, int j, int k) const { return i + nx * (j + ny * k); }
  __host__ __device__ int node(int i, int j, int k) const { return i + (nx + 1) * (j + (ny + 1) * k); }
};

// Geometry parameters, passed by value to kernels.
struct GeomParams {
  int kind;                    // sim_geom
  int nsph;
  double sph[4 * SIM_MAX_SPHERES];
  double c[3], a[3], R[9], v[3], w[3];
  // B-spline wall: control amplitudes (device, SIM_WALL_KNOTS_Y x SIM_WALL_KNOTS_Z,
  // y index major), displacement amp * s(t) * h and velocity amp * s'(t) * h
  const double* knots;
  double wall_s, wall_sd, amp;
  double ly, lz;               // extent of the wall side along y and z
  int wall_imax;               // faces with i > wall_imax are fully fluid
  // parametric solids: the packed solids (device); per solid, the node box
  // (lo x3, extent x3) outside which it cannot be the CSG term of a node
  // whose fractions carry gradient; the distance beyond which no face at a
  // node can be cut (phi there is a lower bound, not exact); and the CSG term
  // of every node (device, one byte per node, kNoSolid in the far field)
  const double* solids;
  int nsolid;
  int sbox[SIM_MAX_SOLIDS][6];
  double solid_far;
  unsigned char* solid_term;
};

struct Domain {
  Dims d;
  int bc[6];
  double dx;
  double inflow;
};

// Face fractions and inverse diagonal of one multigrid level.
struct LevelView {
  Dims d;
  const float* ax;
  const float* ay;
  const float* az;
  const float* invd;
};

// CG scalars kept on the device (no host round trip per iteration).
struct CGScalars {
  double rho;        // r . z
  double alpha;      // step length
  double beta;       // direction update
  double rr;         // r . r
  double bb;         // b . b
  double tol2bb;     // tol^2 * b . b
  double true_rr;    // ||b - A x||^2 recomputed in FP64
  double vscale;     // scale applied to the fine residual before the V-cycle
  double mu;         // mean of the residual over active cells (removed when the system is singular)
  double zmu;        // mean of the preconditioned residual over active cells (singular systems)
  double rho2[2];    // rho and zmu of iteration i in slot i & 1 (read by iteration i + 1 while
  double zmu2[2];    // iteration i + 1's own values go to the other slot)
  double nact;       // number of active cells
  int iters;
  int done;
  int first;
  int nonfinite;
  int maxit;
  int converged;     // true residual reached the tolerance
  int allow;         // a true residual that misses tol may restart CG
  int checks;        // number of true-residual checks that ran in this solve
  int restarts;      // restarts from the true residual in this solve (at most kMaxRestarts)
  int restarted;     // the last true-residual check restarted CG (cleared after the restart V-cycle)
  int final_;        // a true-residual check ended the solve (no further checks run)
  int use_comp;      // residuals are projected region by region (connected-region labels)
  double rr_raw;     // r . r of the initial residual before any projection
  double null_rr;    // the part of r . r along the floating regions' constants
  double comp_rr;    // r . r of the latest CG update (bound of its region sums)
};

// Restarts of CG from the true residual allowed per solve.
constexpr int kMaxRestarts = 8;
// Blocks (and partial sums) of the box-loss kernel: at most this many.
constexpr int kLossBlocks = 2048;
// Connected fluid regions the solver tracks one by one (more: one global mean).
constexpr int kMaxComponents = 65536;

// V-cycle input scale: the residual is scaled to RMS kVcycleRms.
__device__ inline double vscale_of_rr(double rr, long n) {
  double rms = sqrt(rr / (double)n);
  return rms > 0.0 && isfinite(rms) ? kVcycleRms / rms : 1.0;
}

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

// Map the hardware workgroup order (round-robin over the 8 XCDs) to a logical
// order in which each XCD owns one contiguous run of tiles, so neighbouring
// tiles (which share halo data) hit the same L2.
__device__ inline int xcd_block(int b, int nb) {
  const int nx = 8;
  int q = nb / nx, r = nb % nx;
  int x = b % nx, s = b / nx;
  return x * q + (x < r ? x : r) + s;
}

// A wave-uniform value as an opaque register value.  Selecting between struct
// fields by a run-time index otherwise becomes one load from a run-time
// address, which moves the kernel-argument struct to scratch memory.
__device__ inline int uniform_value(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Extent of the domain along axis a.
__device__ inline int extent(const Dims& d, int a) {
  const int nx = uniform_value(d.nx), ny = uniform_value(d.ny), nz = uniform_value(d.nz);
  return a == 0 ? nx : (a == 1 ? ny : nz);
}

// Boundary kind of the domain side a face lies on (-1: interior face).
__device__ inline int side_kind(const Domain& D, int d, int own) {
  const int nd = extent(D.d, d);
  if (own != 0 && own != nd) return -1;
  const int s = 2 * d + (own == 0 ? 0 : 1);
  int v = uniform_value(D.bc[0]);
  v = s == 1 ? uniform_value(D.bc[1]) : v;
  v = s == 2 ? uniform_value(D.bc[2]) : v;
  v = s == 3 ? uniform_value(D.bc[3]) : v;
  v = s == 4 ? uniform_value(D.bc[4]) : v;
  v = s == 5 ? uniform_value(D.bc[5]) : v;
  return v;
}

// Centred cardinal cubic B-spline (support [-2, 2]).
__host__ __device__ inline double bspline3(double s) {
  const double a = s < 0.0 ? -s : s;
  if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
  if (a < 2.0) {
    const double b = 2.0 - a;
    return b * b * b / 6.0;
  }
  return 0.0;
}

// First of the (at most 4) uniform cubic B-spline bases over [0, L] with M
// controls (spacing L / (M - 3), control m centred at m - 1 spacings) that
// are nonzero at s; u = s / spacing.
__host__ __device__ inline int bspline_first(double u) { return (int)floor(u); }

// h(y, z) = sum_mn a_mn B_m(y) B_n(z) of the wall's control amplitudes.
__device__ inline double wall_h(const GeomParams& G, double y, double z) {
  const double uy = y * (SIM_WALL_KNOTS_Y - 3) / G.ly, uz = z * (SIM_WALL_KNOTS_Z - 3) / G.lz;
  const int my = bspline_first(uy), mz = bspline_first(uz);
  double h = 0.0;
  for (int p = 0; p < 4; ++p) {
    const int m = my + p;
    if (m < 0 || m >= SIM_WALL_KNOTS_Y) continue;
    const double by = bspline3(uy - (m - 1));
    double row = 0.0;
    for (int q = 0; q < 4; ++q) {
      const int n = mz + q;
      if (n < 0 || n >= SIM_WALL_KNOTS_Z) continue;
      row += G.knots[m * SIM_WALL_KNOTS_Z + n] * bspline3(uz - (n - 1));
    }
    h += by * row;
  }
  return h;
}

// Normal component of the solid velocity at face (d, i, j, k), with the
// domain-side overrides (WALL: 0, INFLOW: speed into the domain).
__device__ inline double face_solid_velocity(const Domain& D, const GeomParams& G, int d, int i,
                                             int j, int k) {
  int own = d == 0 ? i : (d == 1 ? j : k);
  int sk = side_kind(D, d, own);
  if (sk == SIM_BC_WALL) return 0.0;
  if (sk == SIM_BC_INFLOW) return own == 0 ? D.inflow : -D.inflow;
  if (G.kind == SIM_GEOM_WALL) {
    // the wall moves along x only
    if (d != 0) return 0.0;
    return G.amp * G.wall_sd * wall_h(G, (j + 0.5) * D.dx, (k + 0.5) * D.dx);
  }
  if (G.kind != SIM_GEOM_ELLIPSOID) return 0.0;
  double x[3] = {(i + (d == 0 ? 0.0 : 0.5)) * D.dx, (j + (d == 1 ? 0.0 : 0.5)) * D.dx,
                 (k + (d == 2 ? 0.0 : 0.5)) * D.dx};
  double r0 = x[0] - G.c[0], r1 = x[1] - G.c[1], r2 = x[2] - G.c[2];
  if (d == 0) return G.v[0] + G.w[1] * r2 - G.w[2] * r1;
  if (d == 1) return G.v[1] + G.w[2] * r0 - G.w[0] * r2;
  return G.v[2] + G.w[0] * r1 - G.w[1] * r0;
}

// Decode a flat velocity index into (component, i, j, k) (32-bit arithmetic:
// grids are limited to 2^30 cells).
__device__ inline void face_decode(const Dims& d, long f, int& comp, int& i, int& j, int& k) {
  const unsigned nfx = (unsigned)d.nfx(), nfy = (unsigned)d.nfy();
  unsigned fu = (unsigned)f, sx, sy;
  unsigned long long mx, my;
  if (fu < nfx) {
    comp = 0;
    sx = d.nx + 1;
    sy = d.ny;
    mx = d.mnx1;
    my = d.mny;
  } else if (fu < nfx + nfy) {
    comp = 1;
    fu -= nfx;
    sx = d.nx;
    sy = d.ny + 1;
    mx = d.mnx;
    my = d.mny1;
  } else {
    comp = 2;
    fu -= nfx + nfy;
    sx = d.nx;
    sy = d.ny;
    mx = d.mnx;
    my = d.mny;
  }
  const unsigned t = div_fast(fu, mx);
  i = (int)(fu - t * sx);
  k = (int)div_fast(t, my);
  j = (int)(t - (unsigned)k * sy);
}

// Cell index c (x fastest) into (i, j, k); node index n likewise on the
// (nx + 1) x (ny + 1) node lattice.  32-bit, as face_decode.
__device__ inline void cell_coords(const Dims& d, long c, int& i, int& j, int& k) {
  const unsigned cu = (unsigned)c;
  const unsigned t = div_fast(cu, d.mnx);
  i = (int)(cu - t * (unsigned)d.nx);
  k = (int)div_fast(t, d.mny);
  j = (int)(t - (unsigned)k * (unsigned)d.ny);
}
__device__ inline void node_coords(const Dims& d, long n, int& i, int& j, int& k) {
  const unsigned nu = (unsigned)n;
  const unsigned t = div_fast(nu, d.mnx1);
  i = (int)(nu - t * (unsigned)(d.nx + 1));
  k = (int)div_fast(t, d.mny1);
  j = (int)(t - (unsigned)k * (unsigned)(d.ny + 1));
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Fixed-order block sum of N doubles per thread (deterministic) for a block
// of BS threads.  Result valid in thread 0.  `sh` must hold N * (BS / 64)
// doubles.
template <int N, int BS = kBlock>
__device__ inline void block_sum(double (&v)[N], double* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double s = wave_sum(v[q]);
    if (lane == 0) sh[q * (BS / 64) + wv] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      double s = 0.0;
      for (int w = 0; w < BS / 64; ++w) s += sh[q * (BS / 64) + w];
      v[q] = s;
    }
  }
}

// Write this block's N partial sums to partials[q * gridDim.x + blockIdx.x]
// (fixed-order block sum of a BS-thread block).  A separate single-block
// kernel combines them after the kernel boundary, so no cross-workgroup
// synchronisation is needed.
template <int N, int BS = kBlock>
__device__ inline void block_partials(double (&v)[N], double* partials) {
  __shared__ double sh[N * (BS / 64) + 1];
  block_sum<N, BS>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) partials[(size_t)q * gridDim.x + blockIdx.x] = v[q];
  }
}

// Fixed-order total of N partial arrays of nb entries, by one block of
// kFinBlock threads.  Result valid in thread 0.
constexpr int kFinBlock = 1024;
template <int N>
__device__ inline void finish_partials(const double* partials, int nb, double (&tot)[N]) {
  __shared__ double sh[N * (kFinBlock / 64) + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kFinBlock) s += partials[(size_t)q * nb + b];
    s = wave_sum(s);
    if (lane == 0) sh[q * (kFinBlock / 64) + wv] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      double s = 0.0;
      for (int w = 0; w < kFinBlock / 64; ++w) s += sh[q * (kFinBlock / 64) + w];
      tot[q] = s;
    }
  }
}

// Fixed-order total of N partial arrays of nb entries by every thread block
// of BS threads (each block gets the same bits).  Result valid in thread 0.
template <int N, int BS>
__device__ inline void block_total(const double* partials, int nb, double (&tot)[N]) {
  __shared__ double sh[N * (BS / 64) + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += BS) s += partials[(size_t)q * nb + b];
    s = wave_sum(s);
    if (lane == 0) sh[q * (BS / 64) + wv] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      double s = 0.0;
      for (int w = 0; w < BS / 64; ++w) s += sh[q * (BS / 64) + w];
      tot[q] = s;
    }
  }
}

// The same total in two steps, so that a kernel can issue its own first loads
// between them: partials_load reads the (at most K * BS) partials into
// registers; partials_reduce sums them in block_total's order (result in
// thread 0 and in *out for every thread; it holds a barrier).
template <int K, int BS>
__device__ inline void partials_load(const double* partials, int nb, double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int b = threadIdx.x + k * BS;
    v[k] = b < nb ? partials[b] : 0.0;
  }
}
template <int K, int BS>
__device__ inline double partials_reduce(const double (&v)[K], double* out) {
  __shared__ double sh[BS / 64 + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) s += v[k];
  s = wave_sum(s);
  if (lane == 0) sh[wv] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < BS / 64; ++w) t += sh[w];
    *out = t;
  }
  __syncthreads();
  return *out;
}

// N partial arrays (nb entries each, at most K * BS) read into registers, then
// totalled by every block in block_total's order (the same bits in each block;
// result for every thread; holds two barriers).
template <int N, int K, int BS>
__device__ inline void partials_load_n(const double* partials, int nb, double (&v)[N][K]) {
#pragma unroll
  for (int q = 0; q < N; ++q)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int b = threadIdx.x + k * BS;
      v[q][k] = b < nb ? partials[(size_t)q * nb + b] : 0.0;
    }
}
template <int N, int K, int BS>
__device__ inline void partials_reduce_n(const double (&v)[N][K], double (&tot)[N]) {
  __shared__ double sh[N * (BS / 64)];
  __shared__ double res[N];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) s += v[q][k];
    s = wave_sum(s);
    if (lane == 0) sh[q * (BS / 64) + wv] = s;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double t = 0.0;
    for (int w = 0; w < BS / 64; ++w) t += sh[threadIdx.x * (BS / 64) + w];
    res[threadIdx.x] = t;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < N; ++q) tot[q] = res[q];
}

// Blocks of the CG update kernel (grid-stride): few enough that every block of
// the next kernel can total their r . r partials itself.
constexpr int kUpdateBlocks = 1024;
// Most r . z partials (tiles of the finest level) that every block of the
// direction kernel totals itself; beyond, a one-block kernel totals them.
constexpr int kRzPartsMax = 1024;

}  // namespace nf
