// Connected fluid regions of the pressure system and the null space they
// carry.
//
// Cells joined through faces with alpha > 0 form the connected regions of
// G^T S G.  A region that reaches no OUTFLOW face (no Dirichlet ghost; Sec.
// Projection, App. B Eq. bd:dirichlet) is floating: its pressure is defined up
// to a constant, and its right-hand side must sum to zero over it.  The
// solver projects the residual onto that compatible subspace region by
// region (subtracting each floating region's mean) at the start of a solve and
// at every restart, and measures convergence on the projected residual.
//
// Labelling: union-find over the faces with atomic compare-and-swap (every
// link points from a larger to a smaller cell index, so each chain strictly
// decreases and every find ends), then path flattening, then compact region
// ids in cell order of the regions' smallest cells.  Region sums are formed in
// 64-bit fixed point, so they are the same bits whatever the order of the
// atomic additions.
#include "nf_solver.h"

namespace nf {

namespace {

inline unsigned nblocks(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__device__ inline void cell_of(const Dims& d, long c, int& i, int& j, int& k) { cell_coords(d, c, i, j, k); }

__device__ inline bool cell_active(const Dims& d, const float* ax, const float* ay, const float* az, int i, int j,
                                   int k) {
  return ax[d.fx(i, j, k)] > 0.0f || ax[d.fx(i + 1, j, k)] > 0.0f || ay[d.fy(i, j, k)] > 0.0f ||
         ay[d.fy(i, j + 1, k)] > 0.0f || az[d.fz(i, j, k)] > 0.0f || az[d.fz(i, j, k + 1)] > 0.0f;
}

// Root of x: follow parents until a self-parent (each step decreases the index).
__device__ inline int ccl_find(const int* parent, int x) {
  for (;;) {
    const int p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
    if (p == x) return x;
    x = p;
  }
}

// Join the regions of a and b: the larger root is linked under the smaller one.
// A failed compare-and-swap means another thread linked that root first (the
// number of roots only falls), so the loop ends.
__device__ inline void ccl_unite(int* parent, int a, int b) {
  for (;;) {
    a = ccl_find(parent, a);
    b = ccl_find(parent, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    if (atomicCAS(&parent[a], a, b) == a) return;
  }
}

__global__ void k_ccl_init(Dims d, const float* __restrict__ ax, const float* __restrict__ ay,
                           const float* __restrict__ az, int* __restrict__ parent) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)d.cells()) return;
  int i, j, k;
  cell_of(d, c, i, j, k);
  parent[c] = cell_active(d, ax, ay, az, i, j, k) ? (int)c : -1;
}

__global__ void k_ccl_union(Dims d, const float* __restrict__ ax, const float* __restrict__ ay,
                            const float* __restrict__ az, int* parent) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)d.cells()) return;
  int i, j, k;
  cell_of(d, c, i, j, k);
  // a face with alpha > 0 between two cells makes both of them active
  if (i + 1 < d.nx && ax[d.fx(i + 1, j, k)] > 0.0f) ccl_unite(parent, (int)c, (int)c + 1);
  if (j + 1 < d.ny && ay[d.fy(i, j + 1, k)] > 0.0f) ccl_unite(parent, (int)c, (int)c + d.nx);
  if (k + 1 < d.nz && az[d.fz(i, j, k + 1)] > 0.0f) ccl_unite(parent, (int)c, (int)(c + (long)d.nx * d.ny));
}

__global__ void k_ccl_flatten(long n, int* parent) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || parent[c] < 0) return;
  parent[c] = ccl_find(parent, (int)c);
}

// Number of region roots in each block of cells.
__global__ __launch_bounds__(kBlock) void k_ccl_count_roots(long n, const int* __restrict__ parent,
                                                            int* __restrict__ blockcnt) {
  __shared__ int sh[kBlock / 64];
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool root = c < n && parent[c] == (int)c;
  const unsigned long long b = __ballot(root);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = __popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < kBlock / 64; ++w) s += sh[w];
    blockcnt[blockIdx.x] = s;
  }
}

// Exclusive scan of the block counts (one workgroup, in order); the total is
// the region count.
__global__ __launch_bounds__(1024) void k_ccl_scan(int nb, const int* __restrict__ blockcnt,
                                                   int* __restrict__ blockbase, int* __restrict__ info) {
  __shared__ int sh[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += 1024) {
    const int q = base + (int)threadIdx.x;
    const int v = q < nb ? blockcnt[q] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive Hillis-Steele scan
      const int t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (q < nb) blockbase[q] = carry + sh[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    info[0] = carry;
    info[1] = carry <= kMaxComponents ? 1 : 0;
  }
}

// Region id of each root: its rank among the roots in cell order.
__global__ __launch_bounds__(kBlock) void k_ccl_assign(long n, const int* __restrict__ parent,
                                                       const int* __restrict__ blockbase, int* __restrict__ comp) {
  __shared__ int sh[kBlock / 64];
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool root = c < n && parent[c] == (int)c;
  const unsigned long long b = __ballot(root);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = __popcll(b);
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wv; ++w) before += sh[w];
  const unsigned long long below = lane ? (b & ((1ull << lane) - 1ull)) : 0ull;
  if (root) comp[c] = blockbase[blockIdx.x] + before + __popcll(below);
}

__global__ void k_ccl_spread(long n, const int* __restrict__ parent, int* comp) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int p = parent[c];
  if (p < 0)
    comp[c] = -1;
  else if (p != (int)c)
    comp[c] = comp[p];
}

__global__ void k_comp_clear(int* __restrict__ count, int* __restrict__ ground) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < kMaxComponents; q += gridDim.x * blockDim.x) {
    count[q] = 0;
    ground[q] = 0;
  }
}

// Cells per region, and whether a region has a face with alpha > 0 on an
// OUTFLOW side (a Dirichlet ghost: the region is grounded, not floating).
// The lanes of a wave that all belong to one region count with one atomic.
__global__ __launch_bounds__(kBlock) void k_comp_count(Dims d, Sides sides, const float* __restrict__ ax,
                                                       const float* __restrict__ ay, const float* __restrict__ az,
                                                       const int* __restrict__ comp, const int* __restrict__ info,
                                                       int* count, int* ground) {
  if (!info[1]) return;
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int id = c < (long)d.cells() ? comp[c] : -1;
  const int lead = __shfl(id, 0, 64);
  if (__ballot(id != lead) == 0ull) {
    if (lead >= 0 && (threadIdx.x & 63) == 0) atomicAdd(&count[lead], 64);
  } else if (id >= 0) {
    atomicAdd(&count[id], 1);
  }
  if (id < 0) return;
  int i, j, k;
  cell_of(d, c, i, j, k);
  const bool g = (i == 0 && sides.out[0] && ax[d.fx(0, j, k)] > 0.0f) ||
                 (i == d.nx - 1 && sides.out[1] && ax[d.fx(d.nx, j, k)] > 0.0f) ||
                 (j == 0 && sides.out[2] && ay[d.fy(i, 0, k)] > 0.0f) ||
                 (j == d.ny - 1 && sides.out[3] && ay[d.fy(i, d.ny, k)] > 0.0f) ||
                 (k == 0 && sides.out[4] && az[d.fz(i, j, 0)] > 0.0f) ||
                 (k == d.nz - 1 && sides.out[5] && az[d.fz(i, j, d.nz)] > 0.0f);
  if (g) ground[id] = 1;
}

// parent[] becomes each cell's reference cell: the root (first cell) of its
// region when the region is floating, -1 otherwise.
__global__ void k_comp_ref(long n, const int* __restrict__ comp, const int* __restrict__ ground,
                           const int* __restrict__ info, int* parent) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int id = comp[c];
  if (id < 0 || !info[1] || ground[id]) parent[c] = -1;
}

// The preconditioned residual z of a floating region is defined up to that
// region's constant, and the V-cycle maps constants to large multiples of
// themselves; left in z they would swamp the FP32 search direction.  Each
// region's z is shifted by its value at the reference cell (a null-space
// move: A z and the CG dots against r, whose region sums vanish, keep their
// values), in two passes so that no cell reads a value already shifted.
__global__ void k_comp_zroot(long n, const int* __restrict__ ref, const int* __restrict__ comp,
                             const float* __restrict__ z, float* __restrict__ zroot, const CGScalars* sc) {
  if (sc->done || !sc->use_comp) return;
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n && ref[c] == (int)c) zroot[comp[c]] = z[c];
}
__global__ void k_comp_zshift(long n, const int* __restrict__ ref, const int* __restrict__ comp,
                              const float* __restrict__ zroot, float* __restrict__ z, const CGScalars* sc) {
  if (sc->done || !sc->use_comp) return;
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n && ref[c] >= 0) z[c] -= zroot[comp[c]];
}

// Fixed-point scale of the region sums of r: |r_c| <= sqrt(r.r), so a sum of
// at most n terms stays below 2^61 in magnitude.
__device__ inline double fixed_scale(double rr, double n) {
  const double bound = sqrt(rr) * (n > 1.0 ? n : 1.0);
  if (!(bound > 0.0) || !isfinite(bound)) return 0.0;
  int e;
  frexp(bound, &e);   // bound < 2^e
  return ldexp(1.0, 61 - e);
}

__global__ void k_comp_zero_sums(long long* __restrict__ sums, const int* __restrict__ info) {
  const int ncomp = info[0] < kMaxComponents ? info[0] : kMaxComponents;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < ncomp; q += gridDim.x * blockDim.x) sums[q] = 0;
}

// Region sums of r in fixed point.  The lanes of a wave that all belong to one
// region (the common case) add their total with one atomic.
__global__ __launch_bounds__(kBlock) void k_comp_sums(long n, const int* __restrict__ comp,
                                                      const float* __restrict__ r, const CGScalars* sc,
                                                      const int* __restrict__ info, long long* sums, int iter) {
  if (!info[1] || (iter && (sc->done || !sc->use_comp))) return;
  const double scale = fixed_scale(iter ? sc->comp_rr : sc->rr_raw, (double)n);
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int id = c < n ? comp[c] : -1;
  long long q = id >= 0 ? (long long)llrint((double)r[c] * scale) : 0ll;
  const int lead = __shfl(id, 0, 64);
  const bool uniform = __ballot(id != lead) == 0ull;
  if (uniform) {
    if (lead < 0) return;
    for (int o = 32; o > 0; o >>= 1) q += __shfl_down(q, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd((unsigned long long*)&sums[lead], (unsigned long long)q);
  } else if (id >= 0) {
    atomicAdd((unsigned long long*)&sums[id], (unsigned long long)q);
  }
}

// Region means of r (0 on grounded regions) and the part of r . r along the
// null space, sum over floating regions of sum^2 / count (fixed-order total);
// at the start of a solve (iter = 0) also the convergence state after the
// projection.
__global__ __launch_bounds__(kFinBlock) void k_comp_finish(const long long* __restrict__ sums,
                                                           const int* __restrict__ count,
                                                           const int* __restrict__ ground,
                                                           const int* __restrict__ info, double* __restrict__ mean,
                                                           CGScalars* sc, long ncells, int iter) {
  __shared__ double sh[kFinBlock / 64 + 1];
  if (iter && (sc->done || !sc->use_comp)) return;
  const int ok = info[1];
  const int ncomp = ok ? info[0] : 0;
  const double scale = fixed_scale(iter ? sc->comp_rr : sc->rr_raw, (double)ncells);
  double v[1] = {0.0};
  for (int q = threadIdx.x; q < ncomp; q += kFinBlock) {
    double m = 0.0;
    if (!ground[q] && count[q] > 0 && scale > 0.0) {
      const double s = (double)sums[q] / scale;
      m = s / (double)count[q];
      v[0] += s * m;
    }
    mean[q] = m;
  }
  block_sum<1, kFinBlock>(v, sh);
  if (threadIdx.x == 0 && !iter) {
    sc->use_comp = ok;
    if (!ok) return;
    sc->null_rr = v[0];
    double rr = sc->rr_raw - v[0];
    rr = rr > 0.0 ? rr : 0.0;
    sc->rr = rr;
    sc->true_rr = rr;
    sc->mu = 0.0;
    sc->vscale = vscale_of_rr(rr, ncells);
    sc->converged = (sc->bb == 0.0) || (rr <= sc->tol2bb);
    sc->done = sc->converged || sc->nonfinite || sc->maxit <= 0;
  }
}

// r . r of the CG update (its per-block partials): the bound of the
// fixed-point region sums of the updated residual.
__global__ __launch_bounds__(kFinBlock) void k_comp_rr(int nb, const double* __restrict__ partials, CGScalars* sc) {
  if (sc->done || !sc->use_comp) return;
  double tot[1];
  finish_partials<1>(partials, nb, tot);
  if (threadIdx.x == 0) sc->comp_rr = tot[0];
}

// r -= mean of its region (floating regions; skipped once the solve is done,
// like every solver kernel).  With more regions than tracked, the one global
// mean over active cells of closed domains (sc->mu; 0 otherwise) instead.
__global__ void k_comp_subtract(long n, const int* __restrict__ comp, const double* __restrict__ mean,
                                float* __restrict__ r, const CGScalars* sc, int iter) {
  if (sc->done || (iter && !sc->use_comp)) return;
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int id = comp[c];
  if (id < 0) return;
  const double m = sc->use_comp ? mean[id] : sc->mu;
  r[c] = (float)((double)r[c] - m);
}

}  // namespace

void components_label(Solver& S, hipStream_t st) {
  const Dims& d = S.lev[0].d;
  const long n = (long)d.cells();
  const unsigned nb = nblocks(n);
  Components& K = S.comp;
  hipLaunchKernelGGL(k_ccl_init, dim3(nb), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, K.parent);
  hipLaunchKernelGGL(k_ccl_union, dim3(nb), dim3(kBlock), 0, st, d, S.ax, S.ay, S.az, K.parent);
  hipLaunchKernelGGL(k_ccl_flatten, dim3(nb), dim3(kBlock), 0, st, n, K.parent);
  hipLaunchKernelGGL(k_ccl_count_roots, dim3(nb), dim3(kBlock), 0, st, n, K.parent, K.blockcnt);
  hipLaunchKernelGGL(k_ccl_scan, dim3(1), dim3(1024), 0, st, (int)nb, K.blockcnt, K.blockbase, K.info);
  hipLaunchKernelGGL(k_ccl_assign, dim3(nb), dim3(kBlock), 0, st, n, K.parent, K.blockbase, K.id);
  hipLaunchKernelGGL(k_ccl_spread, dim3(nb), dim3(kBlock), 0, st, n, K.parent, K.id);
  hipLaunchKernelGGL(k_comp_clear, dim3(64), dim3(kBlock), 0, st, K.count, K.ground);
  hipLaunchKernelGGL(k_comp_count, dim3(nb), dim3(kBlock), 0, st, d, S.sides, S.ax, S.ay, S.az, K.id, K.info,
                     K.count, K.ground);
  hipLaunchKernelGGL(k_comp_ref, dim3(nb), dim3(kBlock), 0, st, n, K.id, K.ground, K.info, K.parent);
  K.valid = true;
}

void components_shift_z(Solver& S, hipStream_t st) {
  const long n = (long)S.lev[0].d.cells();
  const unsigned nb = nblocks(n);
  Components& K = S.comp;
  hipLaunchKernelGGL(k_comp_zroot, dim3(nb), dim3(kBlock), 0, st, n, K.parent, K.id, S.z, K.zroot, S.sc);
  hipLaunchKernelGGL(k_comp_zshift, dim3(nb), dim3(kBlock), 0, st, n, K.parent, K.id, K.zroot, S.z, S.sc);
}

void components_project_start(Solver& S, hipStream_t st) {
  const Dims& d = S.lev[0].d;
  const long n = (long)d.cells();
  Components& K = S.comp;
  hipLaunchKernelGGL(k_comp_zero_sums, dim3(64), dim3(kBlock), 0, st, K.sums, K.info);
  hipLaunchKernelGGL(k_comp_sums, dim3(nblocks(n)), dim3(kBlock), 0, st, n, K.id, S.r, S.sc, K.info, K.sums, 0);
  hipLaunchKernelGGL(k_comp_finish, dim3(1), dim3(kFinBlock), 0, st, K.sums, K.count, K.ground, K.info, K.mean,
                     S.sc, n, 0);
  components_subtract(S, st, 0);
}

void components_project_iter(Solver& S, int nrr, hipStream_t st) {
  const Dims& d = S.lev[0].d;
  const long n = (long)d.cells();
  Components& K = S.comp;
  hipLaunchKernelGGL(k_comp_rr, dim3(1), dim3(kFinBlock), 0, st, nrr, S.partials_rr, S.sc);
  hipLaunchKernelGGL(k_comp_zero_sums, dim3(64), dim3(kBlock), 0, st, K.sums, K.info);
  hipLaunchKernelGGL(k_comp_sums, dim3(nblocks(n)), dim3(kBlock), 0, st, n, K.id, S.r, S.sc, K.info, K.sums, 1);
  hipLaunchKernelGGL(k_comp_finish, dim3(1), dim3(kFinBlock), 0, st, K.sums, K.count, K.ground, K.info, K.mean,
                     S.sc, n, 1);
  components_subtract(S, st, 1);
}

void components_subtract(Solver& S, hipStream_t st, int iter) {
  const long n = (long)S.lev[0].d.cells();
  hipLaunchKernelGGL(k_comp_subtract, dim3(nblocks(n)), dim3(kBlock), 0, st, n, S.comp.id, S.comp.mean, S.r, S.sc,
                     iter);
}

}  // namespace nf
