// Semi-Lagrangian advection of the face velocity and its adjoint.
//
// NeuralFluid, Eq. advection_matrix: U~ = B(U^n) U^n, B a linear
// interpolation at back-traced points; App. B, Eqs. advection_1/2 give the
// two-stage (midpoint) back-trace.  Per face f of component d at position x_f
// (index units, X = x / dx; cfl = dt / dx):
//   v0 = V(u; X_f), X_mid = X_f - (cfl/2) v0, v1 = V(u; X_mid),
//   X_src = X_f - cfl v1, U~_f = I_d(u; X_src),
// I_e trilinear on component e's own staggered lattice (offset 1/2 along the
// two other axes), coordinates clamped to the lattice and the base index
// min(floor(s), m - 2).  App. B, Eq. apply_force: U^ = U~ + dt g.
// Positions, cell choices and weights are computed in FP64 (the velocities
// are FP32): the derivative of a trilinear interpolant jumps across cell
// boundaries, so the cell a back-traced point falls in is decided in double
// precision, as in the FP64 reference.
//
// The adjoint reverses the chain: the interpolation weights scatter the
// incoming gradient to their 8 taps (float atomics), and the departure-point
// dependence adds grad_X I terms through X_src and X_mid (Sec.
// Back-propagation through Time, Viscosity and Advection paragraph: the
// dB/dU U^n + B(U^n) terms).
#include "nf_internal.h"

namespace nf {

struct Tap {
  int base;       // flat index of the (i0, j0, k0) corner
  int sx, sxy;    // strides of the component lattice
  double f[3];    // fractions
  int inside;     // bit a: coordinate a lies inside the lattice (d clamped / dX = 1), else clamped (0)
};

// Lattice sizes of component e.
__device__ inline void lattice(const Dims& d, int e, int m[3]) {
  m[0] = d.nx + (e == 0);
  m[1] = d.ny + (e == 1);
  m[2] = d.nz + (e == 2);
}

__device__ inline Tap make_tap(const Dims& d, int e, const double X[3]) {
  int m[3];
  lattice(d, e, m);
  Tap t;
  t.inside = 0;
  int i0[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double s = X[a] - (a == e ? 0.0 : 0.5);
    double hi = (double)(m[a] - 1);
    if (s >= 0.0 && s <= hi) t.inside |= 1 << a;
    s = fmin(fmax(s, 0.0), hi);
    int i = (int)floor(s);
    i = i < m[a] - 2 ? i : m[a] - 2;
    i0[a] = i;
    t.f[a] = s - (double)i;
  }
  t.sx = m[0];
  t.sxy = m[0] * m[1];
  t.base = i0[0] + t.sx * (i0[1] + m[1] * i0[2]);
  return t;
}

struct Corners {
  float v[8];   // v[bx + 2 by + 4 bz] (the velocities are FP32; arithmetic on them is FP64)
};

__device__ inline Corners load_corners(const float* __restrict__ u, const Tap& t) {
  const float* p = u + t.base;
  Corners c;
  c.v[0] = p[0];
  c.v[1] = p[1];
  c.v[2] = p[t.sx];
  c.v[3] = p[t.sx + 1];
  c.v[4] = p[t.sxy];
  c.v[5] = p[t.sxy + 1];
  c.v[6] = p[t.sxy + t.sx];
  c.v[7] = p[t.sxy + t.sx + 1];
  return c;
}

__device__ inline double corner_value(const Corners& c, const Tap& t) {
  const double fx = t.f[0], fy = t.f[1], fz = t.f[2];
  double v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = (double)c.v[q];
  double c00 = v[0] + fx * (v[1] - v[0]);
  double c10 = v[2] + fx * (v[3] - v[2]);
  double c01 = v[4] + fx * (v[5] - v[4]);
  double c11 = v[6] + fx * (v[7] - v[6]);
  double c0 = c00 + fy * (c10 - c00);
  double c1 = c01 + fy * (c11 - c01);
  return c0 + fz * (c1 - c0);
}

__device__ inline double tap_value(const float* __restrict__ u, const Tap& t) {
  return corner_value(load_corners(u, t), t);
}

// d value / dX (index units), zero along clamped axes.
__device__ inline void corner_grad(const Corners& c, const Tap& t, double g[3]) {
  const double fx = t.f[0], fy = t.f[1], fz = t.f[2];
  double v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = (double)c.v[q];
  double gx0 = (1 - fy) * (v[1] - v[0]) + fy * (v[3] - v[2]);
  double gx1 = (1 - fy) * (v[5] - v[4]) + fy * (v[7] - v[6]);
  g[0] = (t.inside & 1) ? (1 - fz) * gx0 + fz * gx1 : 0.0;
  double gy0 = (1 - fx) * (v[2] - v[0]) + fx * (v[3] - v[1]);
  double gy1 = (1 - fx) * (v[6] - v[4]) + fx * (v[7] - v[5]);
  g[1] = (t.inside & 2) ? (1 - fz) * gy0 + fz * gy1 : 0.0;
  double lo = v[0] + fx * (v[1] - v[0]), lo2 = v[2] + fx * (v[3] - v[2]);
  double hi = v[4] + fx * (v[5] - v[4]), hi2 = v[6] + fx * (v[7] - v[6]);
  g[2] = (t.inside & 4) ? (1 - fy) * (hi - lo) + fy * (hi2 - lo2) : 0.0;
}

__device__ inline void face_pos(int comp, int i, int j, int k, double X[3]) {
  X[0] = (double)i + (comp == 0 ? 0.0 : 0.5);
  X[1] = (double)j + (comp == 1 ? 0.0 : 0.5);
  X[2] = (double)k + (comp == 2 ? 0.0 : 0.5);
}

__global__ __launch_bounds__(kBlock) void k_advect(Dims d, double cfl, float g0, float g1, float g2, float dt,
                                                    const float* __restrict__ u, float* __restrict__ out) {
  long nf = (long)d.faces();
  long f = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int comp, i, j, k;
  face_decode(d, f, comp, i, j, k);
  const float* uc[3] = {u, u + d.nfx(), u + d.nfx() + d.nfy()};
  double Xf[3], v0[3], Xm[3], v1[3], Xs[3];
  face_pos(comp, i, j, k, Xf);
#pragma unroll
  for (int e = 0; e < 3; ++e) v0[e] = tap_value(uc[e], make_tap(d, e, Xf));
#pragma unroll
  for (int a = 0; a < 3; ++a) Xm[a] = Xf[a] - 0.5 * cfl * v0[a];
#pragma unroll
  for (int e = 0; e < 3; ++e) v1[e] = tap_value(uc[e], make_tap(d, e, Xm));
#pragma unroll
  for (int a = 0; a < 3; ++a) Xs[a] = Xf[a] - cfl * v1[a];
  double val = tap_value(uc[comp], make_tap(d, comp, Xs));
  float gcomp = comp == 0 ? g0 : (comp == 1 ? g1 : g2);
  out[f] = (float)val + dt * gcomp;
}

// Adjoint scatter target: component lattice e, flat index `idx`, lattice
// coordinates (a, b, c).  Targets inside the workgroup's LDS window are
// accumulated there; others go straight to global memory.
struct Window {
  int o[3];                 // lattice coordinate of the window origin (same for all components)
  float* lds;               // 3 windows of kWin^3 floats
};
constexpr int kBrick = 8;
constexpr int kHalo = 2;
constexpr int kWin = kBrick + 1 + 2 * kHalo;

__device__ inline void scatter_w(const Window& W, float* __restrict__ g, int e, const Tap& t, double w) {
  if (w == 0.0) return;
  const double fx = t.f[0], fy = t.f[1], fz = t.f[2];
  const double wz[2] = {1.0 - fz, fz}, wy[2] = {1.0 - fy, fy}, wx[2] = {1.0 - fx, fx};
  // lattice coordinates of the base corner
  const int a0 = t.base % t.sx, b0 = (t.base / t.sx) % (t.sxy / t.sx), c0 = t.base / t.sxy;
  const int la = a0 - W.o[0], lb = b0 - W.o[1], lc = c0 - W.o[2];
  const bool inside = la >= 0 && lb >= 0 && lc >= 0 && la + 1 < kWin && lb + 1 < kWin && lc + 1 < kWin;
  float* win = W.lds + e * kWin * kWin * kWin;
#pragma unroll
  for (int bz = 0; bz < 2; ++bz)
#pragma unroll
    for (int by = 0; by < 2; ++by)
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        double ww = w * wz[bz] * wy[by] * wx[bx];
        if (ww == 0.0) continue;
        if (inside)
          atomicAdd(win + (la + bx) + kWin * ((lb + by) + kWin * (lc + bz)), (float)ww);
        else
          unsafeAtomicAdd(g + t.base + bx + by * t.sx + bz * t.sxy, (float)ww);
      }
}

// One workgroup per 8^3 brick of cells; it handles the faces owned by the
// brick (a face belongs to the cell on its + side, the upper domain faces to
// the last cell) and accumulates their scatters in LDS windows that cover the
// brick plus a 2-cell halo, then adds each touched window entry to global
// memory once.
__global__ __launch_bounds__(kBlock) void k_advect_adjoint(Dims d, double cfl, const float* __restrict__ u,
                                                            const float* __restrict__ gout,
                                                            float* __restrict__ gin) {
  __shared__ float lds[3 * kWin * kWin * kWin];
  const int nbx = (d.nx + kBrick - 1) / kBrick, nby = (d.ny + kBrick - 1) / kBrick;
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int bxi = bid % nbx, byi = (bid / nbx) % nby, bzi = bid / (nbx * nby);
  const int i0 = bxi * kBrick, j0 = byi * kBrick, k0 = bzi * kBrick;
  Window W;
  W.o[0] = i0 - kHalo;
  W.o[1] = j0 - kHalo;
  W.o[2] = k0 - kHalo;
  W.lds = lds;
  for (int q = threadIdx.x; q < 3 * kWin * kWin * kWin; q += blockDim.x) lds[q] = 0.0f;
  __syncthreads();
  const float* uc[3] = {u, u + d.nfx(), u + d.nfx() + d.nfy()};
  float* gc[3] = {gin, gin + d.nfx(), gin + d.nfx() + d.nfy()};
  // faces of the brick, per component: extents along each axis
  int ext[3][3];
  const int bn[3] = {min(kBrick, d.nx - i0), min(kBrick, d.ny - j0), min(kBrick, d.nz - k0)};
  const bool last[3] = {i0 + kBrick >= d.nx, j0 + kBrick >= d.ny, k0 + kBrick >= d.nz};
  int total = 0, start[4];
  for (int e = 0; e < 3; ++e) {
    start[e] = total;
    for (int a = 0; a < 3; ++a) ext[e][a] = bn[a] + ((a == e && last[a]) ? 1 : 0);
    total += ext[e][0] * ext[e][1] * ext[e][2];
  }
  start[3] = total;
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int comp = q < start[1] ? 0 : (q < start[2] ? 1 : 2);
    const int lq = q - start[comp];
    const int li = lq % ext[comp][0], lj = (lq / ext[comp][0]) % ext[comp][1], lk = lq / (ext[comp][0] * ext[comp][1]);
    const int i = i0 + li, j = j0 + lj, k = k0 + lk;
    const long f = comp == 0 ? (long)d.fx(i, j, k)
                             : (comp == 1 ? (long)d.nfx() + d.fy(i, j, k) : (long)d.nfx() + d.nfy() + d.fz(i, j, k));
    const double g = gout[f];
    if (g == 0.0) continue;
    // recompute the back-trace (the taps of X_f and the corners of X_mid are
    // re-derived / re-loaded where they are needed, to keep registers low)
    double Xf[3], v0[3], Xm[3], v1[3], Xs[3];
    face_pos(comp, i, j, k, Xf);
#pragma unroll
    for (int e = 0; e < 3; ++e) v0[e] = tap_value(uc[e], make_tap(d, e, Xf));
#pragma unroll
    for (int a = 0; a < 3; ++a) Xm[a] = Xf[a] - 0.5 * cfl * v0[a];
    Tap t1[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      t1[e] = make_tap(d, e, Xm);
      v1[e] = tap_value(uc[e], t1[e]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) Xs[a] = Xf[a] - cfl * v1[a];
    const Tap ts = make_tap(d, comp, Xs);
    // U~_f = I_comp(u; X_src)
    scatter_w(W, gc[comp], comp, ts, g);
    double gs[3];
    corner_grad(load_corners(uc[comp], ts), ts, gs);
    double gXm[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const double gv1 = -cfl * g * gs[e];
      scatter_w(W, gc[e], e, t1[e], gv1);
      double ge[3];
      corner_grad(load_corners(uc[e], t1[e]), t1[e], ge);
#pragma unroll
      for (int a = 0; a < 3; ++a) gXm[a] += gv1 * ge[a];
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) scatter_w(W, gc[e], e, make_tap(d, e, Xf), -0.5 * cfl * gXm[e]);
  }
  __syncthreads();
  // flush the windows
  for (int q = threadIdx.x; q < 3 * kWin * kWin * kWin; q += blockDim.x) {
    const float v = lds[q];
    if (v == 0.0f) continue;
    const int e = q / (kWin * kWin * kWin);
    const int r = q % (kWin * kWin * kWin);
    const int a = W.o[0] + r % kWin, b = W.o[1] + (r / kWin) % kWin, c = W.o[2] + r / (kWin * kWin);
    int m[3];
    lattice(d, e, m);
    if (a < 0 || b < 0 || c < 0 || a >= m[0] || b >= m[1] || c >= m[2]) continue;
    unsafeAtomicAdd(gc[e] + a + m[0] * (b + m[1] * c), v);
  }
}

__global__ void k_fill(float* __restrict__ p, long n, float v) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static inline unsigned nblocks(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

void launch_fill(float* p, size_t n, float v, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(kBlock), 0, s, p, (long)n, v);
}

void launch_advect(const Dims& d, double dx, double dt, const double* grav, const float* u, float* out,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_advect, dim3(nblocks(d.faces())), dim3(kBlock), 0, s, d, dt / dx, (float)grav[0],
                     (float)grav[1], (float)grav[2], (float)dt, u, out);
}

void launch_advect_adjoint(const Dims& d, double dx, double dt, const float* u, const float* gout,
                           float* gin, hipStream_t s) {
  const unsigned nb = (unsigned)(((d.nx + kBrick - 1) / kBrick) * ((d.ny + kBrick - 1) / kBrick) *
                                 ((d.nz + kBrick - 1) / kBrick));
  hipLaunchKernelGGL(k_advect_adjoint, dim3(nb), dim3(kBlock), 0, s, d, dt / dx, u, gout, gin);
}

}  // namespace nf
