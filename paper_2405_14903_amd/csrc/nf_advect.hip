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
  double ds[3];   // d(clamped coordinate)/dX: 1 inside the lattice, 0 if clamped
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
  int i0[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double s = X[a] - (a == e ? 0.0 : 0.5);
    double hi = (double)(m[a] - 1);
    t.ds[a] = (s >= 0.0 && s <= hi) ? 1.0 : 0.0;
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
  double v[8];   // v[bx + 2 by + 4 bz]
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
  double c00 = c.v[0] + fx * (c.v[1] - c.v[0]);
  double c10 = c.v[2] + fx * (c.v[3] - c.v[2]);
  double c01 = c.v[4] + fx * (c.v[5] - c.v[4]);
  double c11 = c.v[6] + fx * (c.v[7] - c.v[6]);
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
  const double* v = c.v;
  double gx0 = (1 - fy) * (v[1] - v[0]) + fy * (v[3] - v[2]);
  double gx1 = (1 - fy) * (v[5] - v[4]) + fy * (v[7] - v[6]);
  g[0] = ((1 - fz) * gx0 + fz * gx1) * t.ds[0];
  double gy0 = (1 - fx) * (v[2] - v[0]) + fx * (v[3] - v[1]);
  double gy1 = (1 - fx) * (v[6] - v[4]) + fx * (v[7] - v[5]);
  g[1] = ((1 - fz) * gy0 + fz * gy1) * t.ds[1];
  double lo = v[0] + fx * (v[1] - v[0]), lo2 = v[2] + fx * (v[3] - v[2]);
  double hi = v[4] + fx * (v[5] - v[4]), hi2 = v[6] + fx * (v[7] - v[6]);
  g[2] = ((1 - fy) * (hi - lo) + fy * (hi2 - lo2)) * t.ds[2];
}

__device__ inline void tap_scatter(float* __restrict__ g, const Tap& t, double w) {
  if (w == 0.0) return;
  const double fx = t.f[0], fy = t.f[1], fz = t.f[2];
  const double wz[2] = {1.0 - fz, fz}, wy[2] = {1.0 - fy, fy}, wx[2] = {1.0 - fx, fx};
#pragma unroll
  for (int bz = 0; bz < 2; ++bz)
#pragma unroll
    for (int by = 0; by < 2; ++by)
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        double ww = w * wz[bz] * wy[by] * wx[bx];
        if (ww != 0.0) unsafeAtomicAdd(g + t.base + bx + by * t.sx + bz * t.sxy, (float)ww);
      }
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

__global__ __launch_bounds__(kBlock) void k_advect_adjoint(Dims d, double cfl, const float* __restrict__ u,
                                                            const float* __restrict__ gout,
                                                            float* __restrict__ gin) {
  long nf = (long)d.faces();
  long f = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const double g = gout[f];
  if (g == 0.0) return;
  int comp, i, j, k;
  face_decode(d, f, comp, i, j, k);
  const float* uc[3] = {u, u + d.nfx(), u + d.nfx() + d.nfy()};
  float* gc[3] = {gin, gin + d.nfx(), gin + d.nfx() + d.nfy()};
  double Xf[3], v0[3], Xm[3], v1[3], Xs[3];
  face_pos(comp, i, j, k, Xf);
  Tap t0[3], t1[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    t0[e] = make_tap(d, e, Xf);
    v0[e] = tap_value(uc[e], t0[e]);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) Xm[a] = Xf[a] - 0.5 * cfl * v0[a];
  Corners c1[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    t1[e] = make_tap(d, e, Xm);
    c1[e] = load_corners(uc[e], t1[e]);
    v1[e] = corner_value(c1[e], t1[e]);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) Xs[a] = Xf[a] - cfl * v1[a];
  Tap ts = make_tap(d, comp, Xs);
  // U~_f = I_comp(u; X_src)
  tap_scatter(gc[comp], ts, g);
  double gs[3];
  corner_grad(load_corners(uc[comp], ts), ts, gs);
  double gv1[3], gXm[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 3; ++a) gv1[a] = -cfl * g * gs[a];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    tap_scatter(gc[e], t1[e], gv1[e]);
    double ge[3];
    corner_grad(c1[e], t1[e], ge);
#pragma unroll
    for (int a = 0; a < 3; ++a) gXm[a] += gv1[e] * ge[a];
  }
#pragma unroll
  for (int e = 0; e < 3; ++e) tap_scatter(gc[e], t0[e], -0.5 * cfl * gXm[e]);
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
  hipLaunchKernelGGL(k_advect_adjoint, dim3(nblocks(d.faces())), dim3(kBlock), 0, s, d, dt / dx, u, gout, gin);
}

}  // namespace nf
