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
//
// The adjoint reverses the chain: the interpolation weights scatter the
// incoming gradient to their 8 taps (float atomics), and the departure-point
// dependence adds grad_X I terms through X_src and X_mid (Sec.
// Back-propagation through Time, Viscosity and Advection paragraph: the
// dB/dU U^n + B(U^n) terms).
#include "nf_internal.h"

namespace nf {

struct Tap {
  int base;      // flat index of the (i0, j0, k0) corner
  int sx, sxy;   // strides of the component lattice
  float f[3];    // fractions
  float ds[3];   // d(clamped coordinate)/dX: 1 inside the lattice, 0 if clamped
};

// Lattice sizes of component e.
__device__ inline void lattice(const Dims& d, int e, int m[3]) {
  m[0] = d.nx + (e == 0);
  m[1] = d.ny + (e == 1);
  m[2] = d.nz + (e == 2);
}

__device__ inline Tap make_tap(const Dims& d, int e, const float X[3]) {
  int m[3];
  lattice(d, e, m);
  Tap t;
  int i0[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float s = X[a] - (a == e ? 0.0f : 0.5f);
    float hi = (float)(m[a] - 1);
    t.ds[a] = (s >= 0.0f && s <= hi) ? 1.0f : 0.0f;
    s = fminf(fmaxf(s, 0.0f), hi);
    int i = (int)floorf(s);
    i = i < m[a] - 2 ? i : m[a] - 2;
    i0[a] = i;
    t.f[a] = s - (float)i;
  }
  t.sx = m[0];
  t.sxy = m[0] * m[1];
  t.base = i0[0] + t.sx * (i0[1] + m[1] * i0[2]);
  return t;
}

__device__ inline float tap_value(const float* __restrict__ u, const Tap& t) {
  const float* p = u + t.base;
  float fx = t.f[0], fy = t.f[1], fz = t.f[2];
  float c00 = p[0] + fx * (p[1] - p[0]);
  float c10 = p[t.sx] + fx * (p[t.sx + 1] - p[t.sx]);
  float c01 = p[t.sxy] + fx * (p[t.sxy + 1] - p[t.sxy]);
  float c11 = p[t.sxy + t.sx] + fx * (p[t.sxy + t.sx + 1] - p[t.sxy + t.sx]);
  float c0 = c00 + fy * (c10 - c00);
  float c1 = c01 + fy * (c11 - c01);
  return c0 + fz * (c1 - c0);
}

// d value / dX (index units), zero along clamped axes.
__device__ inline void tap_grad(const float* __restrict__ u, const Tap& t, float g[3]) {
  const float* p = u + t.base;
  float v000 = p[0], v100 = p[1], v010 = p[t.sx], v110 = p[t.sx + 1];
  float v001 = p[t.sxy], v101 = p[t.sxy + 1], v011 = p[t.sxy + t.sx], v111 = p[t.sxy + t.sx + 1];
  float fx = t.f[0], fy = t.f[1], fz = t.f[2];
  float gx0 = (1 - fy) * (v100 - v000) + fy * (v110 - v010);
  float gx1 = (1 - fy) * (v101 - v001) + fy * (v111 - v011);
  g[0] = ((1 - fz) * gx0 + fz * gx1) * t.ds[0];
  float gy0 = (1 - fx) * (v010 - v000) + fx * (v110 - v100);
  float gy1 = (1 - fx) * (v011 - v001) + fx * (v111 - v101);
  g[1] = ((1 - fz) * gy0 + fz * gy1) * t.ds[1];
  float lo = v000 + fx * (v100 - v000), lo2 = v010 + fx * (v110 - v010);
  float hi = v001 + fx * (v101 - v001), hi2 = v011 + fx * (v111 - v011);
  g[2] = ((1 - fy) * (hi - lo) + fy * (hi2 - lo2)) * t.ds[2];
}

__device__ inline void tap_scatter(float* __restrict__ g, const Tap& t, float w) {
  if (w == 0.0f) return;
  float fx = t.f[0], fy = t.f[1], fz = t.f[2];
  float wz[2] = {1.0f - fz, fz}, wy[2] = {1.0f - fy, fy}, wx[2] = {1.0f - fx, fx};
#pragma unroll
  for (int bz = 0; bz < 2; ++bz)
#pragma unroll
    for (int by = 0; by < 2; ++by)
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        float ww = w * wz[bz] * wy[by] * wx[bx];
        if (ww != 0.0f) unsafeAtomicAdd(g + t.base + bx + by * t.sx + bz * t.sxy, ww);
      }
}

__device__ inline void face_pos(int comp, int i, int j, int k, float X[3]) {
  X[0] = (float)i + (comp == 0 ? 0.0f : 0.5f);
  X[1] = (float)j + (comp == 1 ? 0.0f : 0.5f);
  X[2] = (float)k + (comp == 2 ? 0.0f : 0.5f);
}

__global__ __launch_bounds__(kBlock) void k_advect(Dims d, float cfl, float g0, float g1, float g2,
                                                    float dt, const float* __restrict__ u,
                                                    float* __restrict__ out) {
  long nf = (long)d.faces();
  long f = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int comp, i, j, k;
  face_decode(d, f, comp, i, j, k);
  const float* uc[3] = {u, u + d.nfx(), u + d.nfx() + d.nfy()};
  float Xf[3];
  face_pos(comp, i, j, k, Xf);
  float v0[3], Xm[3], v1[3], Xs[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) v0[e] = tap_value(uc[e], make_tap(d, e, Xf));
#pragma unroll
  for (int a = 0; a < 3; ++a) Xm[a] = Xf[a] - 0.5f * cfl * v0[a];
#pragma unroll
  for (int e = 0; e < 3; ++e) v1[e] = tap_value(uc[e], make_tap(d, e, Xm));
#pragma unroll
  for (int a = 0; a < 3; ++a) Xs[a] = Xf[a] - cfl * v1[a];
  float val = tap_value(uc[comp], make_tap(d, comp, Xs));
  float gcomp = comp == 0 ? g0 : (comp == 1 ? g1 : g2);
  out[f] = val + dt * gcomp;
}

__global__ __launch_bounds__(kBlock) void k_advect_adjoint(Dims d, float cfl,
                                                            const float* __restrict__ u,
                                                            const float* __restrict__ gout,
                                                            float* __restrict__ gin) {
  long nf = (long)d.faces();
  long f = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  float g = gout[f];
  if (g == 0.0f) return;
  int comp, i, j, k;
  face_decode(d, f, comp, i, j, k);
  const float* uc[3] = {u, u + d.nfx(), u + d.nfx() + d.nfy()};
  float* gc[3] = {gin, gin + d.nfx(), gin + d.nfx() + d.nfy()};
  float Xf[3];
  face_pos(comp, i, j, k, Xf);
  Tap t0[3], t1[3];
  float v0[3], Xm[3], v1[3], Xs[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    t0[e] = make_tap(d, e, Xf);
    v0[e] = tap_value(uc[e], t0[e]);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) Xm[a] = Xf[a] - 0.5f * cfl * v0[a];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    t1[e] = make_tap(d, e, Xm);
    v1[e] = tap_value(uc[e], t1[e]);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) Xs[a] = Xf[a] - cfl * v1[a];
  Tap ts = make_tap(d, comp, Xs);
  // U~_f = I_comp(u; X_src)
  tap_scatter(gc[comp], ts, g);
  float gs[3];
  tap_grad(uc[comp], ts, gs);
  float gv1[3], gXm[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int a = 0; a < 3; ++a) gv1[a] = -cfl * g * gs[a];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    tap_scatter(gc[e], t1[e], gv1[e]);
    float ge[3];
    tap_grad(uc[e], t1[e], ge);
#pragma unroll
    for (int a = 0; a < 3; ++a) gXm[a] += gv1[e] * ge[a];
  }
#pragma unroll
  for (int e = 0; e < 3; ++e) tap_scatter(gc[e], t0[e], -0.5f * cfl * gXm[e]);
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
  hipLaunchKernelGGL(k_advect, dim3(nblocks(d.faces())), dim3(kBlock), 0, s, d, (float)(dt / dx),
                     (float)grav[0], (float)grav[1], (float)grav[2], (float)dt, u, out);
}

void launch_advect_adjoint(const Dims& d, double dx, double dt, const float* u, const float* gout,
                           float* gin, hipStream_t s) {
  hipLaunchKernelGGL(k_advect_adjoint, dim3(nblocks(d.faces())), dim3(kBlock), 0, s, d,
                     (float)(dt / dx), u, gout, gin);
}

}  // namespace nf
