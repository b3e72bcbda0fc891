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
// min(floor(s), m - 2).  A constant body force g (this library's addition,
// for the hydrostatic check) is added here: U~ + dt g.
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
  int i0[3];      // lattice coordinates of that corner
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
  t.i0[0] = i0[0];
  t.i0[1] = i0[1];
  t.i0[2] = i0[2];
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

// The corners of the tap of component e != comp at the centre of a face of
// component comp with coordinates idx.  There the back-trace's fractions are
// fixed: 1/2 along comp between cell indices idx - 1 and idx (one index, with
// weight 1, at the two ends of the axis, where the coordinate is clamped), 1/2
// along e between face indices idx and idx + 1, and 0 along the third axis.
// So the tap is the mean of the lattice values at flat indices p[0..n-1]
// (n = 4, or 2 at the ends), and its adjoint adds 1/n of the incoming weight
// to each: the weights of the trilinear formula at these fractions, exactly.
// Returns n; with n = 2 the points are p[0], p[1] (p[2], p[3] repeat them).
__device__ inline int face_centre_corners(const Dims& d, int e, int comp, const int idx[3], int p[4], int ix[4][3]) {
  int m[3];
  lattice(d, e, m);
  int lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a == comp) {
      lo[a] = max(idx[a] - 1, 0);
      hi[a] = min(idx[a], m[a] - 1);
    } else if (a == e) {
      lo[a] = idx[a];
      hi[a] = idx[a] + 1;
    } else {
      lo[a] = hi[a] = idx[a];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    // q bit 0: e axis, bit 1: comp axis
#pragma unroll
    for (int a = 0; a < 3; ++a) ix[q][a] = a == e ? ((q & 1) ? hi[a] : lo[a]) : (a == comp ? ((q & 2) ? hi[a] : lo[a]) : lo[a]);
    p[q] = ix[q][0] + m[0] * (ix[q][1] + m[1] * ix[q][2]);
  }
  // (selects, not an index by the run-time comp: that would go through scratch)
  const bool one = comp == 0 ? lo[0] == hi[0] : (comp == 1 ? lo[1] == hi[1] : lo[2] == hi[2]);
  return one ? 2 : 4;
}

__device__ inline double face_centre_value(const Dims& d, const float* __restrict__ ue, int e, int comp,
                                           const int idx[3]) {
  int p[4], ix[4][3];
  const int n = face_centre_corners(d, e, comp, idx, p, ix);
  const double a = 0.5 * ((double)ue[p[0]] + (double)ue[p[1]]);
  return n == 2 ? a : 0.5 * (a + 0.5 * ((double)ue[p[2]] + (double)ue[p[3]]));
}

__device__ inline void face_pos(int comp, int i, int j, int k, double X[3]) {
  X[0] = (double)i + (comp == 0 ? 0.0 : 0.5);
  X[1] = (double)j + (comp == 1 ? 0.0 : 0.5);
  X[2] = (double)k + (comp == 2 ? 0.0 : 0.5);
}

// trace (optional): the back-traced positions X_mid and X_src of every face,
// as six FP64 arrays of d.faces() entries (X_mid x, y, z, X_src x, y, z), for
// the adjoint of the same step.
__global__ __launch_bounds__(kBlock) void k_advect(Dims d, double cfl, float g0, float g1, float g2, float dt,
                                                    const float* __restrict__ u, float* __restrict__ out,
                                                    double* __restrict__ trace) {
  long nf = (long)d.faces();
  long f = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int comp, i, j, k;
  face_decode(d, f, comp, i, j, k);
  const float* uc[3] = {u, u + d.nfx(), u + d.nfx() + d.nfy()};
  double Xf[3], v0[3], Xm[3], v1[3], Xs[3];
  face_pos(comp, i, j, k, Xf);
  // the face's own component at the face is the face's value: its lattice
  // coordinates are integers, so every fraction is 0 (or 1 on the last face,
  // where the lerp returns the upper value exactly); the others are the mean
  // of 4 lattice values (face_centre_corners)
  const int idx[3] = {i, j, k};
#pragma unroll
  for (int e = 0; e < 3; ++e) v0[e] = e == comp ? (double)u[f] : face_centre_value(d, uc[e], e, comp, idx);
#pragma unroll
  for (int a = 0; a < 3; ++a) Xm[a] = Xf[a] - 0.5 * cfl * v0[a];
#pragma unroll
  for (int e = 0; e < 3; ++e) v1[e] = tap_value(uc[e], make_tap(d, e, Xm));
#pragma unroll
  for (int a = 0; a < 3; ++a) Xs[a] = Xf[a] - cfl * v1[a];
  if (trace) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      trace[(size_t)a * nf + f] = Xm[a];
      trace[(size_t)(3 + a) * nf + f] = Xs[a];
    }
  }
  double val = tap_value(uc[comp], make_tap(d, comp, Xs));
  float gcomp = comp == 0 ? g0 : (comp == 1 ? g1 : g2);
  out[f] = (float)val + dt * gcomp;
}

// Adjoint scatter target: component lattice e, flat index `idx`, lattice
// coordinates (a, b, c).  Targets inside the workgroup's LDS window are
// accumulated there in 64-bit fixed point (value * scale, rounded): integer
// LDS atomics run at full rate, float LDS atomics about 3.5x slower than the
// whole rest of the kernel, and the integer sums are also independent of the
// order of the adds.  Others, and any value too large for the fixed-point
// range, go straight to global memory as float atomics.
struct Window {
  int o[3];                       // lattice coordinate of the window origin (same for all components)
  unsigned long long* lds;        // 3 windows of kWinX * kWinY * kWinZ fixed-point sums
  double scale;                   // fixed-point scale of this workgroup
  double limit;                   // largest |value * scale| accumulated in the window
};
// Brick of cells owned by one workgroup (at most 9*8*4 + 8*9*4 + 8*8*5 = 896
// faces, up to four per thread) and the halo of its scatter windows.  Four
// 256-thread workgroups share a CU (the kernel's registers allow 4 waves per
// SIMD), so one workgroup's barriers and window set-up overlap the others'
// scatters: measured at 128^3, 411 us for the pair of kernels against 524 us
// with one 1024-thread workgroup per brick and 584 us with 128 threads.
constexpr int kBX = 8, kBY = 8, kBZ = 4;
constexpr int kAdjThreads = 256;
constexpr int kHalo = 2;
constexpr int kWinX = kBX + 1 + 2 * kHalo, kWinY = kBY + 1 + 2 * kHalo, kWinZ = kBZ + 1 + 2 * kHalo;
constexpr int kWin3 = kWinX * kWinY * kWinZ;

// q / e for 0 <= q < 2^12 and 1 <= e <= 2^7 from a float reciprocal:
// (q + 1/2) / e lies at least 1 / (2e) >= 2^-8 from an integer, and the float
// product is within 2^-22 q / e <= 2^-10 of it.
__device__ inline int small_div(int q, float inv_e) { return (int)(((float)q + 0.5f) * inv_e); }

// Face q of a brick (faces of component 0 first, then 1, then 2, x fastest):
// its component and coordinates in the brick, from the components' first
// indices s1, s2, their extents along x and y (e*0, e*1) and the reciprocals
// of e*0 and e*0 * e*1 (selects rather than an index by the run-time
// component).
struct BrickFace {
  int comp, li, lj, lk;
};
__device__ __forceinline__ BrickFace brick_face(int q, int s1, int s2, int ea0, int ea1, int eb0, int eb1, int ec0,
                                                int ec1, float ra0, float ra01, float rb0, float rb01, float rc0,
                                                float rc01) {
  BrickFace b;
  b.comp = q < s1 ? 0 : (q < s2 ? 1 : 2);
  const bool c0 = b.comp == 0, c1 = b.comp == 1;
  const int lq = q - (c0 ? 0 : (c1 ? s1 : s2));
  const int e0 = c0 ? ea0 : (c1 ? eb0 : ec0);
  const int e1 = c0 ? ea1 : (c1 ? eb1 : ec1);
  const int q0 = small_div(lq, c0 ? ra0 : (c1 ? rb0 : rc0));
  b.lk = small_div(lq, c0 ? ra01 : (c1 ? rb01 : rc01));
  b.li = lq - q0 * e0;
  b.lj = q0 - b.lk * e1;
  return b;
}

// v rounded to the nearest integer (ties to even) as a 64-bit integer, for
// |v| <= 2^51: adding 1.5 * 2^52 leaves the integer in the low mantissa bits.
__device__ inline long long fixed_round(double v) {
  return __double_as_longlong(v + 6755399441055744.0) - 0x4338000000000000LL;
}

__device__ inline void scatter_w(const Window& W, float* __restrict__ g, int e, const Tap& t, double w) {
  if (w == 0.0) return;
  const double fx = t.f[0], fy = t.f[1], fz = t.f[2];
  const int la = t.i0[0] - W.o[0], lb = t.i0[1] - W.o[1], lc = t.i0[2] - W.o[2];
  const bool inside = la >= 0 && lb >= 0 && lc >= 0 && la + 1 < kWinX && lb + 1 < kWinY && lc + 1 < kWinZ;
  const double ws = w * W.scale;   // every tap's value is at most |ws| (weights <= 1)
  if (inside && fabs(ws) <= W.limit) {
    unsigned long long* win = W.lds + e * kWin3 + la + kWinX * (lb + kWinY * lc);
    const double wz[2] = {ws * (1.0 - fz), ws * fz};
#pragma unroll
    for (int bz = 0; bz < 2; ++bz)
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        const double wy = wz[bz] * (by ? fy : 1.0 - fy);
        if (wy == 0.0) continue;
        unsigned long long* row = win + kWinX * (by + kWinY * bz);
        // taps of weight 0 (a fraction of exactly 0 or 1, as at face centres) add nothing
        const long long lo = fixed_round(wy * (1.0 - fx)), hi = fixed_round(wy * fx);
        if (lo) atomicAdd(row, (unsigned long long)lo);
        if (hi) atomicAdd(row + 1, (unsigned long long)hi);
      }
    return;
  }
  const double wz[2] = {1.0 - fz, fz}, wy[2] = {1.0 - fy, fy}, wx[2] = {1.0 - fx, fx};
#pragma unroll
  for (int bz = 0; bz < 2; ++bz)
#pragma unroll
    for (int by = 0; by < 2; ++by)
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        const double ww = w * wz[bz] * wy[by] * wx[bx];
        if (ww != 0.0)
          __hip_atomic_fetch_add(g + t.base + bx + by * t.sx + bz * t.sxy, (float)ww, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
}

// Add w to N lattice points of component e (flat indices p, lattice
// coordinates ix): the same fixed-point window or float-atomic paths as
// scatter_w, with its criterion (every point inside the window and the
// scaled value within the fixed-point range, else every point goes to global
// memory as float atomics).
template <int N>
__device__ inline void scatter_points(const Window& W, float* __restrict__ g, int e, const int p[4], const int ix[4][3],
                                      double w) {
  if (w == 0.0) return;
  const double ws = w * W.scale;
  bool inside = true;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const int la = ix[q][0] - W.o[0], lb = ix[q][1] - W.o[1], lc = ix[q][2] - W.o[2];
    inside = inside && la >= 0 && lb >= 0 && lc >= 0 && la < kWinX && lb < kWinY && lc < kWinZ;
  }
  if (inside && fabs(ws) <= W.limit) {
    const long long v = fixed_round(ws);
    if (v == 0) return;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const int la = ix[q][0] - W.o[0], lb = ix[q][1] - W.o[1], lc = ix[q][2] - W.o[2];
      atomicAdd(W.lds + e * kWin3 + la + kWinX * (lb + kWinY * lc), (unsigned long long)v);
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < N; ++q)
    __hip_atomic_fetch_add(g + p[q], (float)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One workgroup per brick of kBX x kBY x kBZ cells; its threads walk the faces
// owned by the brick (a face belongs to the cell on its + side, the upper
// domain faces to the last cell).  The scatters accumulate in LDS windows that cover
// the brick plus a kHalo-cell halo.  The windows are then stored whole to a
// staging area (coalesced, no atomics); k_advect_adjoint_gather adds, for
// every face, the entries of the windows that cover it.  Taps outside the
// window (more than about one cell of motion per step) are added to gin
// directly with float atomics.
__global__ __launch_bounds__(kAdjThreads) void k_advect_adjoint(Dims d, double cfl, const float* __restrict__ u,
                                                                 const double* __restrict__ trace,
                                                                 const float* __restrict__ gout,
                                                                 float* __restrict__ gin, float* __restrict__ stage) {
  __shared__ unsigned long long lds[3 * kWin3];
  __shared__ float red[2 * (kAdjThreads / 64)];
  const int nbx = (d.nx + kBX - 1) / kBX, nby = (d.ny + kBY - 1) / kBY;
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int bxi = bid % nbx, byi = (bid / nbx) % nby, bzi = bid / (nbx * nby);
  const int i0 = bxi * kBX, j0 = byi * kBY, k0 = bzi * kBZ;
  Window W;
  W.o[0] = i0 - kHalo;
  W.o[1] = j0 - kHalo;
  W.o[2] = k0 - kHalo;
  W.lds = lds;
  const float* uc[3] = {u, u + d.nfx(), u + d.nfx() + d.nfy()};
  float* gc[3] = {gin, gin + d.nfx(), gin + d.nfx() + d.nfy()};
  // Fixed-point scale from bounds of this workgroup's contributions: with
  // G = max |g| over its faces and U = max |u| over the window region, every
  // scattered value is at most G * max(1, 2 cfl U, 6 cfl^2 U^2) (interpolation
  // weights <= 1, trilinear gradients in index units <= 2U); 2^50 / bound
  // leaves room for 2^12 adds per entry below 2^62.  A scatter whose value
  // still exceeds 2^51 (corners outside the window region) takes the float
  // path.
  for (int q = threadIdx.x; q < 3 * kWin3; q += blockDim.x) lds[q] = 0ull;
  // largest |u| over the window region (coordinates clamped to the lattice),
  // one x row of a component per thread
  float um = 0.0f;
  for (int row = threadIdx.x; row < 3 * kWinY * kWinZ; row += blockDim.x) {
    const int e = row / (kWinY * kWinZ), rr = row - e * (kWinY * kWinZ);
    const int m0 = d.nx + (e == 0), m1 = d.ny + (e == 1), m2 = d.nz + (e == 2);
    const int b = min(max(W.o[1] + rr % kWinY, 0), m1 - 1);
    const int c = min(max(W.o[2] + rr / kWinY, 0), m2 - 1);
    const float* base = e == 0 ? u : (e == 1 ? u + d.nfx() : u + d.nfx() + d.nfy());
    const float* rowp = base + (size_t)m0 * ((size_t)b + (size_t)m1 * c);
    // a fixed, unrolled row (clamped like the coordinates): its loads are
    // independent and go out together
#pragma unroll
    for (int t = 0; t < kWinX; ++t) um = fmaxf(um, fabsf(rowp[min(max(W.o[0] + t, 0), m0 - 1)]));
  }
  // faces of the brick, per component: extents along each axis
  int ext[3][3];
  const int bn[3] = {min(kBX, d.nx - i0), min(kBY, d.ny - j0), min(kBZ, d.nz - k0)};
  const bool last[3] = {i0 + kBX >= d.nx, j0 + kBY >= d.ny, k0 + kBZ >= d.nz};
  int total = 0, start[4];
  for (int e = 0; e < 3; ++e) {
    start[e] = total;
    for (int a = 0; a < 3; ++a) ext[e][a] = bn[a] + ((a == e && last[a]) ? 1 : 0);
    total += ext[e][0] * ext[e][1] * ext[e][2];
  }
  start[3] = total;
  // the brick's faces by index (brick_face)
  const int s1 = start[1], s2 = start[2];
  const int ea0 = ext[0][0], ea1 = ext[0][1], eb0 = ext[1][0], eb1 = ext[1][1], ec0 = ext[2][0], ec1 = ext[2][1];
  const float ra0 = 1.0f / (float)ea0, ra01 = 1.0f / (float)(ea0 * ea1);
  const float rb0 = 1.0f / (float)eb0, rb01 = 1.0f / (float)(eb0 * eb1);
  const float rc0 = 1.0f / (float)ec0, rc01 = 1.0f / (float)(ec0 * ec1);
  float gm = 0.0f;
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const BrickFace bf = brick_face(q, s1, s2, ea0, ea1, eb0, eb1, ec0, ec1, ra0, ra01, rb0, rb01, rc0, rc01);
    const int comp = bf.comp, li = bf.li, lj = bf.lj, lk = bf.lk;
    const long f = comp == 0 ? (long)d.fx(i0 + li, j0 + lj, k0 + lk)
                             : (comp == 1 ? (long)d.nfx() + d.fy(i0 + li, j0 + lj, k0 + lk)
                                          : (long)d.nfx() + d.nfy() + d.fz(i0 + li, j0 + lj, k0 + lk));
    gm = fmaxf(gm, fabsf(gout[f]));
  }
  for (int o = 32; o > 0; o >>= 1) {
    um = fmaxf(um, __shfl_down(um, o, 64));
    gm = fmaxf(gm, __shfl_down(gm, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = um;
    red[(kAdjThreads / 64) + (threadIdx.x >> 6)] = gm;
  }
  __syncthreads();
  {
    float U = 0.0f, Gm = 0.0f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      U = fmaxf(U, red[w]);
      Gm = fmaxf(Gm, red[(kAdjThreads / 64) + w]);
    }
    const double cu = cfl * (double)U;
    const double bound = (double)Gm * fmax(1.0, fmax(2.0 * cu, 6.0 * cu * cu));
    W.scale = bound > 0.0 && isfinite(bound) ? 1125899906842624.0 / bound : 1.0;   // 2^50 / bound
    W.limit = 2251799813685248.0;                                                  // 2^51 (fixed_round's range)
  }
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const BrickFace bf = brick_face(q, s1, s2, ea0, ea1, eb0, eb1, ec0, ec1, ra0, ra01, rb0, rb01, rc0, rc01);
    const int comp = bf.comp, li = bf.li, lj = bf.lj, lk = bf.lk;
    const int i = i0 + li, j = j0 + lj, k = k0 + lk;
    const long f = comp == 0 ? (long)d.fx(i, j, k)
                             : (comp == 1 ? (long)d.nfx() + d.fy(i, j, k) : (long)d.nfx() + d.nfy() + d.fz(i, j, k));
    const double g = gout[f];
    if (g == 0.0) continue;
    // the step's back-traced positions (k_advect of the same u); taps are
    // re-derived from them where they are needed instead of being kept
    double Xf[3], Xm[3], Xs[3];
    face_pos(comp, i, j, k, Xf);
    const size_t nf = d.faces();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Xm[a] = trace[(size_t)a * nf + f];
      Xs[a] = trace[(size_t)(3 + a) * nf + f];
    }
    double gs[3];
    {
      // U~_f = I_comp(u; X_src)
      const Tap ts = make_tap(d, comp, Xs);
      scatter_w(W, gc[comp], comp, ts, g);
      corner_grad(load_corners(uc[comp], ts), ts, gs);
    }
    double gXm[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const Tap t1 = make_tap(d, e, Xm);
      const double gv1 = -cfl * g * gs[e];
      scatter_w(W, gc[e], e, t1, gv1);
      double ge[3];
      corner_grad(load_corners(uc[e], t1), t1, ge);
#pragma unroll
      for (int a = 0; a < 3; ++a) gXm[a] += gv1 * ge[a];
    }
    // the taps at the face centre (face_centre_corners): the face itself for
    // its own component, a quarter of the weight on 4 lattice points for the
    // others
    const int idx[3] = {i, j, k};
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const double w = -0.5 * cfl * gXm[e];
      if (e == comp) {
        const int own[4][3] = {{i, j, k}, {i, j, k}, {i, j, k}, {i, j, k}};
        const int p[4] = {(int)(f - (long)(gc[comp] - gin)), 0, 0, 0};
        scatter_points<1>(W, gc[e], e, p, own, w);
      } else {
        int p[4], ix[4][3];
        if (face_centre_corners(d, e, comp, idx, p, ix) == 2)
          scatter_points<2>(W, gc[e], e, p, ix, 0.5 * w);
        else
          scatter_points<4>(W, gc[e], e, p, ix, 0.25 * w);
      }
    }
  }
  __syncthreads();
  // store the three windows of this brick (back from fixed point)
  float* dst = stage + (size_t)bid * (3 * kWin3);
  const double inv = 1.0 / W.scale;
  for (int q = threadIdx.x; q < 3 * kWin3; q += blockDim.x) dst[q] = (float)((double)(long long)lds[q] * inv);
}

// gin_f += sum of the staged window entries of face f over the bricks whose
// window covers it (brick b along an axis with brick size B covers lattice
// coordinates B b - kHalo .. B b - kHalo + (window size) - 1).
__device__ inline int cover_lo(int v, int B, int W) {
  // ceil((v + kHalo - W + 1) / B), clamped at 0 (the offset keeps the division non-negative)
  return max(0, (v + kHalo - W + 1 + B - 1 + 64 * B) / B - 64);
}

__global__ __launch_bounds__(kBlock) void k_advect_adjoint_gather(Dims d, const float* __restrict__ stage,
                                                                   float* __restrict__ gin) {
  const long f = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (f >= (long)d.faces()) return;
  int comp, a, b, c;
  face_decode(d, f, comp, a, b, c);
  const int nbx = (d.nx + kBX - 1) / kBX, nby = (d.ny + kBY - 1) / kBY, nbz = (d.nz + kBZ - 1) / kBZ;
  const int x0 = cover_lo(a, kBX, kWinX), x1 = min(nbx - 1, (a + kHalo) / kBX);
  const int y0 = cover_lo(b, kBY, kWinY), y1 = min(nby - 1, (b + kHalo) / kBY);
  const int z0 = cover_lo(c, kBZ, kWinZ), z1 = min(nbz - 1, (c + kHalo) / kBZ);
  float s = 0.0f;
  for (int bz = z0; bz <= z1; ++bz)
    for (int by = y0; by <= y1; ++by)
      for (int bx = x0; bx <= x1; ++bx) {
        const int la = a - (kBX * bx - kHalo), lb = b - (kBY * by - kHalo), lc = c - (kBZ * bz - kHalo);
        const size_t brick = (size_t)bx + nbx * ((size_t)by + (size_t)nby * bz);
        s += stage[brick * 3 * kWin3 + comp * kWin3 + la + kWinX * (lb + kWinY * lc)];
      }
  gin[f] += s;
}

size_t advect_stage_floats(const Dims& d) {
  const size_t nb = (size_t)((d.nx + kBX - 1) / kBX) * ((d.ny + kBY - 1) / kBY) * ((d.nz + kBZ - 1) / kBZ);
  return nb * 3 * kWin3;
}

__global__ void k_copy(const float* __restrict__ src, float* __restrict__ dst, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_fill(float* __restrict__ p, long n, float v) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static inline unsigned nblocks(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Viscosity (Eq. viscosity_matrix; App. B Eq. apply_force, explicit):
// out = in + c (-G_f^T G_f) in with c = nu dt / dx^2, G_f the differences of
// each velocity component over the edges of its own face lattice: the sum over
// a lattice point's neighbours inside the lattice of (neighbour - point).  The
// operator is symmetric, so the same kernel applies its adjoint.
__global__ __launch_bounds__(kBlock) void k_viscosity(Dims d, float c, const float* __restrict__ in,
                                                      float* __restrict__ out) {
  const long f = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= (long)d.faces()) return;
  int comp, i, j, k;
  face_decode(d, f, comp, i, j, k);
  const int mx = d.nx + (comp == 0), my = d.ny + (comp == 1), mz = d.nz + (comp == 2);
  const long sy = mx, sz = (long)mx * my;
  const float v = in[f];
  float s = 0.0f;
  if (i > 0) s += in[f - 1] - v;
  if (i < mx - 1) s += in[f + 1] - v;
  if (j > 0) s += in[f - sy] - v;
  if (j < my - 1) s += in[f + sy] - v;
  if (k > 0) s += in[f - sz] - v;
  if (k < mz - 1) s += in[f + sz] - v;
  out[f] = v + c * s;
}

void launch_viscosity(const Dims& d, double c, const float* in, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_viscosity, dim3(nblocks(d.faces())), dim3(kBlock), 0, s, d, (float)c, in, out);
}

// max over faces of |u_f| (order-free, so the same bits every time): one
// atomic max per block on the bits of a non-negative float
__global__ __launch_bounds__(kBlock) void k_max_abs(long n, const float* __restrict__ u, unsigned* __restrict__ out) {
  __shared__ float sh[kBlock / 64];
  const long f = (long)blockIdx.x * blockDim.x + threadIdx.x;
  float v = f < n ? fabsf(u[f]) : 0.0f;
  if (!(v == v)) v = __int_as_float(0x7f800000);   // a NaN reads as +inf
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_down(v, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = sh[0];
    for (int w = 1; w < kBlock / 64; ++w) m = fmaxf(m, sh[w]);
    atomicMax(out, __float_as_uint(m));
  }
}

__global__ void k_zero_u32(unsigned* p) { *p = 0u; }

void launch_max_abs(size_t n, const float* u, unsigned* out_bits, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, out_bits);
  if (n) hipLaunchKernelGGL(k_max_abs, dim3(nblocks(n)), dim3(kBlock), 0, s, (long)n, u, out_bits);
}

void launch_copy(const float* src, float* dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(nblocks(n)), dim3(kBlock), 0, s, src, dst, (long)n);
}

void launch_fill(float* p, size_t n, float v, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(kBlock), 0, s, p, (long)n, v);
}

void launch_advect(const Dims& d, double dx, double dt, const double* grav, const float* u, float* out,
                   double* trace, hipStream_t s) {
  hipLaunchKernelGGL(k_advect, dim3(nblocks(d.faces())), dim3(kBlock), 0, s, d, dt / dx, (float)grav[0],
                     (float)grav[1], (float)grav[2], (float)dt, u, out, trace);
}

// gin must hold zeros (the out-of-window taps are added to it first); trace
// holds the positions written by launch_advect for the same u.
void launch_advect_adjoint(const Dims& d, double dx, double dt, const float* u, const double* trace,
                           const float* gout, float* gin, float* stage, hipStream_t s) {
  const unsigned nb = (unsigned)(((d.nx + kBX - 1) / kBX) * ((d.ny + kBY - 1) / kBY) * ((d.nz + kBZ - 1) / kBZ));
  hipLaunchKernelGGL(k_advect_adjoint, dim3(nb), dim3(kAdjThreads), 0, s, d, dt / dx, u, trace, gout, gin, stage);
  hipLaunchKernelGGL(k_advect_adjoint_gather, dim3(nblocks(d.faces())), dim3(kBlock), 0, s, d, stage, gin);
}

}  // namespace nf
