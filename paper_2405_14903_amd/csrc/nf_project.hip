// Pressure projection with cut-cell fractions and its adjoint.
//
// NeuralFluid, Sec. Projection: with S = diag(alpha), k = dt/(rho dx),
//   Eq. projection_matrix:  k G^T S G P = G^T S U^ + G^T (I - S) U_s
//   Eq. u_next_matrix:      U^{n+1} = U^ - k G P
// (faces with alpha = 0 take the solid velocity).  The unit-scaled system
// (G^T S G) P = b / k is solved by the MGPCG in nf_solver.hip.
//
// The stored face velocity is the area average over the face's fluid and
// solid parts: U^{n+1} = alpha W + (1 - alpha) U_s with the fluid velocity
// W = U^ - k G P (Eq. u_next_matrix on fully fluid faces; the solid velocity
// on closed faces; continuous in alpha).
//
// Adjoint (Sec. Back-propagation through Time, Projection paragraph, and Sec.
// Back-propagation through Geometry), derived as the exact transpose of the
// forward with g = dJ/dU^{n+1}:
//   (G^T S G) y = -G^T S g          (the k factors cancel)
//   h = g + G y
//   dJ/dU^ = S h,  dJ/dU_s = (I - S) h,  dJ/dalpha_f = h_f (W_f - U_s,f)
// and dJ/dalpha, dJ/dU_s are carried to the ellipsoid's pose and controls
// through the marching-squares fraction and the rigid velocity field.
#include <algorithm>
#include <cmath>

#include "nf_internal.h"
#include "nf_shapes.h"

namespace nf {

__device__ inline void cell_decode(const Dims& d, long c, int& i, int& j, int& k) { cell_coords(d, c, i, j, k); }

// Flux alpha u + (1 - alpha) u_s through face f of component comp.
__device__ inline double face_flux(const Domain& D, const GeomParams& G, const float* __restrict__ alpha,
                                   const float* __restrict__ u, long f, int comp, int i, int j, int k) {
  float a = alpha[f];
  double fl = (double)a * (double)u[f];
  if (a < 1.0f) fl += (1.0 - (double)a) * face_solid_velocity(D, G, comp, i, j, k);
  return fl;
}

// b_c / k = (sum over lower faces - sum over upper faces of the flux) / k.
__global__ __launch_bounds__(kBlock) void k_rhs(Domain D, GeomParams G, float inv_k,
                                                 const float* __restrict__ alpha,
                                                 const float* __restrict__ uhat, float* __restrict__ b) {
  const Dims& d = D.d;
  long c = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (c >= (long)d.cells()) return;
  int i, j, k;
  cell_decode(d, c, i, j, k);
  long oy = (long)d.nfx(), oz = oy + (long)d.nfy();
  double s = face_flux(D, G, alpha, uhat, d.fx(i, j, k), 0, i, j, k) -
             face_flux(D, G, alpha, uhat, d.fx(i + 1, j, k), 0, i + 1, j, k) +
             face_flux(D, G, alpha, uhat, oy + d.fy(i, j, k), 1, i, j, k) -
             face_flux(D, G, alpha, uhat, oy + d.fy(i, j + 1, k), 1, i, j + 1, k) +
             face_flux(D, G, alpha, uhat, oz + d.fz(i, j, k), 2, i, j, k) -
             face_flux(D, G, alpha, uhat, oz + d.fz(i, j, k + 1), 2, i, j, k + 1);
  b[c] = (float)s * inv_k;
}

// Pressure of the cells on both sides of face (comp, i, j, k); 0 beyond the
// domain (the Dirichlet ghost; on WALL / INFLOW sides alpha = 0 hides it).
__device__ inline void face_cells(const Dims& d, const float* __restrict__ p, int comp, int i, int j,
                                  int k, float& pp, float& pm) {
  if (comp == 0) {
    pp = i < d.nx ? p[d.c(i, j, k)] : 0.0f;
    pm = i > 0 ? p[d.c(i - 1, j, k)] : 0.0f;
  } else if (comp == 1) {
    pp = j < d.ny ? p[d.c(i, j, k)] : 0.0f;
    pm = j > 0 ? p[d.c(i, j - 1, k)] : 0.0f;
  } else {
    pp = k < d.nz ? p[d.c(i, j, k)] : 0.0f;
    pm = k > 0 ? p[d.c(i, j, k - 1)] : 0.0f;
  }
}

__global__ __launch_bounds__(kBlock) void k_update(Domain D, GeomParams G, float kk,
                                                    const float* __restrict__ alpha,
                                                    const float* __restrict__ uhat,
                                                    const float* __restrict__ p, float* __restrict__ out) {
  const Dims& d = D.d;
  long f = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (f >= (long)d.faces()) return;
  int comp, i, j, k;
  face_decode(d, f, comp, i, j, k);
  const float a = alpha[f];
  float v = 0.0f;
  if (a > 0.0f) {
    float pp, pm;
    face_cells(d, p, comp, i, j, k, pp, pm);
    v = a * (uhat[f] - kk * (pp - pm));
  }
  if (a < 1.0f) v += (1.0f - a) * (float)face_solid_velocity(D, G, comp, i, j, k);
  out[f] = v;
}

// rhs_c = -(G^T S g)_c
__global__ __launch_bounds__(kBlock) void k_adj_div(Dims d, const float* __restrict__ alpha,
                                                     const float* __restrict__ g, float* __restrict__ rhs) {
  long c = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (c >= (long)d.cells()) return;
  int i, j, k;
  cell_decode(d, c, i, j, k);
  long oy = (long)d.nfx(), oz = oy + (long)d.nfy();
  long f[6] = {d.fx(i, j, k), d.fx(i + 1, j, k), oy + d.fy(i, j, k), oy + d.fy(i, j + 1, k),
               oz + d.fz(i, j, k), oz + d.fz(i, j, k + 1)};
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    float m = alpha[f[q]] * g[f[q]];
    s += (q & 1) ? -m : m;
  }
  rhs[c] = -s;
}

// ---- geometry partials (FP64) --------------------------------------------

__device__ inline double et(double a, double b) { return a / (a - b); }
__device__ inline void det(double a, double b, double& da, double& db) {
  double den = (a - b) * (a - b);
  da = -b / den;
  db = a / den;
}

// d alpha / d phi for the 4 cyclic corners (same cases as the forward).
__device__ inline void fraction_grad(const double p[4], double g[4]) {
  int f[4], cnt = 0;
  for (int q = 0; q < 4; ++q) {
    f[q] = p[q] > 0.0;
    cnt += f[q];
    g[q] = 0.0;
  }
  if (cnt == 0 || cnt == 4) return;
  if (cnt == 1 || cnt == 3) {
    int k = 0;
    for (int q = 0; q < 4; ++q)
      if (f[q] == (cnt == 1)) k = q;
    int kb = (k + 1) & 3, kd = (k + 3) & 3;
    double a = p[k], b = p[kb], dd = p[kd];
    double tb = et(a, b), td = et(a, dd), da1, db, da2, ddd;
    det(a, b, da1, db);
    det(a, dd, da2, ddd);
    double sg = cnt == 1 ? 0.5 : -0.5;
    g[k] = sg * (da1 * td + tb * da2);
    g[kb] = sg * db * td;
    g[kd] = sg * tb * ddd;
    return;
  }
  for (int k = 0; k < 4; ++k) {
    if (f[k] && f[(k + 1) & 3]) {
      int k1 = (k + 1) & 3, k2 = (k + 2) & 3, k3 = (k + 3) & 3;
      double d0, d3, d1, d2;
      det(p[k], p[k3], d0, d3);
      det(p[k1], p[k2], d1, d2);
      g[k] = 0.5 * d0;
      g[k3] = 0.5 * d3;
      g[k1] = 0.5 * d1;
      g[k2] = 0.5 * d2;
      return;
    }
  }
  int k = f[0] ? 0 : 1;
  int k1 = (k + 1) & 3, k2 = (k + 2) & 3, k3 = (k + 3) & 3;
  double a0 = p[k], a1 = p[k1], a2 = p[k2], a3 = p[k3];
  if (0.25 * (a0 + a1 + a2 + a3) > 0.0) {
    // 1 - 1/2 t(a1,a0) t(a1,a2) - 1/2 t(a3,a0) t(a3,a2)
    double s10 = et(a1, a0), s12 = et(a1, a2), s30 = et(a3, a0), s32 = et(a3, a2);
    double x1a, x0a, x1b, x2b, x3a, x0c, x3b, x2c;
    det(a1, a0, x1a, x0a);
    det(a1, a2, x1b, x2b);
    det(a3, a0, x3a, x0c);
    det(a3, a2, x3b, x2c);
    g[k1] = -0.5 * (x1a * s12 + s10 * x1b);
    g[k3] = -0.5 * (x3a * s32 + s30 * x3b);
    g[k] = -0.5 * (x0a * s12 + x0c * s32);
    g[k2] = -0.5 * (s10 * x2b + s30 * x2c);
  } else {
    // 1/2 t(a0,a1) t(a0,a3) + 1/2 t(a2,a1) t(a2,a3)
    double f01 = et(a0, a1), f03 = et(a0, a3), f21 = et(a2, a1), f23 = et(a2, a3);
    double y0a, y1a, y0b, y3b, y2a, y1b, y2b, y3c;
    det(a0, a1, y0a, y1a);
    det(a0, a3, y0b, y3b);
    det(a2, a1, y2a, y1b);
    det(a2, a3, y2b, y3c);
    g[k] = 0.5 * (y0a * f03 + f01 * y0b);
    g[k2] = 0.5 * (y2a * f23 + f21 * y2b);
    g[k1] = 0.5 * (y1a * f03 + f23 * y1b);
    g[k3] = 0.5 * (f01 * y3b + f21 * y3c);
  }
}

// d phi / d(c, a, R) of the ellipsoid distance estimate at x (15 values).
__device__ inline void ellipsoid_phi_grad(const GeomParams& G, double x, double y, double z, double out[15]) {
  double r[3] = {x - G.c[0], y - G.c[1], z - G.c[2]};
  double p[3], q[3], s[3];
  for (int jj = 0; jj < 3; ++jj) {
    p[jj] = G.R[0 + jj] * r[0] + G.R[3 + jj] * r[1] + G.R[6 + jj] * r[2];
    q[jj] = p[jj] / G.a[jj];
    s[jj] = q[jj] / G.a[jj];
  }
  double k0 = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
  double k1 = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  for (int t = 0; t < 15; ++t) out[t] = 0.0;
  if (k1 == 0.0 || k0 == 0.0) return;
  double dk0 = (2.0 * k0 - 1.0) / k1, dk1 = -k0 * (k0 - 1.0) / (k1 * k1);
  double gp[3];
  for (int jj = 0; jj < 3; ++jj) {
    double a = G.a[jj];
    gp[jj] = dk0 * q[jj] / (k0 * a) + dk1 * s[jj] / (k1 * a * a);
    out[3 + jj] = dk0 * (-q[jj] * q[jj] / (k0 * a)) + dk1 * (-2.0 * s[jj] * s[jj] / (k1 * a));
  }
  for (int ii = 0; ii < 3; ++ii) {
    out[ii] = -(G.R[3 * ii + 0] * gp[0] + G.R[3 * ii + 1] * gp[1] + G.R[3 * ii + 2] * gp[2]);
    for (int jj = 0; jj < 3; ++jj) out[6 + 3 * ii + jj] = r[ii] * gp[jj];
  }
}

__device__ inline void node_xyz(const Dims& d, double dx, int comp, int i, int j, int k, int q, double xyz[3]) {
  // cyclic corners: x-face (j,k) offsets, y-face (i,k), z-face (i,j)
  const int o1[4] = {0, 1, 1, 0}, o2[4] = {0, 0, 1, 1};
  int n[3] = {i, j, k};
  int t1 = comp == 0 ? 1 : 0, t2 = comp == 2 ? 1 : 2;
  n[t1] += o1[q];
  n[t2] += o2[q];
  xyz[0] = n[0] * dx;
  xyz[1] = n[1] * dx;
  xyz[2] = n[2] * dx;
}

__device__ inline int corner_node(const Dims& d, int comp, int i, int j, int k, int q) {
  const int o1[4] = {0, 1, 1, 0}, o2[4] = {0, 0, 1, 1};
  int n[3] = {i, j, k};
  int t1 = comp == 0 ? 1 : 0, t2 = comp == 2 ? 1 : 2;
  n[t1] += o1[q];
  n[t2] += o2[q];
  return d.node(n[0], n[1], n[2]);
}

// Lattice index box per face component: faces lo[c][m] .. lo[c][m] + ext[c][m] - 1
// along axis m; start[c] = first flat thread index of component c.
struct FaceBox {
  int lo[3][3];
  int ext[3][3];
  long start[4];
};

// Per face: dJ/dU^ = alpha h, h = g + G y.
__global__ __launch_bounds__(kBlock) void k_adj_faces(Dims d, const float* __restrict__ alpha,
                                                       const float* __restrict__ g, const float* __restrict__ y,
                                                       float* __restrict__ gu) {
  const long f = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (f >= (long)d.faces()) return;
  int comp, i, j, k;
  face_decode(d, f, comp, i, j, k);
  float yp, ym;
  face_cells(d, y, comp, i, j, k, yp, ym);
  gu[f] = alpha[f] * (g[f] + (yp - ym));
}

// The ellipsoid's pose (15) and control (6) partials, reduced in a fixed
// order in FP64.  Only faces with alpha < 1 contribute, and those have a
// corner node inside the closed ellipsoid, so the kernel walks the faces of
// the ellipsoid's bounding box (FaceBox) only.  uhat and p are the step's
// advected field and pressure (for W on cut faces).
__global__ __launch_bounds__(kBlock) void k_adj_geom(Domain D, GeomParams G, FaceBox B, float kk,
                                                      const float* __restrict__ alpha,
                                                      const double* __restrict__ phi,
                                                      const float* __restrict__ g,
                                                      const float* __restrict__ y,
                                                      const float* __restrict__ uhat,
                                                      const float* __restrict__ p, double* __restrict__ partials) {
  const Dims& d = D.d;
  double acc[21];
#pragma unroll
  for (int t = 0; t < 21; ++t) acc[t] = 0.0;
  const long oy = (long)d.nfx(), oz = oy + (long)d.nfy();
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < B.start[3]; t += (long)gridDim.x * blockDim.x) {
    const int comp = t < B.start[1] ? 0 : (t < B.start[2] ? 1 : 2);
    // per-component box values, selected as registers (see uniform_value)
    auto pick = [&](int v0, int v1, int v2) {
      const int a = uniform_value(v0), b = uniform_value(v1), c = uniform_value(v2);
      return comp == 0 ? a : (comp == 1 ? b : c);
    };
    const long lt = t - (comp == 0 ? 0 : (comp == 1 ? B.start[1] : B.start[2]));
    const int ex = pick(B.ext[0][0], B.ext[1][0], B.ext[2][0]), ey = pick(B.ext[0][1], B.ext[1][1], B.ext[2][1]);
    const int i = pick(B.lo[0][0], B.lo[1][0], B.lo[2][0]) + (int)(lt % ex);
    const int j = pick(B.lo[0][1], B.lo[1][1], B.lo[2][1]) + (int)((lt / ex) % ey);
    const int k = pick(B.lo[0][2], B.lo[1][2], B.lo[2][2]) + (int)(lt / ((long)ex * ey));
    const long f = comp == 0 ? (long)d.fx(i, j, k) : (comp == 1 ? oy + d.fy(i, j, k) : oz + d.fz(i, j, k));
    const float a = alpha[f];
    if (!(a < 1.0f)) continue;
    const int own = comp == 0 ? i : (comp == 1 ? j : k);
    const int sk = side_kind(D, comp, own);
    if (sk == SIM_BC_WALL || sk == SIM_BC_INFLOW) continue;
    float yp, ym;
    face_cells(d, y, comp, i, j, k, yp, ym);
    const float hf = g[f] + (yp - ym);
    if (hf == 0.0f) continue;
    const double us = face_solid_velocity(D, G, comp, i, j, k);
    if (a > 0.0f) {
      // dJ/dalpha = h (W - U_s), W = U^ - k G P
      float pp, pm;
      face_cells(d, p, comp, i, j, k, pp, pm);
      const double W = (double)uhat[f] - (double)kk * ((double)pp - (double)pm);
      const double galpha = (double)hf * (W - us);
      double ph[4], dg[4];
      for (int q = 0; q < 4; ++q) ph[q] = phi[corner_node(d, comp, i, j, k, q)];
      fraction_grad(ph, dg);
      for (int q = 0; q < 4; ++q) {
        if (dg[q] == 0.0) continue;
        double xyz[3], gp[15];
        node_xyz(d, D.dx, comp, i, j, k, q, xyz);
        ellipsoid_phi_grad(G, xyz[0], xyz[1], xyz[2], gp);
        const double w = galpha * dg[q];
#pragma unroll
        for (int s = 0; s < 15; ++s) acc[s] += w * gp[s];
      }
    }
    // dJ/dU_s = (1 - alpha) h, through u_s = v + w x (x - c)
    const double gus = (1.0 - (double)a) * (double)hf;
    const double x0 = (i + (comp == 0 ? 0.0 : 0.5)) * D.dx, x1 = (j + (comp == 1 ? 0.0 : 0.5)) * D.dx,
                 x2 = (k + (comp == 2 ? 0.0 : 0.5)) * D.dx;
    const double r0 = x0 - G.c[0], r1 = x1 - G.c[1], r2 = x2 - G.c[2];
    if (comp == 0) {
      acc[15] += gus;
      acc[19] += gus * r2;  acc[20] -= gus * r1;       // d/dw
      acc[1] += gus * G.w[2]; acc[2] -= gus * G.w[1];  // d/dc = -d/dr
    } else if (comp == 1) {
      acc[16] += gus;
      acc[18] -= gus * r2;  acc[20] += gus * r0;
      acc[0] -= gus * G.w[2]; acc[2] += gus * G.w[0];
    } else {
      acc[17] += gus;
      acc[18] += gus * r1;  acc[19] -= gus * r0;
      acc[0] += gus * G.w[1]; acc[1] -= gus * G.w[0];
    }
  }
  block_partials<21>(acc, partials);
}

// One block per partial: fixed-order total, added to g_theta (0..14) or g_ctrl (15..20).
__global__ __launch_bounds__(kFinBlock) void k_fin_adj_geom(int nb, const double* __restrict__ partials,
                                                             double* __restrict__ g_theta,
                                                             double* __restrict__ g_ctrl) {
  const int q = blockIdx.x;
  double tot[1];
  finish_partials<1>(partials + (size_t)q * nb, nb, tot);
  if (threadIdx.x == 0) {
    if (q < 15) {
      if (g_theta) g_theta[q] += tot[0];
    } else if (g_ctrl) {
      g_ctrl[q - 15] += tot[0];
    }
  }
}

// ---- the B-spline wall's knot gradient (FP64, fixed order) --------------
//
// dJ/da_mn = -amp s sum_nodes dJ/dphi_node B_m(y) B_n(z)
//            + amp s' sum_(x faces) dJ/du_s,f B_m(y_f) B_n(z_f),
// phi = x - d depending on (y, z) only, so both sums first collapse along x
// into per-column totals (k_adj_wall_cols), which each knot then weights over
// its 4 x 4 support (k_adj_wall_knots).  Faces with alpha < 1 have a corner
// with phi <= 0, i.e. x <= max d: only the x range up to G.wall_imax
// contributes.

// dJ/dalpha of face (comp, i, j, k), or 0 where the face does not contribute
// (alpha = 1, a WALL / INFLOW side, or alpha = 0, whose corners are all solid
// so that d alpha / d phi = 0); also dJ/du_s = (1 - alpha) h.
__device__ inline bool wall_face_terms(const Domain& D, const GeomParams& G, float kk, const float* alpha,
                                       const float* g, const float* y, const float* uhat, const float* p, int comp,
                                       int i, int j, int k, double& galpha, double& gus) {
  const Dims& d = D.d;
  galpha = gus = 0.0;
  if (i < 0 || j < 0 || k < 0) return false;
  if (comp == 0 ? (i > d.nx || j >= d.ny || k >= d.nz)
                : (comp == 1 ? (i >= d.nx || j > d.ny || k >= d.nz) : (i >= d.nx || j >= d.ny || k > d.nz)))
    return false;
  const long oy = (long)d.nfx(), oz = oy + (long)d.nfy();
  const long f = comp == 0 ? (long)d.fx(i, j, k) : (comp == 1 ? oy + d.fy(i, j, k) : oz + d.fz(i, j, k));
  const float a = alpha[f];
  if (!(a < 1.0f)) return false;
  const int own = comp == 0 ? i : (comp == 1 ? j : k);
  const int sk = side_kind(D, comp, own);
  if (sk == SIM_BC_WALL || sk == SIM_BC_INFLOW) return false;
  float yp, ym;
  face_cells(d, y, comp, i, j, k, yp, ym);
  const float hf = g[f] + (yp - ym);
  if (hf == 0.0f) return false;
  const double us = face_solid_velocity(D, G, comp, i, j, k);
  if (a > 0.0f) {
    float pp, pm;
    face_cells(d, p, comp, i, j, k, pp, pm);
    const double W = (double)uhat[f] - (double)kk * ((double)pp - (double)pm);
    galpha = (double)hf * (W - us);
  }
  gus = (1.0 - (double)a) * (double)hf;
  return true;
}

// dJ/dphi at node (i, j, k) from its face (comp, fi, fj, fk), where the node
// is the face's cyclic corner q.
__device__ inline double wall_corner_term(const Domain& D, const GeomParams& G, float kk, const float* alpha,
                                          const double* phi, const float* g, const float* y, const float* uhat,
                                          const float* p, int comp, int fi, int fj, int fk, int q) {
  double galpha, gus;
  if (!wall_face_terms(D, G, kk, alpha, g, y, uhat, p, comp, fi, fj, fk, galpha, gus) || galpha == 0.0) return 0.0;
  double ph[4], dg[4];
  for (int c = 0; c < 4; ++c) ph[c] = phi[corner_node(D.d, comp, fi, fj, fk, c)];
  fraction_grad(ph, dg);
  return galpha * dg[q];
}

// dJ/dphi at node (i, j, k), gathered from its 12 faces in a fixed order
// (the node is corner 0 of the face at (i, j, k) and corners 1 .. 3 of the
// faces one step down along the face's two tangents).
__device__ inline double node_phi_adjoint(const Domain& D, const GeomParams& G, float kk, const float* alpha,
                                          const double* phi, const float* g, const float* y, const float* uhat,
                                          const float* p, int i, int j, int k) {
  double sn = 0.0;
  // x faces (tangents y, z): corners (j,k), (j+1,k), (j+1,k+1), (j,k+1)
  sn += wall_corner_term(D, G, kk, alpha, phi, g, y, uhat, p, 0, i, j, k, 0);
  sn += wall_corner_term(D, G, kk, alpha, phi, g, y, uhat, p, 0, i, j - 1, k, 1);
  sn += wall_corner_term(D, G, kk, alpha, phi, g, y, uhat, p, 0, i, j - 1, k - 1, 2);
  sn += wall_corner_term(D, G, kk, alpha, phi, g, y, uhat, p, 0, i, j, k - 1, 3);
  // y faces (tangents x, z)
  sn += wall_corner_term(D, G, kk, alpha, phi, g, y, uhat, p, 1, i, j, k, 0);
  sn += wall_corner_term(D, G, kk, alpha, phi, g, y, uhat, p, 1, i - 1, j, k, 1);
  sn += wall_corner_term(D, G, kk, alpha, phi, g, y, uhat, p, 1, i - 1, j, k - 1, 2);
  sn += wall_corner_term(D, G, kk, alpha, phi, g, y, uhat, p, 1, i, j, k - 1, 3);
  // z faces (tangents x, y)
  sn += wall_corner_term(D, G, kk, alpha, phi, g, y, uhat, p, 2, i, j, k, 0);
  sn += wall_corner_term(D, G, kk, alpha, phi, g, y, uhat, p, 2, i - 1, j, k, 1);
  sn += wall_corner_term(D, G, kk, alpha, phi, g, y, uhat, p, 2, i - 1, j - 1, k, 2);
  sn += wall_corner_term(D, G, kk, alpha, phi, g, y, uhat, p, 2, i, j - 1, k, 3);
  return sn;
}

// One thread per node column (j, k): cn[j + (ny+1) k] = sum over x of
// dJ/dphi at the column's nodes; cf[j + ny k] (j < ny, k < nz) = sum over x of
// dJ/du_s at the column's x faces.
__global__ __launch_bounds__(kBlock) void k_adj_wall_cols(Domain D, GeomParams G, float kk,
                                                           const float* __restrict__ alpha,
                                                           const double* __restrict__ phi,
                                                           const float* __restrict__ g,
                                                           const float* __restrict__ y,
                                                           const float* __restrict__ uhat,
                                                           const float* __restrict__ p, double* __restrict__ cn,
                                                           double* __restrict__ cf) {
  const Dims& d = D.d;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)(d.ny + 1) * (d.nz + 1)) return;
  const int j = (int)(t % (d.ny + 1)), k = (int)(t / (d.ny + 1));
  const int ilast = min(d.nx, G.wall_imax + 1);
  double sn = 0.0, sf = 0.0;
  for (int i = 0; i <= ilast; ++i) {
    sn += node_phi_adjoint(D, G, kk, alpha, phi, g, y, uhat, p, i, j, k);
    if (j < d.ny && k < d.nz) {
      double galpha, gus;
      if (wall_face_terms(D, G, kk, alpha, g, y, uhat, p, 0, i, j, k, galpha, gus)) sf += gus;
    }
  }
  cn[t] = sn;
  if (j < d.ny && k < d.nz) cf[j + (long)d.ny * k] = sf;
}

// One block per control amplitude (m, n): its bases' weights over the column
// totals within its support, added to g_theta[m * SIM_WALL_KNOTS_Z + n].
__global__ __launch_bounds__(kBlock) void k_adj_wall_knots(Domain D, GeomParams G, const double* __restrict__ cn,
                                                            const double* __restrict__ cf,
                                                            double* __restrict__ g_theta) {
  const Dims& d = D.d;
  const int m = blockIdx.x / SIM_WALL_KNOTS_Z, n = blockIdx.x % SIM_WALL_KNOTS_Z;
  const double sy = G.ly / (SIM_WALL_KNOTS_Y - 3), sz = G.lz / (SIM_WALL_KNOTS_Z - 3);
  // nodes and faces with |position / spacing - (m - 1)| < 2
  const int jlo = max(0, (int)floor((m - 3) * sy / D.dx)), jhi = min(d.ny, (int)ceil((m + 1) * sy / D.dx));
  const int klo = max(0, (int)floor((n - 3) * sz / D.dx)), khi = min(d.nz, (int)ceil((n + 1) * sz / D.dx));
  const int wj = jhi - jlo + 1, wk = khi - klo + 1;
  double v[2] = {0.0, 0.0};
  for (int q = threadIdx.x; q < wj * wk; q += blockDim.x) {
    const int j = jlo + q % wj, k = klo + q / wj;
    const double by = bspline3(j * D.dx / sy - (m - 1)), bz = bspline3(k * D.dx / sz - (n - 1));
    v[0] += cn[j + (long)(d.ny + 1) * k] * by * bz;
    if (j < d.ny && k < d.nz) {
      const double fy = bspline3((j + 0.5) * D.dx / sy - (m - 1)), fz = bspline3((k + 0.5) * D.dx / sz - (n - 1));
      v[1] += cf[j + (long)d.ny * k] * fy * fz;
    }
  }
  __shared__ double sh[2 * (kBlock / 64) + 1];
  block_sum<2, kBlock>(v, sh);
  if (threadIdx.x == 0) g_theta[blockIdx.x] += -G.amp * G.wall_s * v[0] + G.amp * G.wall_sd * v[1];
}

// ---- the parametric solids' parameter gradient (FP64, fixed order) -------
//
// dJ/dtheta_q = sum over nodes whose CSG term is solid q of dJ/dphi_node
// d(distance to q)/dtheta_q.  Block row blockIdx.y = q walks q's node box
// (nodes outside it have dJ/dphi = 0 or another CSG term); the term of every
// node was recorded by the forward geometry kernel (a node with a nonzero
// dJ/dphi is a corner of a cut face, never in the far field).  Partials:
// partials[(q * kShapeParams + s) * gridDim.x + blockIdx.x].
__global__ __launch_bounds__(kBlock) void k_adj_solids(Domain D, GeomParams G, float kk,
                                                        const float* __restrict__ alpha,
                                                        const double* __restrict__ phi,
                                                        const float* __restrict__ g,
                                                        const float* __restrict__ y,
                                                        const float* __restrict__ uhat,
                                                        const float* __restrict__ p, double* __restrict__ partials) {
  const int q = blockIdx.y;
  const int* box = G.sbox[q];
  const int ex = box[3], ey = box[4], ez = box[5];
  const long total = (long)ex * ey * ez;
  const double* dirs = G.solids;
  const double* S = G.solids + kShapeHead + (size_t)q * kShapeStride;
  double acc[kShapeParams];
#pragma unroll
  for (int t = 0; t < kShapeParams; ++t) acc[t] = 0.0;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int i = box[0] + (int)(t % ex);
    const int j = box[1] + (int)((t / ex) % ey);
    const int k = box[2] + (int)(t / ((long)ex * ey));
    // the node's CSG term, recorded by the forward geometry kernel
    if (G.solid_term[D.d.node(i, j, k)] != (unsigned char)q) continue;
    const double gphi = node_phi_adjoint(D, G, kk, alpha, phi, g, y, uhat, p, i, j, k);
    if (gphi == 0.0) continue;
    solid_distance_grad(dirs, S, i * D.dx, j * D.dx, k * D.dx, gphi, acc);
  }
  block_partials<kShapeParams>(acc, partials + (size_t)q * kShapeParams * gridDim.x);
}

// One block per (parameter, solid): fixed-order total added to g_theta.
__global__ __launch_bounds__(kFinBlock) void k_fin_adj_solids(int nb, int m, const double* __restrict__ partials,
                                                               double* __restrict__ g_theta) {
  const int s = blockIdx.x, q = blockIdx.y;
  double tot[1];
  finish_partials<1>(partials + ((size_t)q * kShapeParams + s) * nb, nb, tot);
  if (threadIdx.x == 0) g_theta[1 + m + (size_t)q * kShapeParams + s] += tot[0];
}

constexpr int kSolidBlocks = 512;   // blocks per solid of the gradient walk (at most)
size_t solids_partials_doubles() { return (size_t)SIM_MAX_SOLIDS * kShapeParams * kSolidBlocks; }

// J = scale * sum over the outlet faces (z faces with k = nz) of w u; g = scale w
// there, 0 elsewhere (w = 1 when no weights are given).
__global__ __launch_bounds__(kBlock) void k_loss_outlet(Dims d, double scale, const float* __restrict__ w,
                                                         const float* __restrict__ u, float* __restrict__ g,
                                                         double* __restrict__ partials) {
  const long f = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double v[1] = {0.0};
  if (f < (long)d.faces()) {
    const long o = (long)d.nfx() + (long)d.nfy() + (long)d.nx * d.ny * d.nz;   // first outlet face
    if (f >= o) {
      const long q = f - o;
      const double wf = w ? (double)w[q] : 1.0;
      g[f] = (float)(scale * wf);
      v[0] = scale * wf * (double)u[f];
    } else {
      g[f] = 0.0f;
    }
  }
  block_partials<1>(v, partials);
}

// J = sum of u_f^2 over faces whose centre lies in [lo, hi]; g = 2 u there.
// Grid-stride over the faces with at most kLossBlocks blocks, so the partial
// sums never need more than kLossBlocks doubles.
__global__ __launch_bounds__(kBlock) void k_loss_box(Domain D, double lo0, double lo1, double lo2, double hi0,
                                                      double hi1, double hi2, const float* __restrict__ u,
                                                      float* __restrict__ g, double* __restrict__ partials) {
  const Dims& d = D.d;
  const long nf = (long)d.faces();
  double v[1] = {0.0};
  for (long f = (long)blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += (long)gridDim.x * blockDim.x) {
    int comp, i, j, k;
    face_decode(d, f, comp, i, j, k);
    double x = (i + (comp == 0 ? 0.0 : 0.5)) * D.dx, y = (j + (comp == 1 ? 0.0 : 0.5)) * D.dx,
           z = (k + (comp == 2 ? 0.0 : 0.5)) * D.dx;
    const double eps = 1e-12;
    bool in = x >= lo0 - eps && x <= hi0 + eps && y >= lo1 - eps && y <= hi1 + eps && z >= lo2 - eps &&
              z <= hi2 + eps;
    float uf = u[f];
    g[f] = in ? 2.0f * uf : 0.0f;
    v[0] += in ? (double)uf * (double)uf : 0.0;
  }
  block_partials<1>(v, partials);
}

__global__ __launch_bounds__(kFinBlock) void k_fin_loss(int nb, const double* __restrict__ partials,
                                                         double* __restrict__ J) {
  double tot[1];
  finish_partials<1>(partials, nb, tot);
  if (threadIdx.x == 0) *J = tot[0];
}

static inline unsigned nblocks(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int loss_box_blocks(const Dims& d) {
  const unsigned nb = nblocks(d.faces());
  return (int)(nb < (unsigned)kLossBlocks ? nb : (unsigned)kLossBlocks);
}

void launch_loss_box(const Domain& D, const double* lo, const double* hi, const float* u, double* J, float* g,
                     double* partials, hipStream_t s) {
  const int nb = loss_box_blocks(D.d);
  hipLaunchKernelGGL(k_loss_box, dim3(nb), dim3(kBlock), 0, s, D, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], u, g,
                     partials);
  hipLaunchKernelGGL(k_fin_loss, dim3(1), dim3(kFinBlock), 0, s, nb, partials, J);
}

void launch_rhs(const Domain& D, const GeomParams& G, double inv_k, const float* alpha, const float* uhat,
                float* b, hipStream_t s) {
  hipLaunchKernelGGL(k_rhs, dim3(nblocks(D.d.cells())), dim3(kBlock), 0, s, D, G, (float)inv_k, alpha, uhat, b);
}

void launch_update(const Domain& D, const GeomParams& G, double kk, const float* alpha, const float* uhat,
                   const float* p, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(nblocks(D.d.faces())), dim3(kBlock), 0, s, D, G, (float)kk, alpha, uhat,
                     p, out);
}

void launch_adj_div(const Dims& d, const float* alpha, const float* g, float* rhs, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_div, dim3(nblocks(d.cells())), dim3(kBlock), 0, s, d, alpha, g, rhs);
}

size_t adj_faces_partials(const Dims& d) { return (size_t)nblocks(d.faces()) * 21; }

// Faces that can have alpha < 1: a corner node inside the closed ellipsoid
// x = c + R diag(a) u, |u| <= 1, whose extent along world axis m is
// sqrt(sum_j (R_mj a_j)^2); two cells of margin on each side.
FaceBox ellipsoid_face_box(const Dims& d, double dx, const GeomParams& G) {
  FaceBox B;
  const int n[3] = {d.nx, d.ny, d.nz};
  int lo[3], hi[3];
  for (int m = 0; m < 3; ++m) {
    double e2 = 0.0;
    for (int j = 0; j < 3; ++j) e2 += (G.R[3 * m + j] * G.a[j]) * (G.R[3 * m + j] * G.a[j]);
    const double e = std::sqrt(e2);
    const double l = std::floor((G.c[m] - e) / dx) - 2.0, h = std::ceil((G.c[m] + e) / dx) + 2.0;
    lo[m] = (int)std::max(0.0, std::min((double)n[m] + 1.0, l));
    hi[m] = (int)std::max(0.0, std::min((double)n[m] + 1.0, h + 1.0));
  }
  long tot = 0;
  for (int c = 0; c < 3; ++c) {
    B.start[c] = tot;
    long cnt = 1;
    for (int m = 0; m < 3; ++m) {
      const int size = n[m] + (m == c ? 1 : 0);
      const int l = std::min(lo[m], size), h = std::min(hi[m], size);
      B.lo[c][m] = l;
      B.ext[c][m] = std::max(0, h - l);
      cnt *= B.ext[c][m];
    }
    tot += cnt;
  }
  B.start[3] = tot;
  return B;
}

void launch_loss_outlet(const Dims& d, double scale, const float* w, const float* u, double* J, float* g,
                        double* partials, hipStream_t s) {
  const int nb = (int)nblocks(d.faces());
  hipLaunchKernelGGL(k_loss_outlet, dim3(nb), dim3(kBlock), 0, s, d, scale, w, u, g, partials);
  hipLaunchKernelGGL(k_fin_loss, dim3(1), dim3(kFinBlock), 0, s, nb, partials, J);
}

size_t wall_column_doubles(const Dims& d) { return (size_t)(d.ny + 1) * (d.nz + 1) + (size_t)d.ny * d.nz; }

void launch_adj_faces(const Domain& D, const GeomParams& G, bool grad, double kk, const float* alpha,
                      const double* phi, const float* g, const float* y, const float* uhat, const float* p,
                      float* gu, double* partials, double* g_theta, double* g_ctrl, double* geom_scratch,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_adj_faces, dim3(nblocks(D.d.faces())), dim3(kBlock), 0, s, D.d, alpha, g, y, gu);
  if (!grad) return;
  if (G.kind == SIM_GEOM_BEZIER) {
    if (!g_theta) return;
    long most = 1;
    for (int q = 0; q < G.nsolid; ++q) most = std::max(most, (long)G.sbox[q][3] * G.sbox[q][4] * G.sbox[q][5]);
    const int nb = (int)std::min<size_t>(nblocks((size_t)most), kSolidBlocks);
    hipLaunchKernelGGL(k_adj_solids, dim3(nb, G.nsolid), dim3(kBlock), 0, s, D, G, (float)kk, alpha, phi, g, y, uhat,
                       p, geom_scratch);
    hipLaunchKernelGGL(k_fin_adj_solids, dim3(kShapeParams, G.nsolid), dim3(kFinBlock), 0, s, nb, G.nsolid,
                       geom_scratch, g_theta);
    return;
  }
  if (G.kind == SIM_GEOM_WALL) {
    if (!g_theta) return;
    double* cn = geom_scratch;
    double* cf = geom_scratch + (size_t)(D.d.ny + 1) * (D.d.nz + 1);
    hipLaunchKernelGGL(k_adj_wall_cols, dim3(nblocks((size_t)(D.d.ny + 1) * (D.d.nz + 1))), dim3(kBlock), 0, s, D,
                       G, (float)kk, alpha, phi, g, y, uhat, p, cn, cf);
    hipLaunchKernelGGL(k_adj_wall_knots, dim3(SIM_WALL_KNOTS_Y * SIM_WALL_KNOTS_Z), dim3(kBlock), 0, s, D, G, cn,
                       cf, g_theta);
    return;
  }
  const FaceBox B = ellipsoid_face_box(D.d, D.dx, G);
  if (B.start[3] == 0) return;
  // a bounded grid with a grid-stride loop keeps the partial count small
  const int nb = (int)std::min<size_t>(nblocks((size_t)B.start[3]), 1024);
  hipLaunchKernelGGL(k_adj_geom, dim3(nb), dim3(kBlock), 0, s, D, G, B, (float)kk, alpha, phi, g, y, uhat, p,
                     partials);
  hipLaunchKernelGGL(k_fin_adj_geom, dim3(21), dim3(kFinBlock), 0, s, nb, partials, g_theta, g_ctrl);
}

}  // namespace nf
