// Geometry: signed distance at grid nodes, per-face fluid fractions by 2D
// marching squares, and the multigrid hierarchy of face fractions.
//
// NeuralFluid, Sec. Projection (cut-cell paragraph): alpha_f is the fluid
// share of face f, from the zero contour of the solid SDF phi (phi > 0 fluid)
// intersected with the face; the printed one-fluid-corner case is
// alpha = 1/2 * phi_A/(phi_A - phi_B) * phi_A/(phi_A - phi_D).  The other
// corner configurations use the same linear edge intersections; a saddle is
// resolved by the sign of the corner mean.  phi and alpha are evaluated in
// FP64 so that the decision alpha > 0 (which selects the update of a face) is
// taken in double precision; alpha is then stored in FP32 and never rounded
// down to zero when positive.
#include <algorithm>
#include <cmath>

#include "nf_internal.h"
#include "nf_shapes.h"

namespace nf {

__device__ inline double phi_at(const GeomParams& G, double x, double y, double z) {
  if (G.kind == SIM_GEOM_SPHERES) {
    double best = 1e300;
    for (int s = 0; s < G.nsph; ++s) {
      double dx = x - G.sph[4 * s], dy = y - G.sph[4 * s + 1], dz = z - G.sph[4 * s + 2];
      double d = sqrt(dx * dx + dy * dy + dz * dz) - G.sph[4 * s + 3];
      best = d < best ? d : best;
    }
    return best;
  }
  if (G.kind == SIM_GEOM_ELLIPSOID) {
    double r0 = x - G.c[0], r1 = y - G.c[1], r2 = z - G.c[2];
    // p = R^T r (R maps body to world)
    double p0 = G.R[0] * r0 + G.R[3] * r1 + G.R[6] * r2;
    double p1 = G.R[1] * r0 + G.R[4] * r1 + G.R[7] * r2;
    double p2 = G.R[2] * r0 + G.R[5] * r1 + G.R[8] * r2;
    double q0 = p0 / G.a[0], q1 = p1 / G.a[1], q2 = p2 / G.a[2];
    double s0 = q0 / G.a[0], s1 = q1 / G.a[1], s2 = q2 / G.a[2];
    double k0 = sqrt(q0 * q0 + q1 * q1 + q2 * q2);
    double k1 = sqrt(s0 * s0 + s1 * s1 + s2 * s2);
    if (k1 == 0.0) {
      double m = G.a[0] < G.a[1] ? G.a[0] : G.a[1];
      return -(m < G.a[2] ? m : G.a[2]);
    }
    return k0 * (k0 - 1.0) / k1;
  }
  if (G.kind == SIM_GEOM_WALL) return x - G.amp * G.wall_s * wall_h(G, y, z);
  return 1.0;
}

__global__ void k_phi_nodes(Dims d, double dx, GeomParams G, double* __restrict__ phi) {
  long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)d.nodes();
  if (n >= total) return;
  int i, j, k;
  node_coords(d, n, i, j, k);
  phi[n] = phi_at(G, i * dx, j * dx, k * dx);
}

// phi of the parametric-solid scene at every node (its own kernel: the
// per-node work is m polygon walks, read from the packed solids).
__global__ __launch_bounds__(kBlock) void k_phi_solids(Dims d, double dx, GeomParams G, double* __restrict__ phi) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= (long)d.nodes()) return;
  int i, j, k;
  node_coords(d, n, i, j, k);
  unsigned char term;
  phi[n] = scene_phi_fast(G.solids, G.nsolid, G.solid_far, i * dx, j * dx, k * dx, term);
  G.solid_term[n] = term;
}

// Fraction along an edge from the corner with value a to the sign change.
__device__ inline double edge_t(double a, double b) { return a / (a - b); }

// Marching-squares fluid fraction of a face with cyclic corner values p[0..3].
__device__ inline double face_fraction(const double p[4]) {
  int f[4], cnt = 0;
  for (int q = 0; q < 4; ++q) {
    f[q] = p[q] > 0.0;
    cnt += f[q];
  }
  if (cnt == 0) return 0.0;
  if (cnt == 4) return 1.0;
  if (cnt == 1 || cnt == 3) {
    // the odd corner k: fluid if cnt == 1, solid if cnt == 3
    int k = 0;
    for (int q = 0; q < 4; ++q)
      if (f[q] == (cnt == 1)) k = q;
    double a = p[k], b = p[(k + 1) & 3], dd = p[(k + 3) & 3];
    double tri = 0.5 * edge_t(a, b) * edge_t(a, dd);
    return cnt == 1 ? tri : 1.0 - tri;
  }
  // two fluid corners
  for (int k = 0; k < 4; ++k) {
    if (f[k] && f[(k + 1) & 3]) {
      double a0 = p[k], a1 = p[(k + 1) & 3], a2 = p[(k + 2) & 3], a3 = p[(k + 3) & 3];
      return 0.5 * (edge_t(a0, a3) + edge_t(a1, a2));
    }
  }
  // diagonal pair: k and k+2 fluid
  int k = f[0] ? 0 : 1;
  double a0 = p[k], a1 = p[(k + 1) & 3], a2 = p[(k + 2) & 3], a3 = p[(k + 3) & 3];
  double mean = 0.25 * (a0 + a1 + a2 + a3);
  if (mean > 0.0)
    return 1.0 - 0.5 * edge_t(a1, a0) * edge_t(a1, a2) - 0.5 * edge_t(a3, a0) * edge_t(a3, a2);
  return 0.5 * edge_t(a0, a1) * edge_t(a0, a3) + 0.5 * edge_t(a2, a1) * edge_t(a2, a3);
}

// Cyclic corner node values of face (comp, i, j, k).
__device__ inline void face_corners(const Dims& d, const double* __restrict__ phi, int comp, int i,
                                    int j, int k, double p[4]) {
  if (comp == 0) {
    p[0] = phi[d.node(i, j, k)];
    p[1] = phi[d.node(i, j + 1, k)];
    p[2] = phi[d.node(i, j + 1, k + 1)];
    p[3] = phi[d.node(i, j, k + 1)];
  } else if (comp == 1) {
    p[0] = phi[d.node(i, j, k)];
    p[1] = phi[d.node(i + 1, j, k)];
    p[2] = phi[d.node(i + 1, j, k + 1)];
    p[3] = phi[d.node(i, j, k + 1)];
  } else {
    p[0] = phi[d.node(i, j, k)];
    p[1] = phi[d.node(i + 1, j, k)];
    p[2] = phi[d.node(i + 1, j + 1, k)];
    p[3] = phi[d.node(i, j + 1, k)];
  }
}

__device__ inline float store_fraction(double a) {
  float f = (float)a;
  if (a > 0.0 && !(f > 0.0f)) f = 1.17549435e-38f;  // keep alpha > 0 decisions exact
  return f;
}

__global__ void k_alpha(Domain D, const double* __restrict__ phi, float* __restrict__ alpha) {
  long f = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= (long)D.d.faces()) return;
  int comp, i, j, k;
  face_decode(D.d, f, comp, i, j, k);
  int own = comp == 0 ? i : (comp == 1 ? j : k);
  int sk = side_kind(D, comp, own);
  if (sk == SIM_BC_WALL || sk == SIM_BC_INFLOW) {
    alpha[f] = 0.0f;
    return;
  }
  double p[4];
  face_corners(D.d, phi, comp, i, j, k, p);
  alpha[f] = store_fraction(face_fraction(p));
}

// Inverse diagonal of G^T S G on one level: 1 / sum(alpha over the 6 faces), 0
// for inactive cells.
__global__ void k_invdiag(Dims d, const float* __restrict__ ax, const float* __restrict__ ay,
                          const float* __restrict__ az, float* __restrict__ invd) {
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)d.cells()) return;
  int i, j, k;
  cell_coords(d, c, i, j, k);
  float s = ax[d.fx(i, j, k)] + ax[d.fx(i + 1, j, k)] + ay[d.fy(i, j, k)] + ay[d.fy(i, j + 1, k)] +
            az[d.fz(i, j, k)] + az[d.fz(i, j, k + 1)];
  invd[c] = s > 0.0f ? 1.0f / s : 0.0f;
}

static inline unsigned nblocks(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

size_t solids_buffer_doubles() { return shape_buffer_doubles(); }

int pack_solids(const sim_desc& d, const double* theta, double* host, GeomParams& G) {
  if (!theta) return SIM_EINVAL;
  const int m = (d.n_params - 1) / (1 + kShapeParams);
  for (int t = 0; t < d.n_params; ++t)
    if (!std::isfinite(theta[t])) return SIM_EINVAL;
  if (theta[0] != (double)m) return SIM_EINVAL;
  for (int q = 0; q < m; ++q)
    if (theta[1 + q] != 0.0 && theta[1 + q] != 1.0) return SIM_EINVAL;
  // unit vectors of the control angles: segment s's two inner control points
  // sit 2 pi / (3N) inside [2 pi s / N, 2 pi (s + 1) / N]
  for (int r = 0; r < kRadii; ++r) {
    const int sg = r / 2;
    const double off = 2.0 * M_PI / (3.0 * kSegs);
    const double ang = (r % 2 == 0) ? 2.0 * M_PI * sg / kSegs + off : 2.0 * M_PI * (sg + 1) / kSegs - off;
    host[2 * r] = std::cos(ang);
    host[2 * r + 1] = std::sin(ang);
  }
  const int n[3] = {d.n[0], d.n[1], d.n[2]};
  double reach[SIM_MAX_SOLIDS], Ti[SIM_MAX_SOLIDS][3][3], det[SIM_MAX_SOLIDS];
  double lip = 1.0;   // bound on the scene's |grad phi| (the CSG of the solids' bounds)
  for (int q = 0; q < m; ++q) {
    const double* th = theta + 1 + m + (size_t)q * kShapeParams;
    double* S = host + kShapeHead + (size_t)q * kShapeStride;
    if (!(th[13] > th[12])) return SIM_EINVAL;
    for (int t = 0; t < 14; ++t) S[t] = th[t];
    S[14] = q == 0 ? 0.0 : theta[1 + q];
    const double* C = th + 14;
    const double* P = th + 14 + 2 * kKeys;
    for (int t = 0; t < 2 * kKeys; ++t) S[kOffC + t] = C[t];
    for (int t = 0; t < kRadii * kKeys; ++t) S[kOffRho + t] = P[t];
    reach[q] = 0.0;   // bound on |vertex| in the solid's frame (a vertex is c plus a convex mix of rho dir)
    for (int key = 0; key < kKeys; ++key) {
      double rmax = 0.0;
      for (int r = 0; r < kRadii; ++r) rmax = std::max(rmax, std::fabs(P[kRadii * key + r]));
      reach[q] = std::max(reach[q], std::hypot(C[2 * key], C[2 * key + 1]) + rmax);
      for (int v = 0; v < kVerts; ++v) {
        int rr[4];
        double w[4];
        vertex_taps(v, rr, w);
        double vx = C[2 * key], vy = C[2 * key + 1];
        for (int t = 0; t < 4; ++t) {
          vx += w[t] * P[kRadii * key + rr[t]] * host[2 * rr[t]];
          vy += w[t] * P[kRadii * key + rr[t]] * host[2 * rr[t] + 1];
        }
        S[kOffVert + 2 * (kVerts * key + v)] = vx;
        S[kOffVert + 2 * (kVerts * key + v) + 1] = vy;
      }
    }
    S[15] = reach[q];
    // |d(cross-section distance)/dp_z| <= how fast a polygon vertex moves with p_z
    double slope = 0.0;
    for (int key = 0; key + 1 < kKeys; ++key)
      for (int v = 0; v < kVerts; ++v) {
        const double* a = S + kOffVert + 2 * (kVerts * key + v);
        const double* b = a + 2 * kVerts;
        slope = std::max(slope, std::hypot(b[0] - a[0], b[1] - a[1]) * (kKeys - 1) / (th[13] - th[12]));
      }
    // T = R^T (p = T (x - o)): T[a][b] = R[b][a]; (R^T)^-1 = adj(T) / det(T)
    double T[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) T[a][b] = th[3 + 3 * b + a];
    double (&I)[3][3] = Ti[q];
    I[0][0] = T[1][1] * T[2][2] - T[1][2] * T[2][1];
    I[0][1] = T[0][2] * T[2][1] - T[0][1] * T[2][2];
    I[0][2] = T[0][1] * T[1][2] - T[0][2] * T[1][1];
    I[1][0] = T[1][2] * T[2][0] - T[1][0] * T[2][2];
    I[1][1] = T[0][0] * T[2][2] - T[0][2] * T[2][0];
    I[1][2] = T[0][2] * T[1][0] - T[0][0] * T[1][2];
    I[2][0] = T[1][0] * T[2][1] - T[1][1] * T[2][0];
    I[2][1] = T[0][1] * T[2][0] - T[0][0] * T[2][1];
    I[2][2] = T[0][0] * T[1][1] - T[0][1] * T[1][0];
    det[q] = T[0][0] * I[0][0] + T[0][1] * I[1][0] + T[0][2] * I[2][0];
    if (!(std::fabs(det[q]) > 1e-12)) return SIM_EINVAL;
    // |grad_x| <= ||T||_2 |grad_p|, |grad_p| <= sqrt(1 + slope^2); ||T||_2^2 is the
    // largest eigenvalue of the symmetric T^T T (closed form for 3 x 3)
    double A[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) A[a][b] = T[0][a] * T[0][b] + T[1][a] * T[1][b] + T[2][a] * T[2][b];
    double lmax;
    const double p1 = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    if (p1 == 0.0) {
      lmax = std::max(A[0][0], std::max(A[1][1], A[2][2]));
    } else {
      const double qm = (A[0][0] + A[1][1] + A[2][2]) / 3.0;
      const double p2 = (A[0][0] - qm) * (A[0][0] - qm) + (A[1][1] - qm) * (A[1][1] - qm) +
                        (A[2][2] - qm) * (A[2][2] - qm) + 2.0 * p1;
      const double pp = std::sqrt(p2 / 6.0);
      double Bm[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Bm[a][b] = (A[a][b] - (a == b ? qm : 0.0)) / pp;
      const double r = 0.5 * (Bm[0][0] * (Bm[1][1] * Bm[2][2] - Bm[1][2] * Bm[2][1]) -
                              Bm[0][1] * (Bm[1][0] * Bm[2][2] - Bm[1][2] * Bm[2][0]) +
                              Bm[0][2] * (Bm[1][0] * Bm[2][1] - Bm[1][1] * Bm[2][0]));
      lmax = qm + 2.0 * pp * std::cos(std::acos(std::min(1.0, std::max(-1.0, r))) / 3.0);
    }
    lip = std::max(lip, 1.001 * std::sqrt(std::max(lmax, 0.0)) * std::sqrt(1.0 + slope * slope));
  }
  // dJ/dphi is nonzero only at the corners of cut faces (corners of both
  // signs), so |phi| <= lip sqrt(2) dx there; where the node's CSG term is
  // solid q, its distance to q is the same, so its frame point p lies in the
  // box [-reach - e, reach + e]^2 x [z0 - e, z1 + e], e = lip sqrt(2) dx:
  // the world bounds of that box's corners x = o + (R^T)^-1 p, widened by
  // one node.
  const double e = lip * std::sqrt(2.0) * d.dx;
  // nodes whose phi bound exceeds e (with a margin) touch no cut face
  G.solid_far = 1.01 * e;
  for (int q = 0; q < m; ++q) {
    const double* th = theta + 1 + m + (size_t)q * kShapeParams;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int c = 0; c < 8; ++c) {
      const double p[3] = {(c & 1) ? reach[q] + e : -reach[q] - e, (c & 2) ? reach[q] + e : -reach[q] - e,
                           (c & 4) ? th[13] + e : th[12] - e};
      for (int a = 0; a < 3; ++a) {
        const double w = th[a] + (Ti[q][a][0] * p[0] + Ti[q][a][1] * p[1] + Ti[q][a][2] * p[2]) / det[q];
        lo[a] = std::min(lo[a], w);
        hi[a] = std::max(hi[a], w);
      }
    }
    for (int a = 0; a < 3; ++a) {
      const double l = std::max(0.0, std::floor(lo[a] / d.dx) - 1.0);
      const double h = std::min((double)n[a], std::ceil(hi[a] / d.dx) + 1.0);
      G.sbox[q][a] = (int)std::min(l, (double)n[a] + 1.0);
      G.sbox[q][3 + a] = h >= l ? (int)(h - l) + 1 : 0;
    }
  }
  G.nsolid = m;
  return SIM_OK;
}

void launch_phi_nodes(const Domain& D, const GeomParams& G, double* phi, hipStream_t s) {
  if (G.kind == SIM_GEOM_BEZIER) {
    hipLaunchKernelGGL(k_phi_solids, dim3(nblocks(D.d.nodes())), dim3(kBlock), 0, s, D.d, D.dx, G, phi);
    return;
  }
  hipLaunchKernelGGL(k_phi_nodes, dim3(nblocks(D.d.nodes())), dim3(kBlock), 0, s, D.d, D.dx, G, phi);
}

void launch_alpha(const Domain& D, const double* phi, float* alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_alpha, dim3(nblocks(D.d.faces())), dim3(kBlock), 0, s, D, phi, alpha);
}

void launch_invdiag(const Dims& d, const float* ax, const float* ay, const float* az, float* invd,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_invdiag, dim3(nblocks(d.cells())), dim3(kBlock), 0, s, d, ax, ay, az, invd);
}

}  // namespace nf
