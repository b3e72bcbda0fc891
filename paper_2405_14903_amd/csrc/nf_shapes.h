// Parametric solids: closed polar Bezier cross-sections extruded between key
// cross-sections, combined by CSG union / intersection.
//
// NeuralFluid, Sec. Geometry Representation and App. "Geometry Representation
// Implementation":
//  * a cross-section is N cubic Bezier segments around a centre c; segment m
//    spans the polar angles [2 pi m / N, 2 pi (m + 1) / N] and its two inner
//    control points lie 2 pi / (3N) inside that span at polar distances
//    rho_{2m} and rho_{2m+1}; the joint shared by two segments lies on the
//    line through the control points around it (taken here as their midpoint);
//  * a solid is K key cross-sections evenly spaced on the z axis of its own
//    frame between z0 and z1; between keys the centre and the radii are
//    interpolated linearly in s = (z - z0) / (z1 - z0), clamped to [0, 1]
//    (the printed power series does not pass through the keys; linear
//    interpolation does);
//  * each segment is represented by its polyline through kSamples points
//    (Bezier parameter t = k / kSamples), so the signed distance of a point to
//    the cross-section is the exact distance to that polygon (negative inside,
//    by crossing parity), and a solid's distance in its frame p = R^T (x - o)
//    is max(d2(p_x, p_y), z0 - p_z, p_z - z1);
//  * the scene's fluid SDF phi (positive in fluid) is the CSG of the solids'
//    distances left to right: min for a union, max for an intersection.
//
// Device layout of the packed solids (doubles): kShapeDirs control-angle unit
// vectors (cos, sin) at offset 0, then per solid q at kShapeHead +
// q * kShapeStride: o(3) R(9, row-major, body -> world) z0 z1 op reach (the
// radius in the solid's frame of a disk that holds every cross-section), the key
// centres (K x 2), the key radii (K x 2N, key-major), and the polygon
// vertices of every key cross-section (K x kVerts x 2), computed on the host.
// The polygon at s is then the linear interpolation of the two bracketing
// key polygons (the polygon is linear in the centre and radii).
#pragma once

#include "nf_internal.h"

namespace nf {

constexpr int kSegs = SIM_BEZIER_SEGMENTS;                    // Bezier segments per cross-section
constexpr int kRadii = 2 * kSegs;                             // control radii per cross-section
constexpr int kSamples = SIM_BEZIER_SAMPLES;                  // polygon points per segment
constexpr int kVerts = kSegs * kSamples;                      // polygon vertices per cross-section
constexpr int kKeys = SIM_BEZIER_KEYS;                        // key cross-sections per solid
constexpr int kShapeParams = SIM_BEZIER_SHAPE_PARAMS;         // parameters of one solid in theta
constexpr int kShapeDirs = 2 * kRadii;
constexpr int kShapeHead = kShapeDirs;
constexpr int kOffC = 16, kOffRho = kOffC + 2 * kKeys, kOffVert = kOffRho + kRadii * kKeys;
constexpr int kShapeStride = (kOffVert + 2 * kVerts * kKeys + 7) / 8 * 8;
static_assert(kShapeParams == 3 + 9 + 2 + 2 * kKeys + kRadii * kKeys, "solid parameter count");

inline size_t shape_buffer_doubles() { return kShapeHead + (size_t)kShapeStride * SIM_MAX_SOLIDS; }

// Polygon vertex v of a cross-section is c + sum_r w_r rho_r dir_r over four
// radii: the cubic Bernstein weights of its segment's control polygon
// (joint, two control points, joint), each joint the mean of the control
// points around it.
__host__ __device__ inline void vertex_taps(int v, int (&r)[4], double (&w)[4]) {
  const int m = v / kSamples;
  const double t = (double)(v % kSamples) / kSamples, u = 1.0 - t;
  const double b0 = u * u * u, b1 = 3.0 * u * u * t, b2 = 3.0 * u * t * t, b3 = t * t * t;
  r[0] = (2 * m + kRadii - 1) % kRadii;   // control point before the segment's first joint
  r[1] = 2 * m;
  r[2] = 2 * m + 1;
  r[3] = (2 * m + 2) % kRadii;            // control point after its last joint
  w[0] = 0.5 * b0;
  w[1] = 0.5 * b0 + b1;
  w[2] = b2 + 0.5 * b3;
  w[3] = 0.5 * b3;
}

// Where a point falls relative to one solid.
struct SolidHit {
  double val;          // signed distance (negative inside)
  double px, py, pz;   // the point in the solid's frame
  double s;            // (p_z - z0) / (z1 - z0), unclamped
  int key;             // lower bracketing key
  double lam;          // weight of key + 1
  int edge;            // closest polygon edge (vertices edge, edge + 1)
  int which;           // 0: the cross-section, 1: the z0 cap, 2: the z1 cap
  bool inside;         // inside the cross-section's polygon
};

__device__ inline void solid_locate(const double* __restrict__ S, double x, double y, double z, SolidHit& h) {
  const double r0 = x - S[0], r1 = y - S[1], r2 = z - S[2];
  const double* R = S + 3;
  h.px = R[0] * r0 + R[3] * r1 + R[6] * r2;
  h.py = R[1] * r0 + R[4] * r1 + R[7] * r2;
  h.pz = R[2] * r0 + R[5] * r1 + R[8] * r2;
  const double z0 = S[12], z1 = S[13];
  h.s = (h.pz - z0) / (z1 - z0);
  const double u = fmin(fmax(h.s, 0.0), 1.0) * (kKeys - 1);
  h.key = min((int)floor(u), kKeys - 2);
  h.lam = u - h.key;
}

// Signed distance of (x, y, z) to solid S (distance only when `full` is
// false; with it, also the closest edge and the active term).
template <bool full>
__device__ inline double solid_distance(const double* __restrict__ S, double x, double y, double z, SolidHit& h) {
  solid_locate(S, x, y, z, h);
  const double* A = S + kOffVert + 2 * kVerts * h.key;
  const double* B = A + 2 * kVerts;
  const double l1 = h.lam, l0 = 1.0 - h.lam;
  const double qx = h.px, qy = h.py;
  // the squared distance to the closest edge as num / den (no division in the loop)
  double best_num = 1e300, best_den = 1.0;
  int best = 0;
  bool inside = false;
  double ax = l0 * A[0] + l1 * B[0], ay = l0 * A[1] + l1 * B[1];
  for (int v = 0; v < kVerts; ++v) {
    const int vn = v + 1 == kVerts ? 0 : v + 1;
    const double bx = l0 * A[2 * vn] + l1 * B[2 * vn], by = l0 * A[2 * vn + 1] + l1 * B[2 * vn + 1];
    const double ex = bx - ax, ey = by - ay, aqx = qx - ax, aqy = qy - ay;
    const double t = aqx * ex + aqy * ey, den = ex * ex + ey * ey;
    double num, dd = 1.0;
    if (t <= 0.0) {
      num = aqx * aqx + aqy * aqy;
    } else if (t >= den) {
      const double bqx = qx - bx, bqy = qy - by;
      num = bqx * bqx + bqy * bqy;
    } else {
      const double cr = aqx * ey - aqy * ex;
      num = cr * cr;
      dd = den;
    }
    if (num * best_den < best_num * dd) {
      best_num = num;
      best_den = dd;
      best = v;
    }
    // crossing number of the ray from q along +x
    if ((ay > qy) != (by > qy)) {
      const double lhs = (qx - ax) * ey, rhs = (qy - ay) * ex;
      if (ey > 0.0 ? lhs < rhs : lhs > rhs) inside = !inside;
    }
    ax = bx;
    ay = by;
  }
  const double dist = sqrt(best_num / best_den);
  const double d2 = inside ? -dist : dist;
  const double lo = S[12] - h.pz, hi = h.pz - S[13];
  const double cap = fmax(lo, hi);
  h.val = fmax(d2, cap);
  if (full) {
    h.edge = best;
    h.inside = inside;
    h.which = d2 >= cap ? 0 : (lo >= hi ? 1 : 2);
  }
  return h.val;
}

constexpr unsigned char kNoSolid = 0xff;   // CSG term of a far-field node

// A lower bound of solid S's distance at (x, y, z): every cross-section lies
// in the disk of radius `reach` about the frame's axis, so the distance to the
// polygon is at least |p_xy| - reach (also inside, where the polygon's
// boundary is nearer than the disk's), and the caps' terms are exact.
__device__ inline double solid_lower_bound(const double* __restrict__ S, double x, double y, double z) {
  const double r0 = x - S[0], r1 = y - S[1], r2 = z - S[2];
  const double* R = S + 3;
  const double px = R[0] * r0 + R[3] * r1 + R[6] * r2;
  const double py = R[1] * r0 + R[4] * r1 + R[7] * r2;
  const double pz = R[2] * r0 + R[5] * r1 + R[8] * r2;
  return fmax(sqrt(px * px + py * py) - S[15], fmax(S[12] - pz, pz - S[13]));
}

// phi of the scene at (x, y, z) and its CSG term.  The CSG of the solids'
// lower bounds bounds phi from below (min and max are monotone); beyond
// `far` no face at the node can be cut, so there that bound stands in for phi
// (positive: fluid) and the term is kNoSolid.  Nearer, phi is exact: a union
// member whose bound is not below the running value cannot lower it, so its
// polygon walk is skipped.
__device__ inline double scene_phi_fast(const double* __restrict__ shapes, int m, double far, double x, double y,
                                        double z, unsigned char& term) {
  double lb[SIM_MAX_SOLIDS];
  double lbs = 0.0;
  for (int q = 0; q < m; ++q) {
    const double* S = shapes + kShapeHead + (size_t)q * kShapeStride;
    lb[q] = solid_lower_bound(S, x, y, z);
    lbs = q == 0 ? lb[q] : (S[14] == 0.0 ? fmin(lbs, lb[q]) : fmax(lbs, lb[q]));
  }
  if (lbs > far) {
    term = kNoSolid;
    return lbs;
  }
  SolidHit h;
  double phi = solid_distance<false>(shapes + kShapeHead, x, y, z, h);
  term = 0;
  for (int q = 1; q < m; ++q) {
    const double* S = shapes + kShapeHead + (size_t)q * kShapeStride;
    const bool uni = S[14] == 0.0;
    if (uni && lb[q] >= phi) continue;
    const double v = solid_distance<false>(S, x, y, z, h);
    if (uni ? v < phi : v > phi) {
      phi = v;
      term = (unsigned char)q;
    }
  }
  return phi;
}

// acc += w * d(distance of solid S at (x, y, z)) / d(its kShapeParams
// parameters), in the order of theta: o, R, z0, z1, key centres, key radii.
// d2 = sgn |q - Q| with Q the closest point of edge (a, b): d d2 / d Q =
// -n, n = sgn (q - Q) / |q - Q|; Q moves with the centre and, through the
// edge's vertex taps, with the radii; s moves the bracketing interpolation.
__device__ inline void solid_distance_grad(const double* __restrict__ dirs, const double* __restrict__ S, double x,
                                           double y, double z, double w, double (&acc)[kShapeParams]) {
  SolidHit h;
  solid_distance<true>(S, x, y, z, h);
  const double* R = S + 3;
  const double z0 = S[12], z1 = S[13], L = z1 - z0;
  const double r[3] = {x - S[0], y - S[1], z - S[2]};
  double gp[3];
  if (h.which == 0) {
    const double* A = S + kOffVert + 2 * kVerts * h.key;
    const double* B = A + 2 * kVerts;
    const double l1 = h.lam, l0 = 1.0 - h.lam;
    const int e = h.edge, en = e + 1 == kVerts ? 0 : e + 1;
    const double ax = l0 * A[2 * e] + l1 * B[2 * e], ay = l0 * A[2 * e + 1] + l1 * B[2 * e + 1];
    const double bx = l0 * A[2 * en] + l1 * B[2 * en], by = l0 * A[2 * en + 1] + l1 * B[2 * en + 1];
    const double ex = bx - ax, ey = by - ay;
    const double den = ex * ex + ey * ey;
    double tau = den > 0.0 ? ((h.px - ax) * ex + (h.py - ay) * ey) / den : 0.0;
    tau = fmin(fmax(tau, 0.0), 1.0);
    const double dqx = h.px - (ax + tau * ex), dqy = h.py - (ay + tau * ey);
    const double dist = sqrt(dqx * dqx + dqy * dqy);
    const double sg = h.inside ? -1.0 : 1.0;
    const double nx = dist > 0.0 ? sg * dqx / dist : 0.0, ny = dist > 0.0 ? sg * dqy / dist : 0.0;
    // d d2 / d(centre) = -n; d d2 / d rho_r = -wq_r (n . dir_r)
    int ra[4], rb[4];
    double wa[4], wb[4];
    vertex_taps(e, ra, wa);
    vertex_taps(en, rb, wb);
    // (selects with constant indices keep acc and grho in registers)
    double grho[kRadii];
#pragma unroll
    for (int q = 0; q < kRadii; ++q) {
      double wq = 0.0;
#pragma unroll
      for (int t = 0; t < 4; ++t) wq += (ra[t] == q ? (1.0 - tau) * wa[t] : 0.0) + (rb[t] == q ? tau * wb[t] : 0.0);
      grho[q] = -wq * (nx * dirs[2 * q] + ny * dirs[2 * q + 1]);
    }
    const int k0 = h.key, k1 = h.key + 1;
    const double* C = S + kOffC;
    const double* P = S + kOffRho;
    const bool clamped = h.s < 0.0 || h.s > 1.0;
    double dds = 0.0;
    if (!clamped)
      dds = -nx * (C[2 * k1] - C[2 * k0]) * (kKeys - 1) - ny * (C[2 * k1 + 1] - C[2 * k0 + 1]) * (kKeys - 1);
#pragma unroll
    for (int q = 0; q < kRadii; ++q)
      if (!clamped) dds += grho[q] * (P[kRadii * k1 + q] - P[kRadii * k0 + q]) * (kKeys - 1);
#pragma unroll
    for (int kk = 0; kk < kKeys; ++kk) {
      const double wk = kk == k0 ? w * l0 : (kk == k1 ? w * l1 : 0.0);
      acc[14 + 2 * kk] -= wk * nx;
      acc[15 + 2 * kk] -= wk * ny;
#pragma unroll
      for (int q = 0; q < kRadii; ++q) acc[14 + 2 * kKeys + kRadii * kk + q] += wk * grho[q];
    }
    gp[0] = nx;
    gp[1] = ny;
    gp[2] = dds / L;
    acc[12] += w * dds * (h.s - 1.0) / L;
    acc[13] -= w * dds * h.s / L;
  } else {
    gp[0] = gp[1] = 0.0;
    gp[2] = h.which == 1 ? -1.0 : 1.0;
    if (h.which == 1) acc[12] += w;
    else acc[13] -= w;
  }
  // the frame: p = R^T (x - o)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    acc[i] -= w * (R[3 * i] * gp[0] + R[3 * i + 1] * gp[1] + R[3 * i + 2] * gp[2]);
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[3 + 3 * i + j] += w * r[i] * gp[j];
  }
}

}  // namespace nf
