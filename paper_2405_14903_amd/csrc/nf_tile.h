// Tile geometry and addressing of the fused multigrid / CG tile kernels.
//
// One workgroup owns a TX x TY x TZ tile of a grid level and works on the
// tile grown by H cells on every side (its "+H region", H = 0, 1, 2).  A
// region is walked plane by plane: each lane keeps one (x, y) position of a
// plane for the whole launch and P planes are covered per trip, so from trip
// to trip only the plane changes.
//
// Arrays are addressed through buffer resources whose base is the array's
// element at the corner (i0 - 2, j0 - 2, k0 - 2) of the +2 region, so every
// address is a 32-bit byte offset made of
//   * a lane part (the lane's x, y position; fixed for the launch),
//   * a plane part (uniform over the wave when the plane index is; the view
//     base plane is k0 - 2, so the plane part of +2-frame plane z is z times
//     the array's plane length), and
//   * neighbour steps (+1 element in x: an immediate; +1 row or +1 plane: a
//     uniform offset).
// A lane whose (i, j) lies outside the domain carries the lane offset
// kNoCell, beyond the resource's record count: the hardware range check reads
// 0 for it and drops its stores.  The same lane offset stands in for every
// lane of a trip whose plane lies outside the domain, so values outside the
// domain read 0 and nothing outside it is written, without branches.
//
// Everything here is plain integer arithmetic usable on the host, so the
// bounds of every access can be enumerated on the CPU.
#pragma once

#include <stdint.h>

namespace nf {

template <int TX_, int TY_, int TZ_>
struct TileShape {
  static constexpr int TX = TX_, TY = TY_, TZ = TZ_;
};
// The finest level uses long x rows (one +2 plane fills most of a workgroup,
// so plane indices stay uniform), the coarse levels small cubes (their
// launches are latency-bound: less serial work per thread, more workgroups).
using FineTile = TileShape<32, 8, 8>;
using CoarseTile = TileShape<8, 8, 8>;
// Coarse levels of at least kWideTileCells cells: 16-cell rows, half the
// workgroups and less halo per cell.
using CoarseTileH = TileShape<16, 8, 8>;
constexpr long kWideTileCells = 1L << 18;
constexpr int kTileThreads = 512;   // 8 waves per tile

constexpr unsigned kNoCell = 0x80000000u;   // lane offset of a lane outside the domain
constexpr int kViewRecords = 0x7fffffff;    // record count of every view (bytes)

// Walk of the +H region of tile shape S by kTileThreads lanes: X x Y x Z
// cells, PL cells per plane, P planes per trip, T trips.  Lane t sits at plane
// position t % PL of plane-group lz = t / PL and covers planes lz * T + u,
// u = 0 .. T-1.  When the lanes of one wave share lz (P == 1, or PL a multiple
// of 64) the plane index of a trip is uniform over the wave.
template <class S, int H>
struct Walk {
  static constexpr int X = S::TX + 2 * H, Y = S::TY + 2 * H, Z = S::TZ + 2 * H;
  static constexpr int PL = X * Y, N = PL * Z;
  static constexpr int P = kTileThreads / PL < Z ? kTileThreads / PL : Z;
  static constexpr int T = (Z + P - 1) / P;
  static constexpr bool kUniform = P == 1 || PL % 64 == 0;
  static_assert(P >= 1, "a plane of the region must fit the workgroup");
  static_assert(P * T == Z, "plane groups must tile the region exactly");
};

template <class S>
constexpr int tiles_x(int nx) { return (nx + S::TX - 1) / S::TX; }
template <class S>
constexpr int tiles_y(int ny) { return (ny + S::TY - 1) / S::TY; }
template <class S>
constexpr int tiles_z(int nz) { return (nz + S::TZ - 1) / S::TZ; }

// Tile origin of logical tile b (unsigned arithmetic: cheaper divisions).
template <class S>
inline __host__ __device__ void tile_origin_of(int b, int nx, int ny, int& i0, int& j0, int& k0) {
  const unsigned tx = (unsigned)tiles_x<S>(nx), ty = (unsigned)tiles_y<S>(ny), ub = (unsigned)b;
  const unsigned bx = ub / tx, bxy = bx / ty;
  i0 = (int)(ub - bx * tx) * S::TX;
  j0 = (int)(bx - bxy * ty) * S::TY;
  k0 = (int)bxy * S::TZ;
}

// One lane's place in a region walk.
struct Lane {
  int x, y;   // position in the +2 region frame
  int z;      // first plane of the lane, +2 region frame
  int q;      // LDS index (region frame, x fastest) of the lane's first cell
  bool on;    // the lane has cells
  bool in;    // on, and (i, j) inside the domain
  int ce;     // element offset x + nx * y of the lane in the cell frame (cells, y and z faces)
  int fe;     // element offset x + (nx + 1) * y in the x-face frame
};

// lz: the lane's plane group (t / PL; made wave-uniform by the caller where
// the walk allows it).
template <class S, int H>
inline __host__ __device__ Lane lane_of(int t, int lz, int i0, int j0, int nx, int ny) {
  using W = Walk<S, H>;
  Lane L;
  const int r = t - lz * W::PL;
  const int lx = r % W::X, ly = r / W::X;
  L.on = W::P == 1 ? t < W::PL : lz < W::P;
  L.x = lx + 2 - H;
  L.y = ly + 2 - H;
  L.z = lz * W::T + 2 - H;
  L.q = lx + W::X * ly + W::PL * (lz * W::T);
  const int i = i0 - 2 + L.x, j = j0 - 2 + L.y;
  L.in = L.on && i >= 0 && j >= 0 && i < nx && j < ny;
  L.ce = L.x + nx * L.y;
  L.fe = L.x + (nx + 1) * L.y;
  return L;
}

// Planes of a walk inside the domain: bit u is set when plane z0 + u of the
// +2 frame (absolute plane k0 - 2 + z0 + u) lies in [0, nz).  T <= 31.
inline __host__ __device__ unsigned plane_mask(int k0, int z0, int nz, int T) {
  int lo = 2 - k0 - z0, hi = nz - (k0 - 2 + z0);
  lo = lo < 0 ? 0 : lo;
  hi = hi > T ? T : hi;
  return hi > lo ? ((1u << (hi - lo)) - 1u) << lo : 0u;
}

// Whether every plane of the tile's +2 region lies inside the domain (then no
// trip needs a plane check).
template <class S>
inline __host__ __device__ bool planes_inside(int k0, int nz) {
  return k0 >= 2 && k0 + S::TZ + 2 <= nz;
}

// Whether a grid's +2 tile regions fit the views' 31-bit byte offsets
// (largest plane length times the planes a region spans, elements of es
// bytes: 4 for the arrays, 16 for the finest level's packed records).
inline __host__ __device__ bool views_fit(int nx, int ny, int es = 4) {
  const long plane = (long)(nx + 1) * ny > (long)nx * (ny + 1) ? (long)(nx + 1) * ny : (long)nx * (ny + 1);
  const int tz = FineTile::TZ > CoarseTile::TZ ? FineTile::TZ : CoarseTile::TZ;
  return ((long)(tz + 6) * plane + 2L * (nx + 1)) * es < (long)kViewRecords;
}

// Lane byte offset of an array of element size es (kNoCell outside the domain).
inline __host__ __device__ unsigned lane_bytes(bool in, int elems, int es) {
  return in ? (unsigned)elems * (unsigned)es : kNoCell;
}

// One-workgroup bottom solve with one lane per cell on every level: levels
// 0 .. nl-1 of the bottom, each half the one above along every axis, the
// coarsest cnx x cny x cnz.  Lanes are numbered children first: lane t owns on
// level l the cell whose ancestor on the coarsest level is cell t >> 3(nl-1-l)
// (x fastest) and whose child bits (x + 2y + 4z) on the levels below it are
// the octal digits of t, the lowest for level l.  So lanes 8C .. 8C+7 of level
// l own the 8 children of the cell lane C owns on level l+1.  Returns false
// when level l has no cell for lane t.
constexpr int kBottomLaneLevels = 4;   // most bottom levels the lane layout handles
inline __host__ __device__ bool bottom_cell(int t, int l, int nl, int cnx, int cny, int cnz, int& i, int& j, int& k) {
  const int up = 3 * (nl - 1 - l);
  const int top = t >> up;
  if (top >= cnx * cny * cnz) return false;
  i = top % cnx;
  j = (top / cnx) % cny;
  k = top / (cnx * cny);
  for (int s = up - 3; s >= 0; s -= 3) {
    const int b = (t >> s) & 7;
    i = 2 * i + (b & 1);
    j = 2 * j + ((b >> 1) & 1);
    k = 2 * k + (b >> 2);
  }
  return true;
}

}  // namespace nf
