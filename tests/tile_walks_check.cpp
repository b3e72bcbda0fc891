// Host enumeration of every access of the fused tile kernels' region walks:
// every in-domain cell of each +H region is visited exactly once, every visited
// element index (cells, x / y / z faces, parent cells) matches the layout and
// lies inside its array, out-of-domain cells get the out-of-range lane offset,
// and the 31-bit byte offsets hold; and the one-workgroup bottom solve's lane
// layout (one lane per cell, the 8 children of a cell on 8 consecutive lanes).
// nf_tile.h is plain integer code; compiled here for the host only
#define __host__
#define __device__
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "nf_tile.h"
using namespace nf;

static long errors = 0;
#define CHECK(c, ...) do { if (!(c)) { if (errors < 20) { printf(__VA_ARGS__); printf("\n"); } ++errors; } } while (0)

template <class S, int H>
void walk(int nx, int ny, int nz, int b, std::vector<int>& cover) {
  using W = Walk<S, H>;
  int i0, j0, k0;
  tile_origin_of<S>(b, nx, ny, i0, j0, k0);
  const bool zin = planes_inside<S>(k0, nz);
  const long pc = (long)nx * ny, px = (long)(nx + 1) * ny, py = (long)nx * (ny + 1);
  const long nfx = px * nz, nfy = py * nz, nfz = pc * (nz + 1), ncell = pc * nz;
  const int cnx = nx / 2, cny = ny / 2, cnz = nz / 2;   // parent (used when even)
  const bool even = nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0;
  cover.assign(W::N, 0);
  for (int t = 0; t < kTileThreads; ++t) {
    int lz = W::P == 1 ? 0 : t / W::PL;
    if (W::kUniform && W::P > 1) CHECK(lz == (t & ~63) / W::PL, "non-uniform plane group t=%d", t);
    const Lane l = lane_of<S, H>(t, lz, i0, j0, nx, ny);
    const unsigned m = zin ? ~0u : plane_mask(k0, l.z, nz, W::T);
    if (!l.on) continue;
    for (int u = 0; u < W::T; ++u) {
      const int kr = l.z + u;
      const int q = l.q + u * W::PL;
      CHECK(q >= 0 && q < W::N, "lds q out of region");
      cover[q]++;
      // region frame position of q must match lane x, y and plane kr
      const int rx = q % W::X, ry = (q / W::X) % W::Y, rz = q / W::PL;
      CHECK(rx + 2 - H == l.x && ry + 2 - H == l.y && rz + 2 - H == kr, "q/position mismatch");
      const int i = i0 - 2 + l.x, j = j0 - 2 + l.y, k = k0 - 2 + kr;
      const bool indom = i >= 0 && j >= 0 && k >= 0 && i < nx && j < ny && k < nz;
      const bool valid = l.in && ((m >> u) & 1u);
      CHECK(valid == indom, "validity mismatch tile %d t %d u %d (%d,%d,%d) valid %d indom %d zin %d", b, t, u, i, j, k, valid, indom, zin);
      if (zin) CHECK(k >= 0 && k < nz, "zin but plane outside");
      if (!valid) continue;
      // element indices as the kernels form them: view base + lane part + plane part
      const long cbase = (long)(i0 - 2) + (long)nx * (j0 - 2) + pc * (k0 - 2);
      const long c = cbase + l.ce + (long)kr * pc;
      CHECK(c == i + (long)nx * (j + (long)ny * k), "cell index");
      CHECK(c >= 0 && c < ncell, "cell oob");
      const long fxb = (long)(i0 - 2) + (long)(nx + 1) * (j0 - 2) + px * (k0 - 2);
      const long fx = fxb + l.fe + (long)kr * px;
      CHECK(fx == i + (long)(nx + 1) * (j + (long)ny * k), "fx index");
      CHECK(fx >= 0 && fx + 1 < nfx, "fx oob");
      const long fyb = (long)(i0 - 2) + (long)nx * (j0 - 2) + py * (k0 - 2);
      const long fy = fyb + l.ce + (long)kr * py;
      CHECK(fy == i + (long)nx * (j + (long)(ny + 1) * k), "fy index");
      CHECK(fy >= 0 && fy + nx < nfy, "fy oob");
      const long fz = cbase + l.ce + (long)kr * pc;
      CHECK(fz >= 0 && fz + pc < nfz, "fz oob");
      // 32-bit byte offsets (largest element size 4) stay below 2^31
      const long lane_max = (long)l.fe + 1, plane_max = (long)(kr + 1) * (px > py ? px : py);
      CHECK((lane_max + plane_max + nx) * 4 < 0x7fffffffL, "offset exceeds 31 bits");
      if (H == 2 && even) {
        const long eb = (long)((i0 - 2) / 2) + (long)cnx * ((j0 - 2) / 2) + (long)cnx * cny * ((k0 - 2) / 2);
        const long e = eb + (l.x >> 1) + (long)cnx * (l.y >> 1) + (long)(kr >> 1) * cnx * cny;
        CHECK(e == (i >> 1) + (long)cnx * ((j >> 1) + (long)cny * (k >> 1)), "parent index");
        CHECK(e >= 0 && e < (long)cnx * cny * cnz, "parent oob");
      }
      // stencil neighbours in LDS stay inside the region for interior walks
      if constexpr (H < 2) {
        using Wo = Walk<S, H + 1>;
        const int o = 2 - (H + 1);   // outer region origin in the +2 frame
        const int qo = (l.x - o) + Wo::X * (l.y - o) + Wo::PL * (kr - o);
        CHECK(qo - Wo::PL >= 0 && qo + Wo::PL < Wo::N && qo - 1 >= 0 && qo + 1 < Wo::N, "stencil outside outer region");
      }
    }
  }
  for (int q = 0; q < W::N; ++q) CHECK(cover[q] == 1, "region cell %d covered %d times (H=%d)", q, cover[q], H);
}

template <class S>
void check(int nx, int ny, int nz) {
  const int nt = tiles_x<S>(nx) * tiles_y<S>(ny) * tiles_z<S>(nz);
  std::vector<int> cover;
  for (int b = 0; b < nt; ++b) {
    walk<S, 2>(nx, ny, nz, b, cover);
    walk<S, 1>(nx, ny, nz, b, cover);
    walk<S, 0>(nx, ny, nz, b, cover);
  }
  // the tile origins partition the grid
  std::vector<char> seen((size_t)nx * ny * nz, 0);
  for (int b = 0; b < nt; ++b) {
    int i0, j0, k0;
    tile_origin_of<S>(b, nx, ny, i0, j0, k0);
    for (int k = k0; k < k0 + S::TZ && k < nz; ++k)
      for (int j = j0; j < j0 + S::TY && j < ny; ++j)
        for (int i = i0; i < i0 + S::TX && i < nx; ++i) seen[i + (size_t)nx * (j + (size_t)ny * k)]++;
  }
  for (size_t c = 0; c < seen.size(); ++c) CHECK(seen[c] == 1, "cell %zu owned %d times", c, seen[c]);
}

// The bottom's lane layout: on every level each cell has exactly one lane,
// lanes 8C .. 8C+7 own the children of lane C's cell on the next coarser level
// (so 8-lane groups are whole or empty), and no lane beyond the level's cell
// count has a cell.
void check_bottom(int cnx, int cny, int cnz, int nl) {
  for (int l = 0; l < nl; ++l) {
    const int f = 1 << (nl - 1 - l);
    const int nx = cnx * f, ny = cny * f, nz = cnz * f, n = nx * ny * nz;
    std::vector<int> seen((size_t)n, 0);
    for (int t = 0; t < 1024; ++t) {
      int i = -1, j = -1, k = -1;
      const bool on = bottom_cell(t, l, nl, cnx, cny, cnz, i, j, k);
      CHECK(on == (t < n), "bottom lane %d on %d, level %d of %d cells", t, on, l, n);
      if (!on) continue;
      CHECK(i >= 0 && j >= 0 && k >= 0 && i < nx && j < ny && k < nz, "bottom cell out of level");
      if (!(i >= 0 && j >= 0 && k >= 0 && i < nx && j < ny && k < nz)) continue;
      seen[i + (size_t)nx * (j + (size_t)ny * k)]++;
      if (l + 1 < nl) {
        int pi, pj, pk;
        const bool pon = bottom_cell(t >> 3, l + 1, nl, cnx, cny, cnz, pi, pj, pk);
        CHECK(pon && pi == i / 2 && pj == j / 2 && pk == k / 2, "lane %d: parent not on lane %d", t, t >> 3);
        CHECK((i & 1) + 2 * (j & 1) + 4 * (k & 1) == (t & 7), "lane %d: child bits", t);
      }
    }
    for (int c = 0; c < n; ++c) CHECK(seen[c] == 1, "bottom cell %d owned %d times", c, seen[c]);
  }
}

int main() {
  const int dims[][3] = {{128, 128, 128}, {64, 64, 64}, {32, 32, 32}, {16, 16, 16}, {20, 24, 36}, {10, 12, 14},
                         {48, 40, 16}, {8, 8, 8}, {34, 18, 10}, {66, 10, 22}, {30, 30, 30}, {12, 12, 12}, {6, 4, 10}};
  for (auto& d : dims) {
    check<FineTile>(d[0], d[1], d[2]);
    check<CoarseTile>(d[0], d[1], d[2]);
    check<CoarseTileH>(d[0], d[1], d[2]);
    printf("%dx%dx%d done, errors so far %ld\n", d[0], d[1], d[2], errors);
  }
  // bottom chains of at most 1024 cells on the finest bottom level
  const int chains[][4] = {{2, 2, 2, 3}, {1, 1, 1, 4}, {2, 4, 8, 2}, {2, 2, 4, 3}, {3, 5, 2, 2}, {2, 2, 128, 1},
                           {4, 4, 2, 2}, {1, 2, 3, 3}};
  for (auto& c : chains) check_bottom(c[0], c[1], c[2], c[3]);
  printf("bottom lane layouts done, errors so far %ld\n", errors);
  printf(errors ? "FAILED %ld\n" : "OK\n", errors);
  return errors != 0;
}
