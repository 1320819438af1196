// Host-side check of the sort's index algebra (pm_device.h), built and run
// by tests/test_host_sanitizers.py: the tile numbering is a bijection whose
// inverse is tile_coords and whose order is the Morton curve (bits of t_x,
// t_y, t_z interleaved, t_x lowest, compared with a bit-by-bit
// interleave); tile_key splits into (tile, class, half-tile block) as its
// definition states; the 27 bins of a paint tile are those of the tile and
// its lower neighbours with the classes that reach into it; the lattice
// walk of the first sort visits every particle once, a 4^3 brick of
// lattice sites per wave; wrap_pos maps any finite x into [0, n).
#include <cmath>
#include <cstdio>
#include <vector>

#include "pm_device.h"

namespace {
int fails = 0;
void check(bool ok, const char* what, long a, long b) {
  if (!ok && fails < 20) std::printf("FAIL %s (%ld, %ld)\n", what, a, b);
  if (!ok) ++fails;
}
// 16^3 tiles of an n^3 mesh (n = 16 * 2^k), the geometry the library builds
pmk::TileGeom tiles16(int n) {
  pmk::TileGeom g;
  g.n = n;
  g.tx = g.ty = g.tz = 16;
  g.ntx = g.nty = g.ntz = n / 16;
  g.ntiles = g.ntx * g.nty * g.ntz;
  g.lx = g.ly = g.lz = 4;
  g.lnx = g.lny = g.lnz = __builtin_ctz((unsigned)(n / 16));
  return g;
}
uint32_t interleave(uint32_t x, uint32_t y, uint32_t z, int bits) {
  uint32_t t = 0;
  for (int i = 0; i < bits; ++i)
    t |= ((x >> i) & 1u) << (3 * i) | ((y >> i) & 1u) << (3 * i + 1) | ((z >> i) & 1u) << (3 * i + 2);
  return t;
}
}  // namespace

int main() {
  using namespace pmk;
  // tile numbering
  for (int bits = 1; bits <= 6; ++bits) {
    const uint32_t T = 1u << bits;
    const TileGeom g = tiles16((int)(16 * T));
    std::vector<char> seen(T * T * T, 0);
    for (uint32_t z = 0; z < T; ++z)
      for (uint32_t y = 0; y < T; ++y)
        for (uint32_t x = 0; x < T; ++x) {
          const uint32_t t = tile_index(x, y, z);
          check(t == interleave(x, y, z, bits), "Morton order", t, interleave(x, y, z, bits));
          check(t < T * T * T && !seen[t], "tile numbering is a bijection", t, T);
          if (t < T * T * T) seen[t] = 1;
          int tx, ty, tz;
          tile_coords((int)t, g, tx, ty, tz);
          check(tx == (int)x && ty == (int)y && tz == (int)z, "tile_coords inverts tile_index", t, tx);
        }
  }
  // tile keys: (tile * 8 + class) * 8 + block on 16^3 tiles of a 128^3 mesh
  {
    const TileGeom g = tiles16(128);
    for (int ix = 0; ix < 128; ix += 3)
      for (int iy = 0; iy < 128; iy += 5)
        for (int iz = 0; iz < 128; ++iz) {
          const uint32_t k = tile_key(ix, iy, iz, g);
          const uint32_t tile = k >> 6, cls = (k >> 3) & 7u, blk = k & 7u;
          check(tile == tile_index(ix / 16, iy / 16, iz / 16), "key tile", k, ix);
          const uint32_t want_cls = (ix % 16 == 15) | ((iy % 16 == 15) << 1) | ((iz % 16 == 15) << 2);
          const uint32_t want_blk = ((ix % 16) >= 8) | (((iy % 16) >= 8) << 1) | (((iz % 16) >= 8) << 2);
          check(cls == want_cls, "key class", cls, want_cls);
          check(blk == want_blk, "key half-tile block", blk, want_blk);
        }
    // the 27 bins a paint tile reads: with off[k] = k, range r starts at
    // 8 * bin; each is (neighbour tile t - e, class c) with (c & e) == e
    std::vector<uint32_t> off((size_t)g.ntiles * 64 + 1);
    for (size_t k = 0; k < off.size(); ++k) off[k] = (uint32_t)k;
    for (int tz = 0; tz < 8; tz += 7)
      for (int ty = 0; ty < 8; ty += 3)
        for (int tx = 0; tx < 8; ++tx) {
          std::vector<int> got;
          for (int r = 0; r < 27; ++r) {
            uint32_t b0 = 0, b1 = 0;
            range_loads(off.data(), tx, ty, tz, g, r, b0, b1);
            check(b1 == b0 + 8 && b0 % 8 == 0, "bin is eight keys", b0, b1);
            got.push_back((int)(b0 / 8));
          }
          std::vector<int> want;
          for (int e = 0; e < 8; ++e)
            for (int c = 0; c < 8; ++c)
              if ((c & e) == e) {
                const uint32_t sx = (tx - (e & 1)) & 7, sy = (ty - ((e >> 1) & 1)) & 7, sz = (tz - ((e >> 2) & 1)) & 7;
                want.push_back((int)(tile_index(sx, sy, sz) * 8 + c));
              }
          check(got == want, "paint bins", got.size(), want.size());
        }
  }
  // lattice walk of the first sort
  for (int ln = 2; ln <= 7; ++ln) {
    const long n = 1L << ln, n3 = n * n * n;
    std::vector<char> seen((size_t)n3, 0);
    for (long t = 0; t < n3; ++t) {
      const long i = lattice_order(t, ln);
      check(i >= 0 && i < n3 && !seen[(size_t)i], "lattice walk is a bijection", t, i);
      if (i >= 0 && i < n3) seen[(size_t)i] = 1;
      // the wave's first lane fixes its 4^3 brick
      const long i0 = lattice_order(t & ~63L, ln);
      const long dx = (i >> (2 * ln)) - (i0 >> (2 * ln)), dy = ((i >> ln) & (n - 1)) - ((i0 >> ln) & (n - 1)),
                 dz = (i & (n - 1)) - (i0 & (n - 1));
      check(dx >= 0 && dx < 4 && dy >= 0 && dy < 4 && dz >= 0 && dz < 4, "one brick per wave", t, i);
    }
  }
  // periodic wrap
  const float xs[] = {-1e-7f, -0.5f, 0.f, 63.99999f, 64.f, 64.5f, 1000.25f, -1000.25f, NAN, INFINITY};
  for (float x : xs) {
    const float w = wrap_pos(x, 64.f);
    const bool in_range = w >= 0.f && w < 64.f;
    if (!in_range) std::printf("wrap_pos(%g) = %g\n", (double)x, (double)w);
    check(in_range, "wrap_pos range", 0, 0);
    if (std::isfinite(x) && std::fabs(x) < 1e3f) {
      const double d = std::fmod((double)w - (double)x, 64.0);
      const bool periodic = std::fabs(d) < 1e-3 || std::fabs(std::fabs(d) - 64.0) < 1e-3;
      if (!periodic) std::printf("wrap_pos(%g) = %g\n", (double)x, (double)w);
      check(periodic, "wrap_pos period", 0, 0);
    }
  }
  if (fails) {
    std::printf("%d failures\n", fails);
    return 1;
  }
  std::printf("sort index algebra ok\n");
  return 0;
}
