// Device helpers shared by the particle and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "particles.h"

namespace pmk {

constexpr int kTileCells = 16 * 16 * 16;   // largest tile (LDS sizing)

// blockIdx -> tile so that consecutive tiles of one launch land on the same
// XCD (workgroups are dispatched round-robin over the 8 XCDs).
static __device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, slot = b >> 3;
  return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// Base cell (periodic) and fractional offset of one coordinate.
static __host__ __device__ __forceinline__ void cic_base(float x, int n, int& i, float& t) {
  const float f = floorf(x);
  t = x - f;
  i = ((int)f) & (n - 1);
}

// Periodic wrap into [0, n): x - n floor(x / n) for any finite x (n is a
// power of two, so x / n is exact); a result that rounds onto n becomes 0.
// Non-finite positions (invalid input) become 0 so that every later index
// stays inside the mesh.
static __host__ __device__ __forceinline__ float wrap_pos(float x, float n) {
  if (x < 0.f || x >= n) x -= n * floorf(x * (1.f / n));
  if (!(x >= 0.f && x < n)) x = 0.f;
  return x;
}

// Sort key of a particle with CIC base cell (ix, iy, iz):
//   ((tile * 8 + class) * 8 + sub)
// class bit d: the base cell is the last of its tile along d (the particle
// also deposits into the next tile); sub bit d (x lowest, as in the tile
// numbering): the base cell lies in the upper half of the tile along d.
// Paint gathers whole (tile, class) bins,
// eight consecutive keys; inside a bin the half-tile blocks keep the
// particles that one wave reads out close together in the force mesh.
// Tiles are numbered along a Morton (Z-order) curve: the bits of (t_x,
// t_y, t_z) interleaved, t_x lowest (the tiling is cubic, ntx = nty = ntz,
// a power of two up to 2^10).  Tiles close in the sort are then close in
// all three directions, so that the neighbours whose lines a tile shares
// (force-mesh faces, count lines, bins) were walked recently.
static __host__ __device__ __forceinline__ uint32_t morton_spread(uint32_t v) {   // bit i -> bit 3i, v < 2^10
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
static __host__ __device__ __forceinline__ uint32_t morton_compact(uint32_t v) {   // bit 3i -> bit i
  v &= 0x09249249u;
  v = (v ^ (v >> 2)) & 0x030C30C3u;
  v = (v ^ (v >> 4)) & 0x0300F00Fu;
  v = (v ^ (v >> 8)) & 0xFF0000FFu;
  v = (v ^ (v >> 16)) & 0x000003FFu;
  return v;
}
static __host__ __device__ __forceinline__ uint32_t tile_index(uint32_t tx, uint32_t ty, uint32_t tz) {
  return morton_spread(tx) | (morton_spread(ty) << 1) | (morton_spread(tz) << 2);
}

// Particle visited by thread t of a pass over n^3 particles in lattice order
// (index (q_x n + q_y) n + q_z, n = 2^ln >= 4): each wave takes one 4^3
// brick of lattice sites, and the bricks follow the Morton curve of the
// tiles, so that a wave's particles (still near their sites) share a sort
// key and consecutive waves fill consecutive destinations.  A bijection on
// [0, n^3) whatever the positions.
static __host__ __device__ __forceinline__ long lattice_order(long t, int ln) {
  const uint32_t lane = (uint32_t)t & 63u, brick = (uint32_t)(t >> 6);
  const uint32_t qx = (morton_compact(brick) << 2) | (lane >> 4);
  const uint32_t qy = (morton_compact(brick >> 1) << 2) | ((lane >> 2) & 3u);
  const uint32_t qz = (morton_compact(brick >> 2) << 2) | (lane & 3u);
  return ((long)qx << (2 * ln)) | ((long)qy << ln) | (long)qz;
}

static __host__ __device__ __forceinline__ uint32_t tile_key(int ix, int iy, int iz, const TileGeom& g) {
  const uint32_t tile = tile_index((uint32_t)ix >> g.lx, (uint32_t)iy >> g.ly, (uint32_t)iz >> g.lz);
  const uint32_t lx = (uint32_t)ix & (g.tx - 1), ly = (uint32_t)iy & (g.ty - 1), lz = (uint32_t)iz & (g.tz - 1);
  const uint32_t c = (uint32_t)(lx == (uint32_t)g.tx - 1) | ((uint32_t)(ly == (uint32_t)g.ty - 1) << 1) |
                     ((uint32_t)(lz == (uint32_t)g.tz - 1) << 2);
  const uint32_t sub = ((lz >> (g.lz - 1)) << 2) | ((ly >> (g.ly - 1)) << 1) | (lx >> (g.lx - 1));
  return (tile * 8u + c) * 8u + sub;
}

// (x, y, z) tile coordinates of a flattened tile index
static __host__ __device__ __forceinline__ void tile_coords(int tile, const TileGeom& g, int& tx, int& ty, int& tz) {
  (void)g;
  tx = (int)morton_compact((uint32_t)tile);
  ty = (int)morton_compact((uint32_t)tile >> 1);
  tz = (int)morton_compact((uint32_t)tile >> 2);
}

// LDS slot of tile cell (cx, cy, cz): z fastest, rows of tz cells, with the
// z bits XOR-swizzled by (cx%8, bit 1 of cy) so that
//  - the atomics of a wave of lattice-ordered particles (steps of 2 cells in
//    z and y) spread over all banks instead of the even ones, and
//  - the store loop, whose lanes run over x%8 fastest (the x-blocked mesh),
//    reads rows that start on different banks.
// The swizzle permutes cells within a row, so slots stay in [0, tx*ty*tz).
static __device__ __forceinline__ int tile_li(int cx, int cy, int cz, const TileGeom& g) {
  const int swz = (((cx & 7) << 3) | ((cy >> 1) & 1)) & (g.tz - 1);
  return ((((cx << g.ly) | cy) << g.lz) | (cz ^ swz));
}
static __device__ __forceinline__ int tile_cells(const TileGeom& g) { return g.tx * g.ty * g.tz; }
// the i-th cell of the store walk: x%8 fastest, then z, y, x/8 (contiguous
// runs of the x-blocked mesh); tiles narrower than 8 cells along x skip the
// cells with cx >= tx
static __device__ __forceinline__ int store_walk_len(const TileGeom& g) { return ((g.tx + 7) >> 3) * 8 * g.ty * g.tz; }
static __device__ __forceinline__ void store_walk(int c, const TileGeom& g, int& cx, int& cy, int& cz) {
  const int r = c >> 3;
  cz = r & (g.tz - 1);
  cy = (r >> g.lz) & (g.ty - 1);
  cx = ((r >> (g.lz + g.ly)) << 3) | (c & 7);
}

// (x, y, z) cell offsets inside a tile of flattened cell index c (z fastest)
static __device__ __forceinline__ void cell_coords(int c, const TileGeom& g, int& cx, int& cy, int& cz) {
  cz = c & (g.tz - 1);
  cy = (c >> g.lz) & (g.ty - 1);
  cx = c >> (g.lz + g.ly);
}

// Rank of this lane's key among all keys counted so far (count[key] is
// advanced by the group and its old value returned).  Lanes of a wave with
// equal keys share one atomic: the groups are found with ballots
// first, then every group leader issues its atomic in the same instruction,
// so the wave waits for one atomic round trip however many distinct keys it
// holds (particles in lattice order span several tiles per wave).  Must be
// called by the whole wave.
static __device__ __forceinline__ uint32_t agg_rank(uint32_t* count, uint32_t key, bool valid) {
  uint64_t active = __ballot(valid);
  const int lane = __lane_id();
  int my_leader = lane;
  uint32_t my_prefix = 0, group = 0;
  while (active) {
    const int leader = __ffsll((unsigned long long)active) - 1;
    const uint32_t lk = __shfl(key, leader);
    const bool same = valid && key == lk;
    const uint64_t mask = __ballot(same) & active;
    if (same) {
      my_leader = leader;
      my_prefix = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    }
    if (lane == leader) group = (uint32_t)__popcll(mask);
    active &= ~mask;
  }
  uint32_t base = 0;
  if (group) base = atomicAdd(&count[key], group);
  base = __shfl(base, my_leader);
  return valid ? base + my_prefix : 0u;
}

// count[key] += 1 for this lane's key, one atomic per group of equal keys in
// the wave, none of them waited for (the counts are read by a later
// kernel).  Must be called by the whole wave.
static __device__ __forceinline__ void agg_count(uint32_t* count, uint32_t key, bool valid) {
  uint64_t active = __ballot(valid);
  const int lane = __lane_id();
  uint32_t group = 0;
  while (active) {
    const int leader = __ffsll((unsigned long long)active) - 1;
    const uint32_t lk = __shfl(key, leader);
    const uint64_t mask = __ballot(valid && key == lk) & active;
    if (lane == leader) group = (uint32_t)__popcll(mask);
    active &= ~mask;
  }
  if (group) (void)atomicAdd(&count[key], group);
}

// The 27 particle ranges a paint workgroup gathers: for every lower
// neighbour offset e in {0,1}^3 of tile (tx, ty, tz) (e = 0: the tile
// itself), the bins of classes c with (c & e) == e.  Filled cooperatively
// (one thread per range, loads issued in parallel); rpre holds the inclusive
// prefix sums of the range lengths, rstart the first particle of each range.
struct RangeTable {
  uint32_t start[27];
  uint32_t pre[32];   // exclusive prefix of the range lengths; pre[27] = total, pre[28..31] = ~0
};

// Ranges of the 27 (neighbour tile, class) bins whose particles deposit
// into tile (tx, ty, tz), in two halves so that the loads can be issued
// early: range_loads (lanes r < 27 of wave 0) reads the offsets of range r,
// range_publish (the whole of wave 0) scans the lengths with lane shuffles
// and writes the table; a barrier must follow before other waves read it.
static __host__ __device__ __forceinline__ void range_loads(const uint32_t* __restrict__ off, int tx, int ty, int tz,
                                                   const TileGeom& g, int r, uint32_t& b0, uint32_t& b1) {
  // enumerate (e, cls) pairs with (cls & e) == e in a fixed order
  int k = 0, e_sel = 0, c_sel = 0;
  for (int e = 0; e < 8; ++e)
    for (int c = 0; c < 8; ++c)
      if ((c & e) == e) {
        if (k == r) { e_sel = e; c_sel = c; }
        ++k;
      }
  const int sx = (tx - (e_sel & 1)) & (g.ntx - 1), sy = (ty - ((e_sel >> 1) & 1)) & (g.nty - 1),
            sz = (tz - ((e_sel >> 2) & 1)) & (g.ntz - 1);
  const uint32_t bin = tile_index((uint32_t)sx, (uint32_t)sy, (uint32_t)sz) * 8 + c_sel;
  b0 = off[bin * 8];       // its eight half-tile keys
  b1 = off[bin * 8 + 8];
}
static __device__ __forceinline__ void range_publish(RangeTable& rt, int r, uint32_t b0, uint32_t b1) {
  const uint32_t len = r < 27 ? b1 - b0 : 0u;
  if (r < 27) rt.start[r] = b0;
  uint32_t v = len;   // inclusive scan over lanes 0..31
#pragma unroll
  for (int d = 1; d < 32; d <<= 1) {
    const uint32_t t = __shfl_up(v, d, 64);
    if (r >= d) v += t;
  }
  if (r < 27) rt.pre[r + 1] = v;
  if (r == 0) rt.pre[0] = 0;
  if (r >= 28 && r < 32) rt.pre[r] = 0xFFFFFFFFu;
}
// Both halves by wave 0, then one barrier that publishes the table.
static __device__ __forceinline__ void build_ranges(RangeTable& rt, const uint32_t* __restrict__ off, int tx, int ty,
                                                    int tz, const TileGeom& g) {
  const int r = threadIdx.x;
  if (r < 64) {
    uint32_t b0 = 0, b1 = 0;
    if (r < 27) range_loads(off, tx, ty, tz, g, r, b0, b1);
    range_publish(rt, r, b0, b1);
  }
  __syncthreads();
}

// particle index of flattened position idx < rt.pre[27]: the range r with
// pre[r] <= idx < pre[r+1], by a fixed five-step search (no loop)
static __device__ __forceinline__ uint32_t range_particle(const RangeTable& rt, uint32_t idx) {
  uint32_t lo = 0;
#pragma unroll
  for (uint32_t step = 16; step > 0; step >>= 1)
    if (rt.pre[lo + step] <= idx) lo += step;
  return rt.start[lo] + (idx - rt.pre[lo]);
}

}  // namespace pmk
