// Device helpers shared by the particle and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "particles.h"

namespace pmk {

constexpr int kTileCells = 16 * 16 * 32;   // largest tile (LDS sizing)

// blockIdx -> tile so that consecutive tiles of one launch land on the same
// XCD (workgroups are dispatched round-robin over the 8 XCDs).
static __device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, slot = b >> 3;
  return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// Base cell (periodic) and fractional offset of one coordinate.
static __device__ __forceinline__ void cic_base(float x, int n, int& i, float& t) {
  const float f = floorf(x);
  t = x - f;
  i = ((int)f) & (n - 1);
}

static __device__ __forceinline__ float wrap_pos(float x, float n) {
  if (x < 0.f) x += n;
  if (x >= n) x -= n;
  if (!(x >= 0.f && x < n)) x = 0.f;    // rounding onto n, or non-finite
  return x;
}

static __device__ __forceinline__ uint32_t tile_key(int ix, int iy, int iz, const TileGeom& g) {
  const uint32_t tile = ((uint32_t)(ix / g.tx) * g.nty + (uint32_t)(iy / g.ty)) * g.ntz + (uint32_t)(iz / g.tz);
  const uint32_t c = (uint32_t)((ix % g.tx) == g.tx - 1) | ((uint32_t)((iy % g.ty) == g.ty - 1) << 1) |
                     ((uint32_t)((iz % g.tz) == g.tz - 1) << 2);
  return tile * 8u + c;
}

// Rank of this lane's key among all keys counted so far: lanes of a wave
// with equal keys share one atomic (particles arrive nearly sorted, so most
// waves hold one or two distinct keys).  Must be called by the whole wave.
static __device__ __forceinline__ uint32_t agg_rank(uint32_t* count, uint32_t key, bool valid) {
  uint64_t active = __ballot(valid);
  const int lane = __lane_id();
  uint32_t mine = 0;
  while (active) {
    const int leader = __ffsll((unsigned long long)active) - 1;
    const uint32_t lk = __shfl(key, leader);
    const bool same = valid && key == lk;
    const uint64_t mask = __ballot(same) & active;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&count[lk], (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (same) mine = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    active &= ~mask;
  }
  return mine;
}

// The 27 particle ranges a paint workgroup gathers: for every lower
// neighbour offset e in {0,1}^3 of tile (tx, ty, tz) (e = 0: the tile
// itself), the bins of classes c with (c & e) == e.  Filled cooperatively
// (one thread per range, loads issued in parallel); rpre holds the inclusive
// prefix sums of the range lengths, rstart the first particle of each range.
struct RangeTable {
  uint32_t start[27];
  uint32_t pre[28];
};

static __device__ __forceinline__ void build_ranges(RangeTable& rt, const uint32_t* __restrict__ off, int tx, int ty,
                                                    int tz, const TileGeom& g) {
  const int r = threadIdx.x;
  uint32_t len = 0;
  if (r < 27) {
    // enumerate (e, cls) pairs with (cls & e) == e in a fixed order
    int k = 0, e_sel = 0, c_sel = 0;
    for (int e = 0; e < 8; ++e)
      for (int c = 0; c < 8; ++c)
        if ((c & e) == e) {
          if (k == r) { e_sel = e; c_sel = c; }
          ++k;
        }
    const int sx = (tx - (e_sel & 1) + g.ntx) % g.ntx, sy = (ty - ((e_sel >> 1) & 1) + g.nty) % g.nty,
              sz = (tz - ((e_sel >> 2) & 1) + g.ntz) % g.ntz;
    const uint32_t bin = (((uint32_t)sx * g.nty + sy) * g.ntz + sz) * 8 + c_sel;
    const uint32_t b0 = off[bin], b1 = off[bin + 1];
    rt.start[r] = b0;
    len = b1 - b0;
    rt.pre[r + 1] = len;
  }
  if (r == 0) rt.pre[0] = 0;
  __syncthreads();
  if (r == 0) {
    for (int i = 1; i <= 27; ++i) rt.pre[i] += rt.pre[i - 1];
  }
  __syncthreads();
}

// particle index of flattened position idx < rt.pre[27]
static __device__ __forceinline__ uint32_t range_particle(const RangeTable& rt, uint32_t idx) {
  int lo = 0, hi = 27;   // find r with pre[r] <= idx < pre[r+1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rt.pre[mid] <= idx) lo = mid; else hi = mid;
  }
  return rt.start[lo] + (idx - rt.pre[lo]);
}

}  // namespace pmk
