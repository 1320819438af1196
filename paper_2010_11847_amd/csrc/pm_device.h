// Device helpers shared by the particle and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "particles.h"

namespace pmk {

constexpr int kTileMax = 16;   // largest tile side (LDS sizing)

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
  const int t = g.t;
  const uint32_t tile = ((uint32_t)(ix / t) * g.nt + (uint32_t)(iy / t)) * g.nt + (uint32_t)(iz / t);
  const uint32_t c = (uint32_t)((ix % t) == t - 1) | ((uint32_t)((iy % t) == t - 1) << 1) |
                     ((uint32_t)((iz % t) == t - 1) << 2);
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

}  // namespace pmk
