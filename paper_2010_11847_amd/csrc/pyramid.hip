// Multi-grid (pyramid) passes of the two-level force (section 4.2,
// Algorithms 2 and 3).  REDUCE convolves with the 3-D B-spline of order 6
// (the tensor product of the 1-D weights C(6, k) / 64, k = 0..6) and keeps
// every second cell per axis; EXPAND is its transpose times 8, i.e. zeros
// inserted between cells and the same kernel times 2 per axis.  Both are
// separable, so each runs as three one-axis passes; a pass is a stream over
// its destination with 7 (REDUCE) or 4 (EXPAND) taps along the axis, the
// neighbouring taps served from cache: HBM-bound at one read of the source
// and one write of the destination.  Boundaries wrap (one device holds the
// whole periodic mesh); coarse cell i sits on fine cell 2 i.  Every field,
// intermediates included, is x-blocked by 8, so a wave's lanes walk
// consecutive addresses of both source and destination whatever the axis.
#include "layout.h"
#include "pyramid.h"

namespace pmk {
namespace {

constexpr int kThreads = 256;

// B-spline weights C(6, t + 3) / 64 at offsets t = -3..3
__device__ __forceinline__ float bw(int t) {
  switch (t < 0 ? -t : t) {
    case 0: return 20.f / 64.f;
    case 1: return 15.f / 64.f;
    case 2: return 6.f / 64.f;
    default: return 1.f / 64.f;
  }
}

struct Dims {
  int ly, lz;   // log2 of the destination's ny, nz
};

__device__ __forceinline__ long xoff(int x, int y, int z, int ny, int nz) {
  return ((((long)(x >> 3) * ny + y) * nz + z) << 3) + (x & 7);
}

__device__ __forceinline__ long pf_off(const PyrField& f, int c, int x, int y, int z) {
  const long e = xoff(x, y, z, f.ny, f.nz);
  return f.kind == PYR_SEPARATE ? e : 3 * e + c;
}

__device__ __forceinline__ float pf_load(const PyrField& f, int c, int x, int y, int z) {
  return (f.kind == PYR_INTERLEAVED ? f.p[0] : f.p[c])[pf_off(f, c, x, y, z)];
}

template <bool EXPAND, int AXIS, int CH>
__global__ __launch_bounds__(kThreads) void k_pyr_pass(PyrField src, PyrField dst, Dims dd, int mode,
                                                        const float* __restrict__ aux, float alpha) {
  const long total = (long)dst.nx * dst.ny * dst.nz;
  const long stride = (long)gridDim.x * kThreads;
  for (long e = (long)blockIdx.x * kThreads + threadIdx.x; e < total; e += stride) {
    // destination coordinates in its memory order (consecutive threads,
    // consecutive addresses)
    const long r = e >> 3;
    const int z = (int)(r & ((1L << dd.lz) - 1));
    const int y = (int)((r >> dd.lz) & ((1L << dd.ly) - 1));
    const int x = (int)(((r >> (dd.lz + dd.ly)) << 3) + (e & 7));
    const int o = AXIS == 0 ? x : (AXIS == 1 ? y : z);
    const int nin = AXIS == 0 ? src.nx : (AXIS == 1 ? src.ny : src.nz);
    float acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = 0.f;
    if (!EXPAND) {
      // out(o) = sum_t b(t) in(2 o + t)
#pragma unroll
      for (int t = -3; t <= 3; ++t) {
        const int i = (2 * o + t) & (nin - 1);
        const int sx = AXIS == 0 ? i : x, sy = AXIS == 1 ? i : y, sz = AXIS == 2 ? i : z;
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] += bw(t) * pf_load(src, c, sx, sy, sz);
      }
    } else {
      // out(j) = 2 sum_i b(j - 2 i) in(i): i = j/2 - 1 .. j/2 + 2
      const int i0 = o >> 1;
      const bool odd = o & 1;
#pragma unroll
      for (int u = -1; u <= 2; ++u) {
        const int t = o - 2 * (i0 + u);   // in [-3, 3] for odd o; u = 2 drops out for even o
        const float wgt = (!odd && u == 2) ? 0.f : 2.f * bw(t);
        const int i = (i0 + u) & (nin - 1);
        const int sx = AXIS == 0 ? i : x, sy = AXIS == 1 ? i : y, sz = AXIS == 2 ? i : z;
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] += wgt * pf_load(src, c, sx, sy, sz);
      }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      float* dp = (dst.kind == PYR_INTERLEAVED ? dst.p[0] : dst.p[c]) + pf_off(dst, c, x, y, z);
      if (mode == PYR_STORE)
        *dp = acc[c];
      else if (mode == PYR_COMBINE)
        *dp = alpha * aux[3 * xoff(x, y, z, dst.ny, dst.nz) + c] - acc[c];
      else if (mode == PYR_ADD)
        *dp += acc[c];
      else
        *dp -= acc[c];
    }
  }
}

template <bool EXPAND, int AXIS>
void launch_axis(int ch, const PyrField& src, const PyrField& dst, Dims dd, int mode, const float* aux, float alpha,
                 hipStream_t s) {
  const long total = (long)dst.nx * dst.ny * dst.nz;
  long blocks = (total + kThreads - 1) / kThreads;
  if (blocks > (1L << 20)) blocks = 1L << 20;
  const dim3 grid((unsigned)blocks);
  if (ch == 1)
    hipLaunchKernelGGL((k_pyr_pass<EXPAND, AXIS, 1>), grid, dim3(kThreads), 0, s, src, dst, dd, mode, aux, alpha);
  else
    hipLaunchKernelGGL((k_pyr_pass<EXPAND, AXIS, 3>), grid, dim3(kThreads), 0, s, src, dst, dd, mode, aux, alpha);
}

}  // namespace

void launch_pyr_pass(bool expand, int axis, int ch, const PyrField& src, const PyrField& dst, int mode,
                     const float* aux, float alpha, hipStream_t s) {
  const Dims dd{__builtin_ctz(dst.ny), __builtin_ctz(dst.nz)};
  if (expand) {
    if (axis == 0) launch_axis<true, 0>(ch, src, dst, dd, mode, aux, alpha, s);
    else if (axis == 1) launch_axis<true, 1>(ch, src, dst, dd, mode, aux, alpha, s);
    else launch_axis<true, 2>(ch, src, dst, dd, mode, aux, alpha, s);
  } else {
    if (axis == 0) launch_axis<false, 0>(ch, src, dst, dd, mode, aux, alpha, s);
    else if (axis == 1) launch_axis<false, 1>(ch, src, dst, dd, mode, aux, alpha, s);
    else launch_axis<false, 2>(ch, src, dst, dd, mode, aux, alpha, s);
  }
}

}  // namespace pmk
