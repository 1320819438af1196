// Multi-grid (pyramid) passes of the two-level force (section 5.2,
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

// Field kinds of a pass: PYR_SEPARATE or PYR_INTERLEAVED known at compile
// time, so that the three adjacent channels of an interleaved cell move as
// one 12-byte access; kAnyKind reads the kind at run time.
constexpr int kAnyKind = -1;

template <int KIND>
__device__ __forceinline__ bool is_interleaved(const PyrField& f) {
  return KIND == kAnyKind ? f.kind == PYR_INTERLEAVED : KIND == PYR_INTERLEAVED;
}

// the CH channel values of cell (x, y, z)
template <int CH, int KIND>
__device__ __forceinline__ void cell_load(const PyrField& f, int x, int y, int z, float (&v)[CH]) {
  const long e = xoff(x, y, z, f.ny, f.nz);
  if (is_interleaved<KIND>(f)) {
#pragma unroll
    for (int c = 0; c < CH; ++c) v[c] = f.p[0][3 * e + c];
  } else {
#pragma unroll
    for (int c = 0; c < CH; ++c) v[c] = f.p[c][e];
  }
}

template <bool EXPAND, int AXIS, int CH, int SK, int DK>
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
        float v[CH];
        cell_load<CH, SK>(src, sx, sy, sz, v);
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] += bw(t) * v[c];
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
        float v[CH];
        cell_load<CH, SK>(src, sx, sy, sz, v);
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] += wgt * v[c];
      }
    }
    // one loop per mode, so that the channels of an interleaved cell merge
    const long de = xoff(x, y, z, dst.ny, dst.nz);
    const bool dil = is_interleaved<DK>(dst);
    auto dptr = [&](int c) { return dil ? dst.p[0] + 3 * de + c : dst.p[c] + de; };
    if (mode == PYR_STORE) {
#pragma unroll
      for (int c = 0; c < CH; ++c) *dptr(c) = acc[c];
    } else if (mode == PYR_COMBINE) {
      float av[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) av[c] = aux[3 * de + c];
#pragma unroll
      for (int c = 0; c < CH; ++c) *dptr(c) = alpha * av[c] - acc[c];
    } else {
      const float sg = mode == PYR_ADD ? 1.f : -1.f;
      float dv[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) dv[c] = *dptr(c);
#pragma unroll
      for (int c = 0; c < CH; ++c) *dptr(c) = dv[c] + sg * acc[c];
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
  constexpr int SEP = PYR_SEPARATE, IL = PYR_INTERLEAVED;
  const int sk = src.kind, dk = dst.kind;
  if (ch == 1)
    hipLaunchKernelGGL((k_pyr_pass<EXPAND, AXIS, 1, kAnyKind, kAnyKind>), grid, dim3(kThreads), 0, s, src, dst, dd,
                       mode, aux, alpha);
  else if (sk == SEP && dk == SEP)
    hipLaunchKernelGGL((k_pyr_pass<EXPAND, AXIS, 3, SEP, SEP>), grid, dim3(kThreads), 0, s, src, dst, dd, mode, aux,
                       alpha);
  else if (sk == IL && dk == SEP)
    hipLaunchKernelGGL((k_pyr_pass<EXPAND, AXIS, 3, IL, SEP>), grid, dim3(kThreads), 0, s, src, dst, dd, mode, aux,
                       alpha);
  else if (sk == SEP && dk == IL)
    hipLaunchKernelGGL((k_pyr_pass<EXPAND, AXIS, 3, SEP, IL>), grid, dim3(kThreads), 0, s, src, dst, dd, mode, aux,
                       alpha);
  else if (sk == IL && dk == IL)
    hipLaunchKernelGGL((k_pyr_pass<EXPAND, AXIS, 3, IL, IL>), grid, dim3(kThreads), 0, s, src, dst, dd, mode, aux,
                       alpha);
  else
    hipLaunchKernelGGL((k_pyr_pass<EXPAND, AXIS, 3, kAnyKind, kAnyKind>), grid, dim3(kThreads), 0, s, src, dst, dd,
                       mode, aux, alpha);
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
