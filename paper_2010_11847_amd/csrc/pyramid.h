// Launchers of the multi-grid (pyramid) passes (pyramid.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace pmk {

// A 3-D field of up to three channels, x-blocked by 8 like every mesh of the
// library, with power-of-2 dims (nx >= 8):
//   PYR_SEPARATE    p[c] + xoff(x, y, z)
//   PYR_INTERLEAVED p[0] + 3 * xoff(x, y, z) + c
// xoff(x, y, z) = (((x / 8) * ny + y) * nz + z) * 8 + x % 8, which for a cube
// is blk_real.  All passes walk their destination in this memory order.
enum PyrKind : int { PYR_SEPARATE = 0, PYR_INTERLEAVED = 1 };

struct PyrField {
  float* p[3] = {nullptr, nullptr, nullptr};
  int kind = PYR_SEPARATE;
  int nx = 0, ny = 0, nz = 0;
};

// How a pass writes its value v to the destination.
enum PyrMode : int {
  PYR_STORE = 0,     // dst = v
  PYR_COMBINE = 1,   // dst = alpha * aux - v   (aux: interleaved, dst's cube)
  PYR_ADD = 2,       // dst += v
  PYR_SUB = 3,       // dst -= v
};

// One separable pass along axis (0 = x, 1 = y, 2 = z) of REDUCE (centred
// stride-2 convolution with the order-6 B-spline, the axis halves) or of
// EXPAND (the transposed convolution times 2, the axis doubles), periodic,
// over ch channels.  dst's dims must be src's with that axis halved or
// doubled.
void launch_pyr_pass(bool expand, int axis, int ch, const PyrField& src, const PyrField& dst, int mode,
                     const float* aux, float alpha, hipStream_t s);

}  // namespace pmk
