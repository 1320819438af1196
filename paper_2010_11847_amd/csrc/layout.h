// Mesh layout shared by every kernel of the library ("x-blocked by 8").
//
// A real N^3 field is stored as          r[x/8][y][z][x%8]      (float)
// its half spectrum kz < N/2 as          c[kx/8][ky][kz][kx%8]  (float2)
// in the same bytes, and the Nyquist     q[kx/8][ky][kx%8]      (float2)
// plane kz = N/2 in its own array.
//
// Eight consecutive x share one 32-byte (real) or 64-byte (complex) run, so
// a pass along x reads 512-byte runs from N/8 rows 4N^2 complex apart
// instead of 64-byte runs from N rows, one per 4 MB plane at N = 1024: the
// pass touches 8x fewer pages per tile.  The z passes still work in place:
// the 8N reals of one (x/8, y) row and the 4N complex values of its spectrum
// are the same bytes.  A "line" (x, y) has index l = blk_line(x, y): eight
// consecutive lines are the eight x of one row.
#pragma once

#include <hip/hip_runtime.h>

namespace pmk {

__host__ __device__ inline long blk_line(int x, int y, int n) { return (((long)(x >> 3) * n + y) << 3) + (x & 7); }

__host__ __device__ inline long blk_real(int x, int y, int z, int n) {
  return ((((long)(x >> 3) * n + y) * n + z) << 3) + (x & 7);
}

__host__ __device__ inline long blk_spec(int kx, int ky, int kz, int n) {
  return ((((long)(kx >> 3) * n + ky) * (n >> 1) + kz) << 3) + (kx & 7);
}

__host__ __device__ inline long blk_nyq(int kx, int ky, int n) { return blk_line(kx, ky, n); }

// Inverse of blk_real for a power-of-two n = 2^ln: (x, y, z) of element e.
__host__ __device__ inline void blk_real_xyz(long e, int ln, int& x, int& y, int& z) {
  const int xi = (int)(e & 7);
  const long r = e >> 3;
  z = (int)(r & ((1L << ln) - 1));
  y = (int)((r >> ln) & ((1L << ln) - 1));
  x = (int)((r >> (2 * ln)) << 3) + xi;
}

}  // namespace pmk
