// Adjoint (reverse-mode) kernels of the PM run for gfx950.
//
// The reverse sweep needs, at every force evaluation point x_j, the
// vector-Jacobian product of F(x) = readout(G paint(x), x) with a force
// cotangent F_bar = p_bar K (K the sum of the kicks that used F(x_j)):
//   term A  the readout positions: x_bar += sum_c dW/dx (F_bar . M(c)),
//           M the three force meshes recomputed from x_j;
//   term B  the painting positions: R_d = paint(x, F_bar_d) (3 channels,
//           the forward paint kernel with signed per-particle masses),
//           delta_bar = sum_d G_d^T R_d (G_d^T = -G_d, the FD kernel is odd),
//           x_bar += sum_c dW/dx (s delta_bar(c)), s = Ng^3 / Np.
// Cotangents live in particle-index order and are gathered and scattered
// through the sorted ids (each particle is owned by one thread).
#include "particles.h"
#include "pm_device.h"

namespace pmk {
namespace {

constexpr int kThreads = 256;

// x_bar[id] += sum_corners dW/dx * V(c), one sorted particle per thread:
//   NCH = 3: V(c) = k pbar[id] . F(c) with F the interleaved force mesh
//            (x-blocked cells of 3 floats)
//   NCH = 1: V(c) = k M(c) with M a real mesh, x-blocked (STD: [x][y][z])
//   ADD1 (with NCH = 3): V(c) += M1(c), a real x-blocked mesh with weight 1,
//            so that both terms of one force evaluation share one pass
template <int NCH, bool STD, bool ADD1 = false>
__global__ __launch_bounds__(kThreads) void k_readout_grad(const float* __restrict__ pos,
                                                           const uint32_t* __restrict__ id, long np, int n,
                                                           const float* __restrict__ mesh,
                                                           const float* __restrict__ pbar, float k,
                                                           float* __restrict__ xbar,
                                                           const float* __restrict__ m1 = nullptr) {
  const long j = (long)xcd_tile(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  if (j >= np) return;
  int ix, iy, iz;
  float fx, fy, fz;
  cic_base(pos[3 * j + 0], n, ix, fx);
  cic_base(pos[3 * j + 1], n, iy, fy);
  cic_base(pos[3 * j + 2], n, iz, fz);
  const long p = (long)id[j];
  // the by-id loads (the cotangent and the running x-bar) go out together,
  // before the corners; left in place, the x-bar load would follow the sum
  // and add a round trip at the end
  float c0 = k, c1 = 0.f, c2 = 0.f;
  if constexpr (NCH == 3) {
    c0 = pbar[3 * p + 0];
    c1 = pbar[3 * p + 1];
    c2 = pbar[3 * p + 2];
  }
  float xb[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) xb[d] = xbar[3 * p + d];
  asm volatile("" : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(xb[0]), "+v"(xb[1]), "+v"(xb[2]));
  if constexpr (NCH == 3) {
    c0 *= k;
    c1 *= k;
    c2 *= k;
  }
  const int jx = (ix + 1) & (n - 1), jy = (iy + 1) & (n - 1), jz = (iz + 1) & (n - 1);
  const int xs[2] = {ix, jx}, ys[2] = {iy, jy}, zs[2] = {iz, jz};
  const float wx[2] = {1.f - fx, fx}, wy[2] = {1.f - fy, fy}, wz[2] = {1.f - fz, fz};
  float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const long cell = STD ? ((long)xs[a] * n + ys[b]) * n + zs[c] : blk_real(xs[a], ys[b], zs[c], n);
        float val;
        if constexpr (NCH == 3)
          val = c0 * mesh[3 * cell] + c1 * mesh[3 * cell + 1] + c2 * mesh[3 * cell + 2];
        else
          val = c0 * mesh[cell];
        if constexpr (ADD1) val += m1[cell];
        const float sa = a ? 1.f : -1.f, sb = b ? 1.f : -1.f, sc = c ? 1.f : -1.f;
        gx += sa * wy[b] * wz[c] * val;
        gy += wx[a] * sb * wz[c] * val;
        gz += wx[a] * wy[b] * sc * val;
      }
  xbar[3 * p + 0] = xb[0] + gx;
  xbar[3 * p + 1] = xb[1] + gy;
  xbar[3 * p + 2] = xb[2] + gz;
}

// y += a x  (n floats)
__global__ void k_axpy(float* __restrict__ y, const float* __restrict__ x, float a, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] += a * x[i];
}

// LPT: s1_bar_d = cx1 xbar_d + cp1 pbar_d, s2_bar_d = cx2 xbar_d + cp2 pbar_d
// (particle index = lattice site, AoS [np3][3] -> three lattice fields each)
// (the fields are x-blocked: element e holds lattice site blk_real_xyz(e))
__global__ void k_lpt_sbar(const float* __restrict__ xbar, const float* __restrict__ pbar, long n3, int ln,
                           float cx1, float cp1, float cx2, float cp2, float* __restrict__ s10,
                           float* __restrict__ s11, float* __restrict__ s12, float* __restrict__ s20,
                           float* __restrict__ s21, float* __restrict__ s22) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n3; e += stride) {
    int x, y, z;
    blk_real_xyz(e, ln, x, y, z);
    const long i = ((((long)x << ln) + y) << ln) + z;
    const float x0 = xbar[3 * i], x1 = xbar[3 * i + 1], x2 = xbar[3 * i + 2];
    const float p0 = pbar[3 * i], p1 = pbar[3 * i + 1], p2 = pbar[3 * i + 2];
    s10[e] = cx1 * x0 + cp1 * p0;
    s11[e] = cx1 * x1 + cp1 * p1;
    s12[e] = cx1 * x2 + cp1 * p2;
    s20[e] = cx2 * x0 + cp2 * p0;
    s21[e] = cx2 * x1 + cp2 * p1;
    s22[e] = cx2 * x2 + cp2 * p2;
  }
}

// phi (xx, yy, zz, xy, xz, yz) -> phi_bar in place, given delta2_bar:
// phi_bar_ii = d2b (phi_jj + phi_kk), phi_bar_ij = -2 d2b phi_ij
__global__ void k_lpt_phibar(float* __restrict__ xx, float* __restrict__ yy, float* __restrict__ zz,
                             float* __restrict__ xy, float* __restrict__ xz, float* __restrict__ yz,
                             const float* __restrict__ d2b, long n3) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += stride) {
    const float a = xx[i], b = yy[i], c = zz[i], d = d2b[i];
    xx[i] = d * (b + c);
    yy[i] = d * (a + c);
    zz[i] = d * (a + b);
    xy[i] = -2.f * d * xy[i];
    xz[i] = -2.f * d * xz[i];
    yz[i] = -2.f * d * yz[i];
  }
}

inline int grid_for(long n) {
  long g = (n + kThreads - 1) / kThreads;
  if (g < 1) g = 1;
  return (int)(g > 65536 ? 65536 : g);
}

}  // namespace

void launch_readout_grad3(const float* pos, const uint32_t* id, long np, int n, const float* fi, const float* pbar,
                          float k, float* xbar, hipStream_t s) {
  const int grid = (int)((np + kThreads - 1) / kThreads);
  hipLaunchKernelGGL((k_readout_grad<3, false>), dim3(grid), dim3(kThreads), 0, s, pos, id, np, n, fi, pbar, k,
                     xbar);
}

void launch_readout_grad31(const float* pos, const uint32_t* id, long np, int n, const float* fi, const float* pbar,
                           float k, const float* m1, float* xbar, hipStream_t s) {
  const int grid = (int)((np + kThreads - 1) / kThreads);
  hipLaunchKernelGGL((k_readout_grad<3, false, true>), dim3(grid), dim3(kThreads), 0, s, pos, id, np, n, fi, pbar, k,
                     xbar, m1);
}

void launch_readout_grad1(const float* pos, const uint32_t* id, long np, int n, const float* m0, float k, float* xbar,
                          bool std_layout, hipStream_t s) {
  const int grid = (int)((np + kThreads - 1) / kThreads);
  if (std_layout)
    hipLaunchKernelGGL((k_readout_grad<1, true>), dim3(grid), dim3(kThreads), 0, s, pos, id, np, n, m0,
                       (const float*)nullptr, k, xbar);
  else
    hipLaunchKernelGGL((k_readout_grad<1, false>), dim3(grid), dim3(kThreads), 0, s, pos, id, np, n, m0,
                       (const float*)nullptr, k, xbar);
}

void launch_axpy(float* y, const float* x, float a, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(kThreads), 0, s, y, x, a, n);
}

void launch_lpt_sbar(const float* xbar, const float* pbar, long n3, float cx1, float cp1, float cx2, float cp2,
                     float* const* s1, float* const* s2, hipStream_t s) {
  int ln = 0;
  while ((1L << (3 * (ln + 1))) <= n3) ++ln;   // n3 = n^3, n a power of two
  hipLaunchKernelGGL(k_lpt_sbar, dim3(grid_for(n3)), dim3(kThreads), 0, s, xbar, pbar, n3, ln, cx1, cp1, cx2, cp2,
                     s1[0], s1[1], s1[2], s2[0], s2[1], s2[2]);
}

void launch_lpt_phibar(float* const* phi6, const float* d2b, long n3, hipStream_t s) {
  hipLaunchKernelGGL(k_lpt_phibar, dim3(grid_for(n3)), dim3(kThreads), 0, s, phi6[0], phi6[1], phi6[2], phi6[3],
                     phi6[4], phi6[5], d2b, n3);
}

}  // namespace pmk
