// MAP reconstruction of the initial white noise from the final overdensity
// (section 7, reconstruction from dark matter): the two elementwise passes
// around the forward run and its adjoint.
//
//   residual : the derivative of the chi^2 term, 2 (delta_m - delta_e) /
//              sigma^2, written over the model overdensity, and the chi^2
//              itself;
//   adam     : one Adam step (Kingma & Ba 2015, Algorithm 1) on the noise w
//              with the gradient of chi^2 + sum w^2, and the prior sum w^2.
//
// Both are HBM-bound streams (12 and 20 bytes per element); the sums are
// accumulated in float64, per workgroup and then in one workgroup, in a
// fixed order, so the reported losses are deterministic.
#include "recon.h"

namespace pmk {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) t += red[i];
  return t;
}

__global__ __launch_bounds__(kThreads) void k_residual(const float* d, const float* __restrict__ data, float* g,
                                                       long n, float inv_sigma, double* __restrict__ partials) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  const long stride = (long)gridDim.x * kThreads;
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
    const float r = (d[i] - data[i]) * inv_sigma;
    acc += (double)r * (double)r;
    g[i] = 2.f * r * inv_sigma;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(kThreads) void k_adam(float* __restrict__ w, const float* __restrict__ g_like,
                                                   float* __restrict__ m, float* __restrict__ v, long n, float lr,
                                                   float beta1, float beta2, float eps, float inv_bc1, float inv_bc2,
                                                   double* __restrict__ partials) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  const long stride = (long)gridDim.x * kThreads;
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
    const float wi = w[i];
    acc += (double)wi * (double)wi;
    const float g = g_like[i] + 2.f * wi;
    const float mi = beta1 * m[i] + (1.f - beta1) * g;
    const float vi = beta2 * v[i] + (1.f - beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    w[i] = wi - lr * (mi * inv_bc1) / (sqrtf(vi * inv_bc2) + eps);
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// one workgroup: the sum of nb partials, in a fixed order
__global__ __launch_bounds__(kThreads) void k_sum(const double* __restrict__ partials, int nb, double* __restrict__ out) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kThreads) acc += partials[i];
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) *out = t;
}

int blocks_for(long n) {
  const long b = (n + kThreads - 1) / kThreads;
  return (int)(b < kReducePartials ? (b < 1 ? 1 : b) : kReducePartials);
}

}  // namespace

void launch_residual(const float* delta, const float* data, float* grad, long n, float inv_sigma, double* partials,
                     double* out, hipStream_t s) {
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(k_residual, dim3(nb), dim3(kThreads), 0, s, delta, data, grad, n, inv_sigma, partials);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, s, partials, nb, out);
}

void launch_adam(float* w, const float* g_like, float* m, float* v, long n, float lr, float beta1, float beta2,
                 float eps, float inv_bc1, float inv_bc2, double* partials, double* out, hipStream_t s) {
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(k_adam, dim3(nb), dim3(kThreads), 0, s, w, g_like, m, v, n, lr, beta1, beta2, eps, inv_bc1,
                     inv_bc2, partials);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, s, partials, nb, out);
}

}  // namespace pmk
