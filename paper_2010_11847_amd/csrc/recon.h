// Launchers of the reconstruction kernels (recon.hip): the likelihood
// residual of the final overdensity and the Adam update of the white noise,
// each with a float64 sum reduced per workgroup and then in one workgroup.
#pragma once

#include <hip/hip_runtime.h>

namespace pmk {

// Workgroups of the first reduction stage (the partial sums array holds
// this many doubles).
constexpr int kReducePartials = 1024;

// g = 2 (delta - data) / sigma^2 into grad (which may be delta itself) and
// *out = sum ((delta - data) / sigma)^2.
void launch_residual(const float* delta, const float* data, float* grad, long n, float inv_sigma, double* partials,
                     double* out, hipStream_t s);

// Adam on w with gradient g_like + 2 w (the white-noise prior), step
// lr * (m / bc1) / (sqrt(v / bc2) + eps); *out = sum w^2 before the update.
void launch_adam(float* w, const float* g_like, float* m, float* v, long n, float lr, float beta1, float beta2,
                 float eps, float inv_bc1, float inv_bc2, double* partials, double* out, hipStream_t s);

}  // namespace pmk
