// Internal declarations of the PM library: context, workspace layout and the
// launchers of the HIP kernels.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "batch.h"
#include "layout.h"
#include "pm.h"

namespace pmk {

// A real N^3 mesh in the x-blocked layout (layout.h), stored so that its
// r2c transform fits in place:
//   real view    r[N/8][N][N][8]       (float)
//   complex view c[N/8][N][N/2][8]     (float2, same bytes, kz = 0 .. N/2-1)
//   Nyquist plane q[N/8][N][8]         (float2, kz = N/2)
struct Field {
  float* r = nullptr;
  float2* q = nullptr;
  float2* c() const { return reinterpret_cast<float2*>(r); }
};

// Device tables of one FFT size N.
struct FftTables {
  int n = 0;
  float2* tw_n = nullptr;   // exp(-2 pi i k / N), k in [0, N)
  float2* tw_h = nullptr;   // exp(-2 pi i k / (N/2)), k in [0, N/2)
  // FD kernel tables (float32 from float64):  x/y axes use the signed
  // frequency of numpy's fftfreq, the z axis k in [0, N/2].
  float* dxy = nullptr;     // D(w)  = (8 sin w - sin 2w) / 6
  float* kxy = nullptr;     // K1(w) = (2 sin(w/2))^2
  float* wxy = nullptr;     // sinc^2(w/2)  (CIC window per axis)
  float* sxy = nullptr;     // exp(-w^2 rs^2) (split filter per axis)
  float* dz = nullptr;
  float* kz = nullptr;
  float* wz = nullptr;
  float* sz = nullptr;
};

// Spectral multiplication applied between the forward and the inverse x
// transforms of the fused x pass.
// Fan-out kinds read one input spectrum and write n_out outputs; fan-in
// kinds (the transposes, used by the adjoint) read n_in inputs and write the
// sum of their conjugate-multiplied spectra to one output; they overwrite
// their inputs.
enum SpecOpKind : int {
  OP_IDENTITY = 0,   // 1 output: X (round trip, scaled)
  OP_FORCE = 1,      // 3 outputs: i D_d g X with g = scale W^-n S / K^2
  OP_LPT1 = 2,       // 9 outputs from delta_L = X * pk[n^2]: s1 (3), phi_ij (6)
  OP_LPT2 = 3,       // 3 outputs: -i D_d / K^2 X * scale
  OP_LINEAR = 4,     // 1 output: X * pk[n^2]
  OP_LPT_PHI = 5,    // 6 outputs: phi_ij of delta_L = X * pk[n^2] (xx, yy, zz, xy, xz, yz)
  OP_FORCE_XS = 6,   // 2 outputs after the x pass: i D_x g X (F_x) and i g X, the factor
                     // F_y and F_z share until their y and z passes (N >= 64 only)
  OP_FORCE_T = 16,   // fan-in 3: sum_d conj(i D_d g) X_d
  OP_LPT2_T = 17,    // fan-in 3: sum_d conj(-i D_d scale / K^2) X_d
  OP_LPT1_T = 18,    // fan-in 9: pk[n^2] (sum_d conj(i D_d / K^2) X_d + sum_ij D_i D_j / K^2 X_ij)
};

inline bool op_fan_in(int kind) { return kind >= 16; }

constexpr int kMaxOut = 9;

struct SpecOp {
  int kind = OP_IDENTITY;
  int n_out = 1;
  int n_in = 1;
  float scale = 1.f;
  int deconv = 0;
  int split = 0;
  const float* pk = nullptr;  // table indexed by integer |n|^2
  float2* out_c[kMaxOut] = {};
  float2* out_q[kMaxOut] = {};
  // fan-in inputs (forward y transformed); the op consumes them: the first
  // input of the lowest D(w_x) power holds partial sums between launches
  float2* in_c[kMaxOut] = {};
  float2* in_q[kMaxOut] = {};
};

// ---- FFT launchers (fft.hip) ---------------------------------------------
// Forward r2c: z pass (real -> complex + Nyquist plane), then y pass.
void fft_r2c_zy(const FftTables& t, Field* f, int nf, hipStream_t s);
// Forward x pass only (complex, in place), for spectra that are measured.
void fft_x_forward(const FftTables& t, Field* f, int nf, hipStream_t s);
// Fused x pass: forward x transform of `in`, spectral op, inverse x
// transforms written to op.out_*.  `in` may alias out[0].
void fft_x_fused(const FftTables& t, const Field& in, const SpecOp& op, hipStream_t s);
// The force's x pass in one launch: forward x transform of `in`, times the
// Green's function, inverse x transforms into op.out_* (out[0] may alias
// `in`).  N >= 64 takes OP_FORCE_XS (out[0] = F_x, out[1] = the factor F_y
// and F_z share), smaller meshes OP_FORCE (three components).
// Batched launches (bat.d != null) cover every member of a plan; they need
// N >= 64, as do the batched forms of the passes below.
void fft_x_force(const FftTables& t, const Field& in, const SpecOp& op, hipStream_t s,
                 const BatchArg& bat = BatchArg());
// Inverse y pass of the three force meshes after an OP_FORCE_XS x pass:
// f[0] holds F_x, f[2] the shared factor i g X.  f[2] becomes F_z times
// D(w_z) in place and f[1] receives F_y = transform of D(w_y) i g X; one
// read of the shared factor feeds both.  N >= 64.
void fft_y_force(const FftTables& t, Field* f, hipStream_t s, const BatchArg& bat = BatchArg());
// x pass of the transposed force (OP_FORCE_T: op.scale, deconv, split) over
// the forward-(z, y) spectra f[0..2] of its x, y, z inputs; the result (the
// fan-in, inverse-x transformed) replaces f[0]; below 64^3 the other two
// inputs may be overwritten as well.
void fft_x_force_t(const FftTables& t, Field* f, const SpecOp& op, hipStream_t s);
// Single passes (the composites above call these).
void fft_z_r2c(const FftTables& t, Field* f, int nf, hipStream_t s, const BatchArg& bat = BatchArg());
void fft_y(const FftTables& t, Field* f, int nf, int dir, hipStream_t s, const BatchArg& bat = BatchArg());
void fft_z_c2r(const FftTables& t, Field* f, int nf, hipStream_t s);
// z pass of three fields written as one interleaved real mesh
// out[x/8][y][z][x%8][3] (the force meshes the particle readout gathers from).
// The three fields must be equally spaced in memory (f[2] - f[1] == f[1] - f[0]
// for both the arrays and the Nyquist planes), as the workspace meshes are.
void fft_z_c2r_interleaved3(const FftTables& t, const Field* f, float* out, hipStream_t s,
                            const BatchArg& bat = BatchArg());
// Inverse: y pass then z pass (complex + Nyquist plane -> real), unnormalised.
void fft_c2r_yz(const FftTables& t, Field* f, int nf, hipStream_t s);
// Plain inverse x pass (complex, in place).
void fft_x_inverse(const FftTables& t, Field* f, int nf, hipStream_t s);

}  // namespace pmk
