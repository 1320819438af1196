// Launchers and argument blocks of the particle-side kernels (particles.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch.h"
#include "layout.h"

namespace pmk {

// Tiles of tx * ty * tz cells (tz is the contiguous axis): ntx * nty * ntz
// tiles (ntx = nty = ntz), numbered along a Morton curve (tile_index in
// pm_device.h).
// Every size here is a power of two; the log2 fields let kernels split
// indices with shifts and masks instead of integer division.
struct TileGeom {
  int n = 0;                   // mesh cells per side
  int tx = 0, ty = 0, tz = 0;  // tile size in cells
  int ntx = 0, nty = 0, ntz = 0;
  int ntiles = 0;
  int lx = 0, ly = 0, lz = 0;        // log2 of tx, ty, tz
  int lnx = 0, lny = 0, lnz = 0;     // log2 of ntx, nty, ntz
};

// Paint/sort tiles of the n^3 mesh: 16^3 cells, or n/2 per side below 32^3
// (at least two tiles per side, so that a particle's 7 upper CIC neighbours
// never wrap into its own tile).
TileGeom make_tile_geom(int n);

struct LptParticleArgs {
  int np = 0;             // particles per side
  int ratio = 1;          // B = n_mesh / n_part
  float shift = 0.f;
  float nmesh = 0.f;
  float cx1 = 0.f, cx2 = 0.f;   // B D1, B D2
  float cp1 = 0.f, cp2 = 0.f;   // B a0^2 E f1 D1, B a0^2 E f2 D2
  const float* s1[3] = {};      // device pointers, passed by value
  const float* s2[3] = {};      // device pointers; used when has_s2
  int has_s2 = 0;
  float* pos = nullptr;
  float* mom = nullptr;
  float* psi1 = nullptr;        // optional: B s1 and B s2 by particle, [np][3] (the COLA frame)
  float* psi2 = nullptr;
};

struct ScatterArgs {
  long np = 0;
  const float* pos = nullptr;
  const float* mom = nullptr;      // may be null
  const uint32_t* id = nullptr;    // null: identity
  const uint32_t* key = nullptr;
  uint32_t* cursor = nullptr;      // per key: the next free slot (the scan's copy of the offsets)
  float* pos_out = nullptr;
  float* mom_out = nullptr;
  uint32_t* id_out = nullptr;
  int lat_ln = -1;                 // >= 0: the source is in lattice order over 2^(3 lat_ln) particles
  BatchArg bat;                    // batched: every pointer is a workspace pointer of member 0
};

enum ReadoutFlags : int {
  RO_KICK = 1,           // p += F kick_a; (checkpoint); p += F kick_b
  RO_DRIFT = 2,          // x += p drift, wrapped
  RO_WRITE_SORTED = 4,   // write x, p back in sorted order
  RO_XP_BYID = 8,        // write x, p to pos_out/mom_out at the particle id
  RO_FORCE_BYID = 16,    // write F to force_out at the particle id
  RO_KEYS = 32,          // tile key of the new position, counted per key
  RO_CKPT = 64,          // write x and p (after kick_a) to ckpt_x/ckpt_p at the id
  RO_TO_ALT = 128,       // write x, p and the id to pos_alt/mom_alt/id_alt at the same (sorted) index
  RO_COLA = 256,         // LPT frame: kick with F - c1 psi1 - c2 psi2, drift adds dD1 psi1 + dD2 psi2
  RO_COLA_OUT = 512,     // momentum written by id is p + q1 psi1 + q2 psi2 (cola_out)
};

struct ReadoutArgs {
  TileGeom g;
  long np = 0;
  float* pos = nullptr;            // sorted
  float* mom = nullptr;            // sorted, may be null
  const uint32_t* id = nullptr;    // sorted ids
  const float* fi = nullptr;       // force mesh, interleaved x-blocked [n/8][n][n][8][3]
  float kick_a = 0.f, kick_b = 0.f, drift = 0.f;
  int flags = 0;
  float* force_out = nullptr;
  float* pos_out = nullptr;
  float* mom_out = nullptr;
  float* ckpt_x = nullptr;
  float* ckpt_p = nullptr;
  uint32_t* key_out = nullptr;
  uint32_t* count = nullptr;
  // A run's step loop reads its factors from device memory, so that one
  // captured graph serves every step: at i = *step_i, steps[i] = {kick_a,
  // kick_b, drift, 0} and, with RO_CKPT, the checkpoint pair starts at
  // *ckpt_base + 2 i ckpt_stride floats.  steps == null: the fields above.
  const float4* steps = nullptr;
  const uint32_t* step_i = nullptr;
  float* const* ckpt_base = nullptr;
  long ckpt_stride = 0;
  // RO_COLA: the frame's fields by particle id and its factors {c1, c2, dD1,
  // dD2}, per step from cola_steps[*step_i] when steps is set, else `cola`
  const float* psi1 = nullptr;
  const float* psi2 = nullptr;
  const float4* cola_steps = nullptr;
  float4 cola = {0.f, 0.f, 0.f, 0.f};
  float2 cola_out = {0.f, 0.f};
  // RO_TO_ALT destinations
  float* pos_alt = nullptr;
  float* mom_alt = nullptr;
  uint32_t* id_alt = nullptr;
  // Batched (bat.d != null): every pointer above is a workspace pointer of
  // member 0; the factors and checkpoint pointers come from the member's
  // descriptor (kick_close, kick_open, drift; RO_CKPT if it asks for it).
  BatchArg bat;
};

struct PowerArgs {
  int n = 0;
  int n_bins = 0;
  int n_max = 0;
  int deconv = 0;
  const float2* c = nullptr;
  const float2* q = nullptr;
  const float* wxy = nullptr;
  const float* wz = nullptr;
  double* partial = nullptr;
};

// white noise of n_side^3 sites; blocked: x-blocked layout, else [x][y][z]
void launch_noise(uint64_t seed, int n_side, float* out, bool blocked, hipStream_t s);
// plain [x][y][z] <-> x-blocked copy of a real n_side^3 mesh (out != in)
void launch_relayout(const float* in, float* out, int n_side, bool to_blocked, hipStream_t s);
void launch_lpt_delta2(float* const* phi6, long n, float* out, hipStream_t s);
void launch_lpt_particles(const LptParticleArgs& a, hipStream_t s);
void launch_fill_u32(uint32_t* p, long n, uint32_t v, hipStream_t s, const BatchArg& bat = BatchArg());
// tile keys of np particles, counted per key into count (zeroed first)
// lat_ln >= 0: the np = 2^(3 lat_ln) particles are in lattice order, and the
// pass walks them brick by brick (lattice_order in pm_device.h)
void launch_keys(const float* pos, long np, const TileGeom& g, uint32_t* key, uint32_t* count, hipStream_t s,
                 int lat_ln = -1);
long scan_scratch_words(long n);
// off = exclusive scan of count[0..n), off[n] = total; count[0..n) is then
// overwritten with a copy of off[0..n) (the scatter's cursors)
void launch_scan(uint32_t* count, long n, uint32_t* off, uint32_t* bsum, hipStream_t s,
                 const BatchArg& bat = BatchArg());
void launch_scatter(const ScatterArgs& a, hipStream_t s);
// std_layout: write [x][y][z] instead of the x-blocked layout
void launch_paint(const float* pos_sorted, const uint32_t* off, const TileGeom& g, float* out, float scale,
                  float offset, bool std_layout, hipStream_t s, const BatchArg& bat = BatchArg());
void launch_readout(const ReadoutArgs& a, hipStream_t s);
// *ctr += 1 (the step counter of a run's device-side step loop)
void launch_step_inc(uint32_t* ctr, hipStream_t s);
// *bits = bit pattern of max_i |v_i| over n floats
void launch_absmax(const float* v, long n, uint32_t* bits, hipStream_t s);
// x-blocked paint of signed masses wts[3 id + comp] * k (the adjoint's
// cotangent channels); *maxbits must hold max |wts| (launch_absmax).
// comp < 0: the three components in one launch, component d into
// out + d * out_stride.
void launch_paint_weighted(const float* pos_sorted, const uint32_t* id_sorted, const uint32_t* off, const TileGeom& g,
                           const float* wts, int comp, float k, const uint32_t* maxbits, float* out, hipStream_t s,
                           long out_stride = 0);
void launch_kick_drift(float* pos, float* mom, const float* f, long np, float kick, float drift, float nmesh,
                       hipStream_t s);
// mom[j] += u1 psi1[id[j]] + u2 psi2[id[j]] over np sorted particles (the
// change between the full and the LPT-frame momentum)
void launch_frame_shift(float* mom, const uint32_t* id, const float* psi1, const float* psi2, long np, float u1,
                        float u2, hipStream_t s);
void launch_spec_to_numpy(const float2* c, const float2* q, float2* out, int n, float scale, hipStream_t s);
void launch_spec_from_numpy(const float2* in, float2* c, float2* q, int n, float scale, hipStream_t s);
void launch_scale(float* p, long n, float v, hipStream_t s);
// adjoint kernels (adjoint.hip)
void launch_readout_grad3(const float* pos, const uint32_t* id, long np, int n, const float* fi, const float* pbar,
                          float k, float* xbar, hipStream_t s);
// Both readout terms of one force evaluation in one pass: the readout_grad3
// term plus that of the real x-blocked mesh m1 with weight 1.
void launch_readout_grad31(const float* pos, const uint32_t* id, long np, int n, const float* fi, const float* pbar,
                           float k, const float* m1, float* xbar, hipStream_t s);
// m0: real mesh, x-blocked (std_layout: plain [x][y][z])
void launch_readout_grad1(const float* pos, const uint32_t* id, long np, int n, const float* m0, float k, float* xbar,
                          bool std_layout, hipStream_t s);
void launch_axpy(float* y, const float* x, float a, long n, hipStream_t s);
void launch_lpt_sbar(const float* xbar, const float* pbar, long n3, float cx1, float cp1, float cx2, float cp2,
                     float* const* s1, float* const* s2, hipStream_t s);
void launch_lpt_phibar(float* const* phi6, const float* d2b, long n3, hipStream_t s);
int power_max_bins();
long power_partial_doubles(int n_bins);
void launch_power(const PowerArgs& a, double* out3, hipStream_t s);

}  // namespace pmk
