// Hand-written batched 3D real FFT for gfx950 (CDNA4).
//
// The PM force of section 2 of the paper takes one forward real-to-complex 3D
// transform and three inverse transforms per step (section 3), each built
// from 1D transforms along the three axes.  Here each axis is one pass
// over HBM.  Inside a pass a 1D transform of length N = R1 * R2 is done as a
// four-step decomposition:
//
//   stage A : R1-point DFTs in registers over elements n = R2*j1 + j2,
//             twiddle exp(-/+ 2 pi i j2 l1 / N), exchange through LDS;
//   stage B : R2-point DFTs in registers over j2, output k = l1 + R1*l2.
//
// Meshes use the x-blocked layout of layout.h.  The z passes take whole
// (x/8, y) rows, contiguous regions staged through LDS with 16-byte accesses,
// and use the real<->complex packing of N reals as N/2 complex values.  The
// strided passes (y, x) give each workgroup a tile of M adjacent columns; in
// the x pass eight consecutive rows share one run of memory, so a tile reads
// 512-byte runs from N/8 places instead of 64-byte runs from N places.  The
// Nyquist plane kz = N/2 lives in its own array so that all strided tiles
// are aligned.  No MFMA: the transform is bandwidth bound.
//
// The x pass can be fused with a spectral multiplication and the inverse x
// transform of each output (the Green's-function/gradient kernel of the
// force, the LPT kernels), so the spectrum is read once per basis power of
// the gradient symbol and the product spectra are never written.
#include "pm_internal.h"

namespace pmk {
namespace {

constexpr int kThreads = 256;

// ---- complex helpers ------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// non-temporal load of one complex value (the line is marked to leave L2
// first)
__device__ __forceinline__ float2 ldnt(const float2* p) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
  return make_float2(v.x, v.y);
}
// multiply by DIR * i  (DIR = -1: -i, DIR = +1: +i)
template <int DIR>
__device__ __forceinline__ float2 cmul_i(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// exp(DIR * 2 pi i idx / 32) applied to a; idx is a compile-time constant
// after unrolling, so the branches fold.
template <int DIR>
__device__ __forceinline__ float2 twiddle32(float2 a, int idx) {
  constexpr float c32[32] = {
      1.000000000e+00f, 9.807852804e-01f, 9.238795325e-01f, 8.314696123e-01f,
      7.071067812e-01f, 5.555702330e-01f, 3.826834324e-01f, 1.950903220e-01f,
      0.0f, -1.950903220e-01f, -3.826834324e-01f, -5.555702330e-01f,
      -7.071067812e-01f, -8.314696123e-01f, -9.238795325e-01f, -9.807852804e-01f,
      -1.000000000e+00f, -9.807852804e-01f, -9.238795325e-01f, -8.314696123e-01f,
      -7.071067812e-01f, -5.555702330e-01f, -3.826834324e-01f, -1.950903220e-01f,
      0.0f, 1.950903220e-01f, 3.826834324e-01f, 5.555702330e-01f,
      7.071067812e-01f, 8.314696123e-01f, 9.238795325e-01f, 9.807852804e-01f};
  if (idx == 0) return a;
  if (idx == 8) return cmul_i<DIR>(a);
  if (idx == 16) return make_float2(-a.x, -a.y);
  if (idx == 24) return cmul_i<-DIR>(a);
  const float c = c32[idx & 31];
  const float s = (DIR < 0 ? -1.f : 1.f) * c32[(idx + 24) & 31];   // sin(2 pi idx/32)
  return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
}

template <int R>
__host__ __device__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// In-register DFT of R = 1..32 points (power of two), natural order in and
// out: radix-2 decimation in frequency followed by a bit-reversal that the
// compiler resolves into register renaming.
template <int R, int DIR>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
  if constexpr (R > 1) {
#pragma unroll
    for (int len = R; len >= 2; len >>= 1) {
      const int half = len >> 1;
#pragma unroll
      for (int s = 0; s < R; s += len) {
#pragma unroll
        for (int k = 0; k < half; ++k) {
          const float2 a = v[s + k], b = v[s + k + half];
          v[s + k] = cadd(a, b);
          v[s + k + half] = twiddle32<DIR>(csub(a, b), k * (32 / len));
        }
      }
    }
    float2 t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) t[i] = v[bitrev<R>(i)];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = t[i];
  }
}

template <int N> struct Split;
template <> struct Split<4> { static constexpr int R1 = 4, R2 = 1; };
template <> struct Split<8> { static constexpr int R1 = 8, R2 = 1; };
template <> struct Split<16> { static constexpr int R1 = 16, R2 = 1; };
template <> struct Split<32> { static constexpr int R1 = 32, R2 = 1; };
template <> struct Split<64> { static constexpr int R1 = 8, R2 = 8; };
template <> struct Split<128> { static constexpr int R1 = 16, R2 = 8; };
template <> struct Split<256> { static constexpr int R1 = 16, R2 = 16; };
template <> struct Split<512> { static constexpr int R1 = 32, R2 = 16; };
template <> struct Split<1024> { static constexpr int R1 = 32, R2 = 32; };

// Columns per workgroup tile of the strided passes.
template <int N> struct Cols { static constexpr int M = N >= 1024 ? 8 : 16; };

// Tile of a y pass (columns of 8-byte values, rows 4N values apart): 16
// columns fill each row's 128-byte line, so that no line is written half by
// one workgroup and half by another.  At N = 1024 such a tile's exchange
// takes 135 KB of LDS, one workgroup per CU, and runs on 512 threads so that
// each thread keeps the work of the 8-column tile on 256 threads.
template <int N> struct YTile {
  static constexpr int M = 16;
  static constexpr int TH = (N >= 1024) ? 512 : kThreads;
};

// twiddle exp(DIR 2 pi i e / N) from the table of exp(-2 pi i k / N)
template <int DIR>
__device__ __forceinline__ float2 tw_get(const float2* __restrict__ tw, int e) {
  const float2 w = tw[e];
  return DIR < 0 ? w : cconj(w);
}

// blockIdx -> tile index so that consecutive tiles of one launch land on the
// same XCD (workgroups are dispatched round-robin over the 8 XCDs, each with
// its own L2): neighbouring column tiles share cache lines.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, slot = b >> 3;
  return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// Tile -> (batch b, first column c0) of a column pass with nbat batches of
// ntc column tiles.  The y pass walks columns fastest: neighbouring tiles
// share 128-byte lines.  The x passes walk batches (ky rows) fastest: the
// workgroups in flight then spread over many rows of every x block instead
// of a few (measured 10% faster at 1024^3); the force x pass takes its main
// array in blocks of 8 ky rows instead, eight column tiles of each in flight
// together (1.5% faster again).
template <bool BATCH_FAST>
__device__ __forceinline__ void tile_bc(int tile, int nbat, int ntc, int M, int& b, int& c0) {
  if (BATCH_FAST) {
    b = tile % nbat;
    c0 = (tile / nbat) * M;
  } else {
    b = tile / ntc;
    c0 = (tile - b * ntc) * M;
  }
}

// ===========================================================================
// Strided (column-tile) pass: element (batch b, row n, column c) at
//   data + b*sb + row(n) + c*CS,  n in [0, N), c in [0, ncols)
// with row(n) = n*sn for the y pass (CS = 1) and, for the x pass over the
// x-blocked layout, row(n) = (n/8)*sn + n%8 (CS = 8): eight rows share one
// 64-byte run per column.
// ===========================================================================
struct ColGeom {
  long sb, sn;
  int ncols, ntc;   // columns, column tiles per batch
};

template <bool BLK>
__device__ __forceinline__ long row_off(int n, long sn) {
  return BLK ? (long)(n >> 3) * sn + (n & 7) : (long)n * sn;
}

template <int N, int M>
struct ColLds {
  static constexpr int R1 = Split<N>::R1, R2 = Split<N>::R2;
  // forward exchange [l1][j2][m] with a padded l1 stride; the inverse
  // exchange of the fused pass uses [l1'][l1][m] (R2 x R1)
  static constexpr int SA = R2 * M + M;
  static constexpr int SB = R1 * M + M;
  static constexpr int size = (R2 > 1) ? (R1 * SA > R2 * SB ? R1 * SA : R2 * SB) : 1;
};

// One launch covers the main arrays (tiles [0, nb_main)) and the Nyquist
// planes (the remaining tiles) of up to three fields (blockIdx.y).
struct ColPass {
  float2* main[3];
  float2* plane[3];
  ColGeom gm, gp;
  int nb_main;
  int ntiles;   // main + plane tiles per field
  BatchArg bat; // batched launches: blockIdx.z selects the member
};

template <int N, int M, int DIR, bool BLK, int TH = kThreads>
__global__ __launch_bounds__(TH) void k_fft_cols(ColPass p, const float2* __restrict__ tw) {
  constexpr int R1 = Split<N>::R1, R2 = Split<N>::R2;
  constexpr int CS = BLK ? 8 : 1;
  constexpr int IA = (M * R2 + TH - 1) / TH;
  constexpr int IB = (M * R1 + TH - 1) / TH;
  __shared__ float2 lds[ColLds<N, M>::size];
  int tile = xcd_tile(blockIdx.x, gridDim.x);
  const bool is_plane = tile >= p.nb_main;
  if (is_plane) tile -= p.nb_main;
  const ColGeom& g = is_plane ? p.gp : p.gm;
  const long bo = batch_bytes(p.bat);
  if (bo < 0) return;
  float2* data = byte_adv(is_plane ? p.plane[blockIdx.y] : p.main[blockIdx.y], bo);
  int b, c0;
  tile_bc<BLK>(tile, is_plane ? ((int)gridDim.x - p.nb_main) / g.ntc : p.nb_main / g.ntc, g.ntc, M, b, c0);
  float2* base = data + b * g.sb + (long)c0 * CS;
  const int tid = threadIdx.x;

  if constexpr (R2 == 1) {
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int it = tid + i * TH;
      const int m = it % M;
      if (it < M && c0 + m < g.ncols) {
        float2 v[R1];
#pragma unroll
        for (int j = 0; j < R1; ++j) v[j] = base[row_off<BLK>(j, g.sn) + m * CS];
        dft<R1, DIR>(v);
#pragma unroll
        for (int j = 0; j < R1; ++j) base[row_off<BLK>(j, g.sn) + m * CS] = v[j];
      }
    }
  } else {
    constexpr int SA = ColLds<N, M>::SA;
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int it = tid + i * TH;
      if (it < M * R2) {
        const int m = it % M, j2 = it / M;
        const bool ok = c0 + m < g.ncols;
        float2 v[R1];
#pragma unroll
        for (int j1 = 0; j1 < R1; ++j1)
          v[j1] = ok ? base[row_off<BLK>(R2 * j1 + j2, g.sn) + m * CS] : make_float2(0.f, 0.f);
        dft<R1, DIR>(v);
#pragma unroll
        for (int l1 = 0; l1 < R1; ++l1) lds[l1 * SA + j2 * M + m] = l1 == 0 ? v[l1] : cmul(v[l1], tw_get<DIR>(tw, j2 * l1));
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      const int it = tid + i * TH;
      if (it < M * R1) {
        const int m = it % M, l1 = it / M;
        float2 v[R2];
#pragma unroll
        for (int j2 = 0; j2 < R2; ++j2) v[j2] = lds[l1 * SA + j2 * M + m];
        dft<R2, DIR>(v);
        if (c0 + m < g.ncols) {
#pragma unroll
          for (int l2 = 0; l2 < R2; ++l2) base[row_off<BLK>(l1 + R1 * l2, g.sn) + m * CS] = v[l2];
        }
      }
    }
  }
}

// Inverse y pass of the force meshes after an OP_FORCE_XS x pass
// (blockIdx.y = 0: F_x in place; 1: the shared factor i g X).  A shared-
// factor tile is loaded once and transformed twice from registers: first
// times D(w_y), which varies along y and so must come before the
// transform, stored to F_y; then plain, in place, its output times D(w_z),
// constant along a column, as F_z.  The stage-A twiddles come from an
// R1 x R2 table in LDS, filled with the first loads, so that the second
// transform's stage A issues no global load behind the first one's stores.
// p.main/p.plane hold F_x, the shared factor (F_z) and F_y, in that order.
template <int N, int M, int TH>
__global__ __launch_bounds__(TH) void k_fft_cols_force(ColPass p, const float2* __restrict__ tw,
                                                             const float* __restrict__ dy_tab,
                                                             const float* __restrict__ dz_tab) {
  constexpr int R1 = Split<N>::R1, R2 = Split<N>::R2;
  static_assert(R2 > 1, "columns split over two stages");
  constexpr int IA = (M * R2 + TH - 1) / TH;
  constexpr int IB = (M * R1 + TH - 1) / TH;
  constexpr int SA = ColLds<N, M>::SA;
  constexpr int IT = (R1 * R2 + TH - 1) / TH;
  __shared__ float2 lds[ColLds<N, M>::size];
  __shared__ float2 tws[R1 * R2];   // exp(+2 pi i j l / N), j < R2, l < R1
  int tile = xcd_tile(blockIdx.x, gridDim.x);
  const bool is_plane = tile >= p.nb_main;
  if (is_plane) tile -= p.nb_main;
  const ColGeom& g = is_plane ? p.gp : p.gm;
  const bool shared = blockIdx.y == 1;   // uniform
  const int b = tile / g.ntc;
  const int c0 = (tile - b * g.ntc) * M;
  const long bo = batch_bytes(p.bat);
  if (bo < 0) return;
  const long off = b * g.sb + c0 + bo / (long)sizeof(float2);
  float2* base = (is_plane ? p.plane[blockIdx.y] : p.main[blockIdx.y]) + off;
  const int tid = threadIdx.x;

  // every global load of stage A first: the twiddle table, the row factors
  // D(w_y) of a shared tile and the columns
  float2 twv[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int e = tid + k * TH;
    if (e < R1 * R2) twv[k] = tw_get<1>(tw, (e / R1) * (e % R1));
  }
  float2 v0[IA][R1];
  float d[IA][R1];
#pragma unroll
  for (int i = 0; i < IA; ++i) {
    const int it = tid + i * TH;
    const int m = it % M, j2 = it / M;
    const bool ok = it < M * R2 && c0 + m < g.ncols;
    if (shared) {
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1) d[i][j1] = it < M * R2 ? dy_tab[R2 * j1 + j2] : 0.f;
    }
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) v0[i][j1] = ok ? base[(long)(R2 * j1 + j2) * g.sn + m] : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int e = tid + k * TH;
    if (e < R1 * R2) tws[e] = twv[k];
  }
  __syncthreads();

  // stage A: the loaded columns (times D(w_y) of the row when row_factor),
  // R1-point transforms, twiddles, into the exchange
  auto stage_a = [&](bool row_factor) {
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int it = tid + i * TH;
      if (it < M * R2) {
        const int m = it % M, j2 = it / M;
        float2 v[R1];
#pragma unroll
        for (int j1 = 0; j1 < R1; ++j1) v[j1] = row_factor ? cscale(v0[i][j1], d[i][j1]) : v0[i][j1];
        dft<R1, 1>(v);
#pragma unroll
        for (int l1 = 0; l1 < R1; ++l1) lds[l1 * SA + j2 * M + m] = l1 == 0 ? v[l1] : cmul(v[l1], tws[j2 * R1 + l1]);
      }
    }
  };
  // stage B: R2-point transforms out of the exchange, stored through dst
  // times D(w_z) of the column when col_factor
  auto stage_b = [&](float2* dst, bool col_factor) {
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      const int it = tid + i * TH;
      if (it < M * R1) {
        const int m = it % M, l1 = it / M;
        const bool ok = c0 + m < g.ncols;
        // kz = c / 8 in the main array, N/2 on the Nyquist plane
        const float cf = col_factor && ok ? dz_tab[is_plane ? N / 2 : (c0 + m) >> 3] : 1.f;
        float2 v[R2];
#pragma unroll
        for (int j2 = 0; j2 < R2; ++j2) v[j2] = lds[l1 * SA + j2 * M + m];
        dft<R2, 1>(v);
        if (ok) {
#pragma unroll
          for (int l2 = 0; l2 < R2; ++l2) dst[(long)(l1 + R1 * l2) * g.sn + m] = cscale(v[l2], cf);
        }
      }
    }
  };

  if (shared) {
    stage_a(true);
    __syncthreads();
    stage_b((is_plane ? p.plane[2] : p.main[2]) + off, false);
    __syncthreads();   // the exchange buffer is reused
  }
  stage_a(false);
  __syncthreads();
  stage_b(base, shared);
}

// ===========================================================================
// Contiguous z passes over the x-blocked layout.  A workgroup takes L lines
// l0 .. l0+L-1 (L a multiple of 8): L/8 whole (x/8, y) rows, one contiguous
// region of L*N floats = L*N/2 complex values, which holds the block's real
// input and, after the pass, its spectrum (in place).  Line m of the block
// (xi = m % 8, row rr = m / 8) has its real z at region float
// rr*8N + z*8 + xi; the packed complex value j = (x[2j], x[2j+1]) is the
// float pair (rr*8N + 16j + xi, +8); spectrum kz is region complex
// rr*4N + kz*8 + xi.  The region is staged through LDS with 16-byte loads
// and stores, so global traffic is fully coalesced.
// ===========================================================================
// Geometry of a workgroup of LINES lines of length N (H = N/2 complex).
template <int N, int LINES>
struct ZGeomL {
  static constexpr int NN = N;
  static constexpr int H = N / 2;
  static constexpr int R1 = Split<H>::R1, R2 = Split<H>::R2;
  static constexpr int L = LINES;
  static constexpr int LP = L + 1;                          // padded line stride of the exchange
  // padded natural-order Z: a row stride of 4 (mod 32) float2 puts lanes
  // that run over the line index on different banks (<= 2-way conflicts)
  static constexpr int ZP = H >= 32 ? H + 4 : H + 1;
  static constexpr int XS = (R2 > 1) ? H * LP : 1;          // exchange [l1][j2][m]
  static constexpr int ZS = L * ZP;                         // natural-order Z[m][k]
  static constexpr int RS = L * H;                          // staged region (complex)
  static constexpr int size = (XS > ZS ? XS : ZS) > RS ? (XS > ZS ? XS : ZS) : RS;
  static_assert(L % 8 == 0, "whole (x/8, y) rows per workgroup");
};

// the in-place passes take 8192 / H lines (64 KB of data) per workgroup
template <int N>
using ZGeom = ZGeomL<N, (8192 / (N / 2) < N * N ? 8192 / (N / 2) : N * N)>;

// copy N16 16-byte words from global memory to LDS (whole workgroup): every
// load of a thread is issued before its first LDS store, so the loads are in
// flight together instead of one round trip per word
// NT: non-temporal loads (the lines are marked to leave L2 first), for
// passes whose output, not their input, benefits from staying in L2.
template <int N16, bool NT = false>
__device__ __forceinline__ void copy16(float4* __restrict__ dst, const float4* __restrict__ src) {
  if constexpr (N16 % kThreads == 0) {
    constexpr int K = N16 / kThreads;
    float4 t[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if constexpr (NT) {
        typedef float f4v __attribute__((ext_vector_type(4)));
        const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(src) + threadIdx.x + k * kThreads);
        t[k] = make_float4(v.x, v.y, v.z, v.w);
      } else {
        t[k] = src[threadIdx.x + k * kThreads];
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) dst[threadIdx.x + k * kThreads] = t[k];
  } else {   // small meshes: fewer words than threads
    for (int i = threadIdx.x; i < N16; i += kThreads) dst[i] = src[i];
  }
}

// Length-H complex transform of the L lines of a workgroup.  load(m, n)
// returns element n of line m (it may read the staged region in lds: every
// load happens before the first write to lds).  On return Z[m][k] is in lds
// at m*ZP + k (natural order).  Items map with the line m fastest so that
// LDS accesses of a wave spread over the banks.
template <class G, int DIR, class Load>
__device__ __forceinline__ void zline_transform(float2* lds, const float2* __restrict__ twh, Load load) {
  constexpr int R1 = G::R1, R2 = G::R2, L = G::L, LP = G::LP, ZP = G::ZP;
  const int tid = threadIdx.x;
  if constexpr (R2 == 1) {
    constexpr int IA = (L + kThreads - 1) / kThreads;
    float2 v[IA][R1];
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int m = tid + i * kThreads;
      if (m < L) {
#pragma unroll
        for (int j = 0; j < R1; ++j) v[i][j] = load(m, j);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int m = tid + i * kThreads;
      if (m < L) {
        dft<R1, DIR>(v[i]);
#pragma unroll
        for (int j = 0; j < R1; ++j) lds[m * ZP + j] = v[i][j];
      }
    }
  } else {
    constexpr int IA = (L * R2 + kThreads - 1) / kThreads;
    constexpr int IB = (L * R1 + kThreads - 1) / kThreads;
    float2 v[IA][R1];
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int it = tid + i * kThreads;
      if (it < L * R2) {
        const int m = it % L, j2 = it / L;
#pragma unroll
        for (int j1 = 0; j1 < R1; ++j1) v[i][j1] = load(m, R2 * j1 + j2);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int it = tid + i * kThreads;
      if (it < L * R2) {
        const int m = it % L, j2 = it / L;
        dft<R1, DIR>(v[i]);
#pragma unroll
        for (int l1 = 0; l1 < R1; ++l1)
          lds[(l1 * R2 + j2) * LP + m] = l1 == 0 ? v[i][l1] : cmul(v[i][l1], tw_get<DIR>(twh, j2 * l1));
      }
    }
    __syncthreads();
    float2 w[IB][R2];
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      const int it = tid + i * kThreads;
      if (it < L * R1) {
        const int m = it % L, l1 = it / L;
#pragma unroll
        for (int j2 = 0; j2 < R2; ++j2) w[i][j2] = lds[(l1 * R2 + j2) * LP + m];
        dft<R2, DIR>(w[i]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      const int it = tid + i * kThreads;
      if (it < L * R1) {
        const int m = it % L, l1 = it / L;
#pragma unroll
        for (int l2 = 0; l2 < R2; ++l2) lds[m * ZP + l1 + R1 * l2] = w[i][l2];
      }
    }
  }
  __syncthreads();
}

// Real-to-complex along z, in place: the N reals of each line become
// X[0..N/2-1] (region) and X[N/2] (Nyquist plane, q[l]).
template <int N>
__global__ __launch_bounds__(kThreads) void k_r2c_z(float* __restrict__ r0, float* __restrict__ r1,
                                                     float* __restrict__ r2, float2* __restrict__ q0,
                                                     float2* __restrict__ q1, float2* __restrict__ q2,
                                                     const float2* __restrict__ twh,
                                                     const float2* __restrict__ twn, BatchArg bat) {
  using G = ZGeom<N>;
  constexpr int H = G::H, L = G::L, ZP = G::ZP;
  __shared__ float2 lds[G::size];
  const long bo = batch_bytes(bat);
  if (bo < 0) return;
  float* r = byte_adv(blockIdx.y == 0 ? r0 : (blockIdx.y == 1 ? r1 : r2), bo);
  float2* q = byte_adv(blockIdx.y == 0 ? q0 : (blockIdx.y == 1 ? q1 : q2), bo);
  const long l0 = (long)xcd_tile(blockIdx.x, gridDim.x) * L;
  float2* reg = reinterpret_cast<float2*>(r) + l0 * H;   // region: L*H complex = L*N floats
  copy16<L * H / 2>(reinterpret_cast<float4*>(lds), reinterpret_cast<const float4*>(reg));
  __syncthreads();
  const float* lf = reinterpret_cast<const float*>(lds);
  zline_transform<G, -1>(lds, twh, [&](int m, int n) {
    const int o = (m >> 3) * 8 * N + 16 * n + (m & 7);
    return make_float2(lf[o], lf[o + 8]);
  });
  // post-processing: X[k] = E + w^k O, X[H-k] = conj(E - w^k O); line m fastest
  constexpr int NK = H / 2 + 1;
  for (int it = threadIdx.x; it < L * NK; it += kThreads) {
    const int m = it % L, k = it / L;
    const float2 zk = lds[m * ZP + k];
    const float2 zm = cconj(lds[m * ZP + ((H - k) & (H - 1))]);
    const float2 e = cscale(cadd(zk, zm), 0.5f);
    const float2 dif = csub(zk, zm);
    const float2 o = make_float2(0.5f * dif.y, -0.5f * dif.x);   // (zk - zm) / (2i)
    const float2 t = cmul(o, twn[k]);
    float2* out = reg + (m >> 3) * 4 * N + (m & 7);
    if (k == 0) {
      out[0] = make_float2(e.x + t.x, 0.f);
      q[l0 + m] = make_float2(e.x - t.x, 0.f);
    } else {
      out[8 * k] = cadd(e, t);
      if (k != H - k) out[8 * (H - k)] = cconj(csub(e, t));
    }
  }
}

// Complex-to-real along z (unnormalised), in place: X[0..N/2] -> N reals.
// The imaginary parts of X[0] and X[N/2] are discarded.
template <int N>
__global__ __launch_bounds__(kThreads) void k_c2r_z(float* __restrict__ r0, float* __restrict__ r1,
                                                     float* __restrict__ r2, const float2* __restrict__ q0,
                                                     const float2* __restrict__ q1, const float2* __restrict__ q2,
                                                     const float2* __restrict__ twh,
                                                     const float2* __restrict__ twn) {
  using G = ZGeom<N>;
  constexpr int H = G::H, L = G::L, ZP = G::ZP;
  __shared__ float2 lds[G::size];
  float* r = blockIdx.y == 0 ? r0 : (blockIdx.y == 1 ? r1 : r2);
  const float2* q = blockIdx.y == 0 ? q0 : (blockIdx.y == 1 ? q1 : q2);
  const long l0 = (long)xcd_tile(blockIdx.x, gridDim.x) * L;
  float2* reg = reinterpret_cast<float2*>(r) + l0 * H;
  copy16<L * H / 2>(reinterpret_cast<float4*>(lds), reinterpret_cast<const float4*>(reg));
  __syncthreads();
  zline_transform<G, +1>(lds, twh, [&](int m, int k) {
    const float2* line = lds + (m >> 3) * 4 * N + (m & 7);
    float2 a, b;
    if (k == 0) {
      a = make_float2(line[0].x, 0.f);
      b = make_float2(q[l0 + m].x, 0.f);
    } else {
      a = line[8 * k];
      b = cconj(line[8 * (H - k)]);
    }
    const float2 e = cadd(a, b);
    const float2 o = cmulc(csub(a, b), twn[k]);     // (a - b) exp(+2 pi i k / N)
    return make_float2(e.x - o.y, e.y + o.x);       // e + i o
  });
  // region float e = rr*8N + z*8 + xi holds component z&1 of Z[rr*8 + xi][z/2]
  const float* lf = reinterpret_cast<const float*>(lds);
  float4* o4 = reinterpret_cast<float4*>(reg);
  for (int i = threadIdx.x; i < L * N / 4; i += kThreads) {
    const int e = 4 * i;
    const int xi = e & 7, z = (e >> 3) & (N - 1), rr = e / (8 * N);
    const int zo = 2 * (z >> 1) + (z & 1);
    const float* zl = lf + 2 * ((rr * 8 + xi) * ZP) + zo;
    o4[i] = make_float4(zl[0], zl[2 * ZP], zl[4 * ZP], zl[6 * ZP]);
  }
}

// Complex-to-real along z of three fields (the force components) written as
// one interleaved real mesh in the x-blocked order
//   out[x/8][y][z][x%8][3],  element ((l/8 * N + z) * 8 + x%8) * 3 + field,
// the layout the particle readout gathers from: the 3 components of a cell
// are one 12-byte load, and x, x+1 of one block are adjacent.  A workgroup
// transforms one field of one (x/8, y) row (8 lines) through LDS and stores
// its component; the three workgroups of a row have consecutive tile indices,
// which the XCD-aware mapping places on one XCD, so their stores into each
// 192-byte run of the output merge in that XCD's L2.
template <int N>
using Z3Geom = ZGeomL<N, 8>;

template <int N>
__global__ __launch_bounds__(kThreads) void k_c2r_z3(const float* __restrict__ r0, long fstride,
                                                      const float2* __restrict__ q0, long qstride,
                                                      float* __restrict__ out, const float2* __restrict__ twh,
                                                      const float2* __restrict__ twn, BatchArg bat) {
  using G = Z3Geom<N>;
  constexpr int H = G::H, L = G::L, ZP = G::ZP;
  __shared__ float2 lds[G::size];
  {
    const long bo = batch_bytes(bat);
    if (bo < 0) return;
    r0 = byte_adv(r0, bo);
    q0 = byte_adv(q0, bo);
    out = byte_adv(out, bo);
  }
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int row = tile / 3, f = tile - 3 * row;
  const long l0 = (long)row * L;
  // field f by stride arithmetic (a choice among pointer arguments can
  // compile to a lookup table in private memory)
  const float2* reg = reinterpret_cast<const float2*>(r0 + f * fstride) + l0 * H;
  const float2* q = q0 + f * qstride;
  // non-temporal: each 96-byte output run is filled by three workgroups, and
  // their partial writes merge in L2 only while the output lines stay there
  copy16<L * H / 2, true>(reinterpret_cast<float4*>(lds), reinterpret_cast<const float4*>(reg));
  __syncthreads();
  zline_transform<G, +1>(lds, twh, [&](int m, int k) {
    const float2* line = lds + m;   // one row: line m is xi = m
    float2 a, b;
    if (k == 0) {
      a = make_float2(line[0].x, 0.f);
      b = make_float2(q[l0 + m].x, 0.f);
    } else {
      a = line[8 * k];
      b = cconj(line[8 * (H - k)]);
    }
    const float2 e = cadd(a, b);
    const float2 o2 = cmulc(csub(a, b), twn[k]);    // (a - b) exp(+2 pi i k / N)
    return make_float2(e.x - o2.y, e.y + o2.x);     // e + i o
  });
  // Z[m][j] = (x[2j], x[2j+1]) of line m: cells z = 2j, 2j+1 of xi = m
  float* o = out + (long)row * N * 24 + f;
  for (int idx = threadIdx.x; idx < L * H; idx += kThreads) {
    const int m = idx & 7, j = idx >> 3;
    const float2 v = lds[m * ZP + j];
    o[((2 * j) * 8 + m) * 3] = v.x;
    o[((2 * j + 1) * 8 + m) * 3] = v.y;
  }
}

// ===========================================================================
// Fused x pass: forward x transform, spectral op, inverse x transform(s).
// Geometry as in k_fft_cols with rows n = kx.  mode 0: the main array
// (b = ky, c = kz < N/2); mode 1: the Nyquist plane (b = 0, c = ky, kz = N/2).
// ===========================================================================
struct FusedArgs {
  SpecOp op;
  ColGeom gm, gp;          // main array (mode 0) and Nyquist plane (mode 1)
  int nb_main;
  int pbasis;              // the power of D(w_x) this launch handles (N > 32)
  int first, last;         // fan-in: first / last basis launch of the op
  float2* park_main;       // fan-in: x-spectrum partial sum between launches
  float2* park_nyq;
  const float2* in_main;   // input spectrum (forward-y transformed)
  const float2* in_nyq;
  FftTables t;
  BatchArg bat;            // batched launches (k_fft_x_force): blockIdx.z selects the member
};

template <int N>
__device__ __forceinline__ int sfreq(int n) { return n < N / 2 ? n : n - N; }

// The spectral multiplier of every op factorises into
//   c(k) * D(w_x)^p * coef(column),
// a real common factor c(k) (Green's function, deconvolution, split filter,
// P(k) scaling), a power p in {0, 1, 2} of the FD gradient symbol along the
// transform axis x, and a complex coefficient that is constant along x
// (built from D(w_y), D(w_z) and +-i).  Because that coefficient commutes
// with the x transform, a fan-out op needs one inverse x transform per
// distinct power p (force: 2, LPT: 3) and every output is a scaled copy of
// one of them; a fan-in op (a transpose) combines its inputs of equal power
// before one forward x transform each.
struct Term {
  int p;       // power of D(w_x)
  int sel;     // 0: 1, 1: D_y, 2: D_z, 3: D_y^2, 4: D_z^2, 5: D_y D_z
  int phase;   // 0: 1, 1: +i, 2: -i
};

__host__ __device__ __forceinline__ Term op_term(int kind, int o) {
  // component order of the LPT outputs: s1 x, y, z, phi xx, yy, zz, xy, xz, yz
  constexpr int lp[9] = {1, 0, 0, 2, 0, 0, 1, 1, 0};
  constexpr int ls[9] = {0, 1, 2, 0, 3, 4, 1, 2, 5};
  switch (kind) {
    case OP_FORCE: return Term{o == 0 ? 1 : 0, o, 1};
    case OP_FORCE_XS: return Term{o == 0 ? 1 : 0, 0, 1};
    case OP_FORCE_T: return Term{o == 0 ? 1 : 0, o, 2};
    case OP_LPT2: return Term{o == 0 ? 1 : 0, o, 2};
    case OP_LPT2_T: return Term{o == 0 ? 1 : 0, o, 1};
    case OP_LPT1: return Term{lp[o], ls[o], o < 3 ? 1 : 0};
    case OP_LPT1_T: return Term{lp[o], ls[o], o < 3 ? 2 : 0};
    case OP_LPT_PHI: return Term{lp[o + 3], ls[o + 3], 0};
    default: return Term{0, 0, 0};   // IDENTITY, LINEAR
  }
}

__device__ __forceinline__ float2 coef_of(const Term& tm, float dy, float dz) {
  float v;
  switch (tm.sel) {
    case 0: v = 1.f; break;
    case 1: v = dy; break;
    case 2: v = dz; break;
    case 3: v = dy * dy; break;
    case 4: v = dz * dz; break;
    default: v = dy * dz; break;
  }
  return tm.phase == 0 ? make_float2(v, 0.f) : (tm.phase == 1 ? make_float2(0.f, v) : make_float2(0.f, -v));
}

template <int N>
__device__ __forceinline__ float common_factor(const SpecOp& op, const FftTables& t, int kx, int ky, int kz) {
  const float kk = t.kxy[kx] + t.kxy[ky] + t.kz[kz];
  const float inv = kk > 0.f ? __builtin_amdgcn_rcpf(kk) : 0.f;   // <= 1 ulp
  auto pk = [&]() {
    const int fx = sfreq<N>(kx), fy = sfreq<N>(ky);
    return op.pk[fx * fx + fy * fy + kz * kz];
  };
  switch (op.kind) {
    case OP_IDENTITY:
      return op.scale;
    case OP_LINEAR:
      return pk();
    case OP_FORCE:
    case OP_FORCE_XS:
    case OP_FORCE_T: {
      float g = op.scale * inv;
      if (op.deconv) {
        const float w = t.wxy[kx] * t.wxy[ky] * t.wz[kz];
        g *= __builtin_amdgcn_rcpf(op.deconv == 1 ? w : w * w);
      }
      if (op.split) {
        const float sv = t.sxy[kx] * t.sxy[ky] * t.sz[kz];
        g *= (op.split == 1 ? sv : 1.f - sv);
      }
      return g;
    }
    case OP_LPT1:
    case OP_LPT_PHI:
    case OP_LPT1_T:
      return pk() * inv;
    case OP_LPT2:
    case OP_LPT2_T:
      return op.scale * inv;
    default:
      return 0.f;
  }
}

__device__ __forceinline__ float powp(float d, int p) { return p == 0 ? 1.f : (p == 1 ? d : d * d); }

template <int N, int M, bool FANIN>
__global__ __launch_bounds__(kThreads) void k_fft_x_fused(FusedArgs a) {
  constexpr int R1 = Split<N>::R1, R2 = Split<N>::R2;
  constexpr int IA = (M * R2 + kThreads - 1) / kThreads;   // stage A and inverse stage B'
  constexpr int IB = (M * R1 + kThreads - 1) / kThreads;   // stage B and inverse stage A'
  constexpr int SA = ColLds<N, M>::SA, SB = ColLds<N, M>::SB;
  __shared__ float2 lds[ColLds<N, M>::size];
  int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int mode = tile >= a.nb_main ? 1 : 0;
  if (mode) tile -= a.nb_main;
  const ColGeom& g = mode ? a.gp : a.gm;
  int b, c0;
  tile_bc<true>(tile, mode ? ((int)gridDim.x - a.nb_main) / g.ntc : a.nb_main / g.ntc, g.ntc, M, b, c0);
  const long off = b * g.sb + (long)c0 * 8;
  const int tid = threadIdx.x;
  const SpecOp& op = a.op;
  const FftTables& t = a.t;
  const int kind = op.kind;
  const int nterm = FANIN ? op.n_in : op.n_out;
  int pmask = 0;
  if (FANIN)
    for (int o = 0; o < nterm; ++o) pmask |= 1 << op_term(kind, o).p;
  auto src_of = [&](int in) -> const float2* {
    if (FANIN) return (mode == 0 ? op.in_c[in] : op.in_q[in]) + off;
    return (mode == 0 ? a.in_main : a.in_nyq) + off;
  };
  auto dst_of = [&](int o) -> float2* { return (mode == 0 ? op.out_c[o] : op.out_q[o]) + off; };
  // (ky, kz) of column m; masked columns map to the zero mode
  auto freq = [&](int m, int& ky, int& kz) {
    if (c0 + m >= g.ncols) { ky = 0; kz = 0; }
    else if (mode == 0) { ky = b; kz = c0 + m; }
    else { ky = c0 + m; kz = N / 2; }
  };
  auto col_d = [&](int m, float& dy, float& dz) {
    int ky, kz;
    freq(m, ky, kz);
    dy = t.dxy[ky];
    dz = t.dz[kz];
  };

  if constexpr (R2 == 1) {
    // N <= 32: a whole column fits in one thread's registers
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int m = tid + i * kThreads;
      if (m < M && c0 + m < g.ncols) {
        int ky, kz;
        freq(m, ky, kz);
        float dy, dz;
        col_d(m, dy, dz);
        float2 X[R1], Y[R1];
#pragma unroll
        for (int j = 0; j < R1; ++j) Y[j] = make_float2(0.f, 0.f);
        if (FANIN) {
          for (int p = 0; p < 3; ++p) {
            if (!(pmask >> p & 1)) continue;
#pragma unroll
            for (int j = 0; j < R1; ++j) X[j] = make_float2(0.f, 0.f);
            for (int in = 0; in < nterm; ++in) {
              const Term tm = op_term(kind, in);
              if (tm.p != p) continue;
              const float2 cf = coef_of(tm, dy, dz);
              const float2* src = src_of(in);
#pragma unroll
              for (int j = 0; j < R1; ++j) X[j] = cadd(X[j], cmul(src[row_off<true>(j, g.sn) + m * 8], cf));
            }
            dft<R1, -1>(X);
#pragma unroll
            for (int kx = 0; kx < R1; ++kx) Y[kx] = cadd(Y[kx], cscale(X[kx], powp(t.dxy[kx], p)));
          }
#pragma unroll
          for (int kx = 0; kx < R1; ++kx) Y[kx] = cscale(Y[kx], common_factor<N>(op, t, kx, ky, kz));
          dft<R1, 1>(Y);
          float2* dst = dst_of(0);
#pragma unroll
          for (int j = 0; j < R1; ++j) dst[row_off<true>(j, g.sn) + m * 8] = Y[j];
        } else {
          const float2* src = src_of(0);
#pragma unroll
          for (int j = 0; j < R1; ++j) X[j] = src[row_off<true>(j, g.sn) + m * 8];
          dft<R1, -1>(X);
#pragma unroll
          for (int kx = 0; kx < R1; ++kx) X[kx] = cscale(X[kx], common_factor<N>(op, t, kx, ky, kz));
          {
            const int p = a.pbasis;
#pragma unroll
            for (int kx = 0; kx < R1; ++kx) Y[kx] = cscale(X[kx], powp(t.dxy[kx], p));
            dft<R1, 1>(Y);
            for (int o = 0; o < nterm; ++o) {
              const Term tm = op_term(kind, o);
              if (tm.p != p) continue;
              const float2 cf = coef_of(tm, dy, dz);
              float2* dst = dst_of(o);
#pragma unroll
              for (int j = 0; j < R1; ++j) dst[row_off<true>(j, g.sn) + m * 8] = cmul(Y[j], cf);
            }
          }
        }
      }
    }
    return;
  } else {
    // forward x transform of one (combined) input into X[item][l2], kx = l1 + R1*l2;
    // the multiplied spectrum Y reuses the same registers
    float2 X[IB][R2];
    float2 (&Y)[IB][R2] = X;
    auto forward = [&](int p) {
#pragma unroll
      for (int i = 0; i < IA; ++i) {
        const int it = tid + i * kThreads;
        if (it < M * R2) {
          const int m = it % M, j2 = it / M;
          const bool ok = c0 + m < g.ncols;
          float2 v[R1];
          if (FANIN) {
            float dy, dz;
            col_d(m, dy, dz);
#pragma unroll
            for (int j1 = 0; j1 < R1; ++j1) v[j1] = make_float2(0.f, 0.f);
#pragma unroll 1
            for (int in = 0; in < nterm; ++in) {
              const Term tm = op_term(kind, in);
              if (tm.p != p || !ok) continue;
              const float2 cf = coef_of(tm, dy, dz);
              const float2* src = src_of(in);
#pragma unroll
              for (int j1 = 0; j1 < R1; ++j1) v[j1] = cadd(v[j1], cmul(src[row_off<true>(R2 * j1 + j2, g.sn) + m * 8], cf));
            }
          } else {
            const float2* src = src_of(0);
#pragma unroll
            for (int j1 = 0; j1 < R1; ++j1) v[j1] = ok ? src[row_off<true>(R2 * j1 + j2, g.sn) + m * 8] : make_float2(0.f, 0.f);
          }
          dft<R1, -1>(v);
#pragma unroll
          for (int l1 = 0; l1 < R1; ++l1)
            lds[l1 * SA + j2 * M + m] = l1 == 0 ? v[l1] : cmul(v[l1], tw_get<-1>(t.tw_n, j2 * l1));
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < IB; ++i) {
        const int it = tid + i * kThreads;
        if (it < M * R1) {
          const int m = it % M, l1 = it / M;
#pragma unroll
          for (int j2 = 0; j2 < R2; ++j2) X[i][j2] = lds[l1 * SA + j2 * M + m];
          dft<R2, -1>(X[i]);
        }
      }
      __syncthreads();
    };
    // inverse x transform of Y (spectral, item layout) and store with the
    // coefficients of every output term of power p (fan-in: output 0)
    auto inverse_store = [&](int p) {
#pragma unroll
      for (int i = 0; i < IB; ++i) {
        const int it = tid + i * kThreads;
        if (it < M * R1) {
          const int m = it % M, l1 = it / M;
          dft<R2, 1>(Y[i]);   // in place: Y is rebuilt before the next use
#pragma unroll
          for (int lp = 0; lp < R2; ++lp)
            lds[lp * SB + l1 * M + m] = lp == 0 ? Y[i][lp] : cmul(Y[i][lp], tw_get<1>(t.tw_n, l1 * lp));
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < IA; ++i) {
        const int it = tid + i * kThreads;
        if (it < M * R2) {
          const int m = it % M, lp = it / M;
          float2 v[R1];
#pragma unroll
          for (int l1 = 0; l1 < R1; ++l1) v[l1] = lds[lp * SB + l1 * M + m];
          dft<R1, 1>(v);
          if (c0 + m < g.ncols) {
            if (FANIN) {
              float2* dst = dst_of(0);
#pragma unroll
              for (int l2p = 0; l2p < R1; ++l2p) dst[row_off<true>(lp + R2 * l2p, g.sn) + m * 8] = v[l2p];
            } else {
              float dy, dz;
              col_d(m, dy, dz);
#pragma unroll 1
              for (int o = 0; o < nterm; ++o) {
                const Term tm = op_term(kind, o);
                if (tm.p != p) continue;
                const float2 cf = coef_of(tm, dy, dz);
                float2* dst = dst_of(o);
#pragma unroll
                for (int l2p = 0; l2p < R1; ++l2p) dst[row_off<true>(lp + R2 * l2p, g.sn) + m * 8] = cmul(v[l2p], cf);
              }
            }
          }
        }
      }
      __syncthreads();
    };

    if (FANIN) {
      // one launch per basis power p (increasing): the inputs of power p are
      // combined and forward transformed, scaled by c(k) D(w_x)^p and added
      // to the partial sum of the earlier bases.  The partial sum is parked
      // in x-spectral order in this tile's region of an input of the first
      // basis (read by this tile before it is written); the last launch
      // inverse transforms the total into output 0.
      const int p = a.pbasis;
      forward(p);
      float2* park = (mode == 0 ? a.park_main : a.park_nyq) + off;
#pragma unroll
      for (int i = 0; i < IB; ++i) {
        const int it = tid + i * kThreads;
        if (it < M * R1) {
          const int m = it % M, l1 = it / M;
          int ky, kz;
          freq(m, ky, kz);
#pragma unroll
          for (int l2 = 0; l2 < R2; ++l2) {
            const int kx = l1 + R1 * l2;
            float2 v = cscale(X[i][l2], common_factor<N>(op, t, kx, ky, kz) * powp(t.dxy[kx], p));
            if (!a.first && c0 + m < g.ncols) v = cadd(v, park[row_off<true>(kx, g.sn) + m * 8]);
            Y[i][l2] = v;
          }
          if (!a.last && c0 + m < g.ncols) {
#pragma unroll
            for (int l2 = 0; l2 < R2; ++l2) park[row_off<true>(l1 + R1 * l2, g.sn) + m * 8] = Y[i][l2];
          }
        }
      }
      if (a.last) inverse_store(0);
    } else {
      // fan-out: this launch handles the outputs of one basis power p: the
      // input tile is transformed, scaled by c(k) D(w_x)^p and inverse
      // transformed.  The host launches the bases in increasing p (one
      // launch each, so that the register arrays of one basis are all that
      // is live); an output that aliases the input has the highest p of its
      // op, so the input is intact for every earlier basis.
      const int p = a.pbasis;
      forward(0);
#pragma unroll
      for (int i = 0; i < IB; ++i) {
        const int it = tid + i * kThreads;
        const int m = it % M, l1 = it / M;
        int ky, kz;
        freq(m, ky, kz);
#pragma unroll
        for (int l2 = 0; l2 < R2; ++l2) {
          const int kx = l1 + R1 * l2;
          Y[i][l2] = it < M * R1 ? cscale(X[i][l2], common_factor<N>(op, t, kx, ky, kz) * powp(t.dxy[kx], p))
                                 : make_float2(0.f, 0.f);
        }
      }
      inverse_store(p);
    }
  }
}


// The force's common factor c(k) = scale W(k)^-n S(k) / K^2(k) at
// kx = l1 + R1 l2 for every l2 of one stage-B item (column (ky, kz)).  The
// per-kx table values are loaded together and pinned before use: a table
// load issued after a store through another pointer would wait for that
// store.  The reciprocal is the hardware one (<= 1 ulp); an IEEE divide per
// element costs about ten instructions.  FILT = false leaves out the
// deconvolution and split branches (their registers included): callers
// that take it are launched only for ops with neither.
template <int R1, int R2, bool FILT = true>
__device__ __forceinline__ void force_factors(const FftTables& t, const SpecOp& op, int l1, int ky, int kz,
                                              float (&fac)[R2]) {
  float aux[R2];
#pragma unroll
  for (int l2 = 0; l2 < R2; ++l2) fac[l2] = t.kxy[l1 + R1 * l2];
#pragma unroll
  for (int l2 = 0; l2 < R2; ++l2) asm volatile("" : "+v"(fac[l2]));
  const float kyz = t.kxy[ky] + t.kz[kz];
#pragma unroll
  for (int l2 = 0; l2 < R2; ++l2) {
    const float kk = fac[l2] + kyz;
    fac[l2] = kk > 0.f ? op.scale * __builtin_amdgcn_rcpf(kk) : 0.f;
  }
  if (FILT && op.deconv) {
    const float wyz = t.wxy[ky] * t.wz[kz];
#pragma unroll
    for (int l2 = 0; l2 < R2; ++l2) aux[l2] = t.wxy[l1 + R1 * l2];
#pragma unroll
    for (int l2 = 0; l2 < R2; ++l2) {
      const float wv = aux[l2] * wyz;
      fac[l2] *= __builtin_amdgcn_rcpf(op.deconv == 1 ? wv : wv * wv);
    }
  }
  if (FILT && op.split) {
    const float syz = t.sxy[ky] * t.sz[kz];
#pragma unroll
    for (int l2 = 0; l2 < R2; ++l2) aux[l2] = t.sxy[l1 + R1 * l2];
#pragma unroll
    for (int l2 = 0; l2 < R2; ++l2) {
      const float sv = aux[l2] * syz;
      fac[l2] *= (op.split == 1 ? sv : 1.f - sv);
    }
  }
}

// The force's whole x pass in one tile (OP_FORCE_XS, N >= 64): the forward
// x transform, times c(k), then two inverse x transforms, each output times
// i: D(w_x) c X into out[0] (F_x, over the input) and c X into out[1] (the
// factor F_y and F_z share).  The forward transform leaves item (m, l1)
// holding kx = l1 + R1 l2 for every l2, which are exactly the inputs of the
// inverse's first stage (an R2-point transform over l2, then R1 points over
// l1): the scaled spectrum stays in registers between the transforms, and
// the pass moves one read and two writes of the spectrum instead of three
// of each.  The inverse twiddles come from an R1 x R2 table in LDS, filled
// with the first loads, so no global load waits behind the stores of the
// first output.
template <int N, int M>
__global__ __launch_bounds__(kThreads) void k_fft_x_force(FusedArgs a) {
  constexpr int R1 = Split<N>::R1, R2 = Split<N>::R2;
  static_assert(R2 > 1, "columns split over two stages");
  constexpr int IA = (M * R2 + kThreads - 1) / kThreads;   // forward stage A, inverse stage B
  constexpr int IB = (M * R1 + kThreads - 1) / kThreads;   // forward stage B, inverse stage A
  constexpr int SA = ColLds<N, M>::SA, SB = ColLds<N, M>::SB;
  __shared__ float2 lds[ColLds<N, M>::size];
  __shared__ float2 tws[R1 * R2];   // exp(-2 pi i l j / N), l < R1, j < R2
  int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int mode = tile >= a.nb_main ? 1 : 0;
  if (mode) tile -= a.nb_main;
  const ColGeom& g = mode ? a.gp : a.gm;
  int b, c0;
  if (mode == 0) {   // blocks of 8 ky rows, walked column chunk by column chunk
    const int blk = tile / (8 * g.ntc), r = tile - blk * (8 * g.ntc);
    b = blk * 8 + (r & 7);
    c0 = (r >> 3) * M;
  } else {
    tile_bc<true>(tile, ((int)gridDim.x - a.nb_main) / g.ntc, g.ntc, M, b, c0);
  }
  const long bo = batch_bytes(a.bat);
  if (bo < 0) return;
  const long off = b * g.sb + (long)c0 * 8 + bo / (long)sizeof(float2);
  const int tid = threadIdx.x;
  const SpecOp& op = a.op;
  const FftTables& t = a.t;
  const float2* src = (mode == 0 ? a.in_main : a.in_nyq) + off;
  // (ky, kz) of column m; masked columns map to the zero mode
  auto freq = [&](int m, int& ky, int& kz) {
    if (c0 + m >= g.ncols) { ky = 0; kz = 0; }
    else if (mode == 0) { ky = b; kz = c0 + m; }
    else { ky = c0 + m; kz = N / 2; }
  };
  constexpr int IT = (R1 * R2 + kThreads - 1) / kThreads;
  float2 twv[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int e = tid + k * kThreads;
    if (e < R1 * R2) twv[k] = t.tw_n[(e / R2) * (e % R2)];
  }
  // forward stage A: rows x = R2 j1 + j2, all loads first (non-temporal:
  // the two outputs, not the input, gain from staying in L2, measured 3.61
  // -> 3.30 ms); the twiddles come from the table once it is in LDS
  float2 v[IA][R1];
#pragma unroll
  for (int i = 0; i < IA; ++i) {
    const int it = tid + i * kThreads;
    const int m = it % M, j2 = it / M;
    const bool ok = it < M * R2 && c0 + m < g.ncols;
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1)
      v[i][j1] = ok ? ldnt(&src[row_off<true>(R2 * j1 + j2, g.sn) + m * 8]) : make_float2(0.f, 0.f);
  }
  // c(k) and D(w_x) of the stage-B item (m, l1), kx = l1 + R1 l2, loaded
  // behind the columns and before any store
  float fac[IB][R2], dxv[IB][R2];
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    const int it = tid + i * kThreads;
    if (it < M * R1) {
      const int m = it % M, l1 = it / M;
      int ky, kz;
      freq(m, ky, kz);
      force_factors<R1, R2>(t, op, l1, ky, kz, fac[i]);
#pragma unroll
      for (int l2 = 0; l2 < R2; ++l2) dxv[i][l2] = t.dxy[l1 + R1 * l2];
    }
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int e = tid + k * kThreads;
    if (e < R1 * R2) tws[e] = twv[k];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IA; ++i) {
    const int it = tid + i * kThreads;
    if (it < M * R2) {
      const int m = it % M, j2 = it / M;
      dft<R1, -1>(v[i]);
#pragma unroll
      for (int l1 = 0; l1 < R1; ++l1) lds[l1 * SA + j2 * M + m] = l1 == 0 ? v[i][l1] : cmul(v[i][l1], tws[l1 * R2 + j2]);
    }
  }
  __syncthreads();
  // forward stage B: kx = l1 + R1 l2, times c(k) into X
  float2 X[IB][R2];
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    const int it = tid + i * kThreads;
    if (it < M * R1) {
      const int m = it % M, l1 = it / M;
#pragma unroll
      for (int l2 = 0; l2 < R2; ++l2) X[i][l2] = lds[l1 * SA + l2 * M + m];
      dft<R2, -1>(X[i]);
#pragma unroll
      for (int l2 = 0; l2 < R2; ++l2) X[i][l2] = cscale(X[i][l2], fac[i][l2]);
    }
  }
  __syncthreads();
  // inverse of D(w_x)^p c X; outputs x = lp + R2 l2p, stored times i
  auto inverse = [&](int p, float2* dst) {
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      const int it = tid + i * kThreads;
      if (it < M * R1) {
        const int m = it % M, l1 = it / M;
        float2 y[R2];
#pragma unroll
        for (int l2 = 0; l2 < R2; ++l2) y[l2] = p ? cscale(X[i][l2], dxv[i][l2]) : X[i][l2];
        dft<R2, 1>(y);
#pragma unroll
        for (int lp = 0; lp < R2; ++lp)
          lds[lp * SB + l1 * M + m] = lp == 0 ? y[0] : cmulc(y[lp], tws[l1 * R2 + lp]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int it = tid + i * kThreads;
      if (it < M * R2) {
        const int m = it % M, lp = it / M;
        float2 v[R1];
#pragma unroll
        for (int l1 = 0; l1 < R1; ++l1) v[l1] = lds[lp * SB + l1 * M + m];
        dft<R1, 1>(v);
        if (c0 + m < g.ncols) {
#pragma unroll
          for (int l2p = 0; l2p < R1; ++l2p) dst[row_off<true>(lp + R2 * l2p, g.sn) + m * 8] = cmul_i<1>(v[l2p]);
        }
      }
    }
  };
  inverse(0, (mode == 0 ? op.out_c[1] : op.out_q[1]) + off);
  __syncthreads();
  inverse(1, (mode == 0 ? op.out_c[0] : op.out_q[0]) + off);
}


// The transposed force's whole x pass (OP_FORCE_T, N >= 64) in one tile:
// with Y_d the forward-(z, y) spectra of the three painted channels, the
// result is the inverse x transform of -i g(k) times the forward x
// transform of
//   w(x) = S[Y_x](x) + D(w_y) Y_y(x) + D(w_z) Y_z(x),
// where S is the periodic five-point stencil whose discrete Fourier symbol
// is exactly D(w_x) (shift theorem):
//   S[Y](x) = [8 (Y(x+1) - Y(x-1)) - (Y(x+2) - Y(x-2))] / (12 i),
// so one forward transform serves all three channels.  D(w_y) and D(w_z)
// are constant along x.  A tile holds whole x columns, so the stencil reads
// its neighbours from a staging copy of the Y_x tile in LDS.  The result
// replaces Y_x; the register hand-over between the forward and the inverse
// transform is that of k_fft_x_force.  (The stencil differences a painted
// cotangent field, not a smooth potential, so it costs no precision that
// the spectral product keeps.)
template <int N, int M, bool FILT>
__global__ __launch_bounds__(kThreads) void k_fft_x_force_t(FusedArgs a) {
  constexpr int R1 = Split<N>::R1, R2 = Split<N>::R2;
  static_assert(R2 > 1, "columns split over two stages");
  static_assert(N * M <= ColLds<N, M>::size, "the staging copy fits the exchange buffer");
  constexpr int IA = (M * R2 + kThreads - 1) / kThreads;   // forward stage A, inverse stage B
  constexpr int IB = (M * R1 + kThreads - 1) / kThreads;   // forward stage B, inverse stage A
  constexpr int SA = ColLds<N, M>::SA, SB = ColLds<N, M>::SB;
  constexpr int IT = (R1 * R2 + kThreads - 1) / kThreads;
  __shared__ float2 lds[ColLds<N, M>::size];
  __shared__ float2 tws[R1 * R2];   // exp(-2 pi i l j / N), l < R1, j < R2
  int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int mode = tile >= a.nb_main ? 1 : 0;
  if (mode) tile -= a.nb_main;
  const ColGeom& g = mode ? a.gp : a.gm;
  int b, c0;
  tile_bc<true>(tile, mode ? ((int)gridDim.x - a.nb_main) / g.ntc : a.nb_main / g.ntc, g.ntc, M, b, c0);
  const long off = b * g.sb + (long)c0 * 8;
  const int tid = threadIdx.x;
  const SpecOp& op = a.op;
  const FftTables& t = a.t;
  const float2* yx = (mode == 0 ? op.in_c[0] : op.in_q[0]) + off;
  const float2* yy = (mode == 0 ? op.in_c[1] : op.in_q[1]) + off;
  const float2* yz = (mode == 0 ? op.in_c[2] : op.in_q[2]) + off;
  // (ky, kz) of column m; masked columns map to the zero mode
  auto freq = [&](int m, int& ky, int& kz) {
    if (c0 + m >= g.ncols) { ky = 0; kz = 0; }
    else if (mode == 0) { ky = b; kz = c0 + m; }
    else { ky = c0 + m; kz = N / 2; }
  };
  float2 twv[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int e = tid + k * kThreads;
    if (e < R1 * R2) twv[k] = t.tw_n[(e / R2) * (e % R2)];
  }
  // rows x = R2 j1 + j2: Y_x to the staging copy, D(w_y) Y_y + D(w_z) Y_z
  // into w
  float2 w[IA][R1];
#pragma unroll
  for (int i = 0; i < IA; ++i) {
    const int it = tid + i * kThreads;
    const int m = it % M, j2 = it / M;
    const bool ok = it < M * R2 && c0 + m < g.ncols;
    int ky, kz;
    freq(m, ky, kz);
    const float dy = t.dxy[ky], dz = t.dz[kz];
    float2 vx[R1];
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) vx[j1] = ok ? yx[row_off<true>(R2 * j1 + j2, g.sn) + m * 8] : make_float2(0.f, 0.f);
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      const float2 py = ok ? yy[row_off<true>(R2 * j1 + j2, g.sn) + m * 8] : make_float2(0.f, 0.f);
      const float2 pz = ok ? yz[row_off<true>(R2 * j1 + j2, g.sn) + m * 8] : make_float2(0.f, 0.f);
      w[i][j1] = make_float2(dy * py.x + dz * pz.x, dy * py.y + dz * pz.y);
    }
    if (it < M * R2) {
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1) lds[(R2 * j1 + j2) * M + m] = vx[j1];
    }
  }
  // c(k) of the stage-B item (m, l1), kx = l1 + R1 l2
  float fac[IB][R2];
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    const int it = tid + i * kThreads;
    if (it < M * R1) {
      const int m = it % M, l1 = it / M;
      int ky, kz;
      freq(m, ky, kz);
      force_factors<R1, R2, FILT>(t, op, l1, ky, kz, fac[i]);
    }
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int e = tid + k * kThreads;
    if (e < R1 * R2) tws[e] = twv[k];
  }
  __syncthreads();
  // w += S[Y_x]: d / (12 i) = (d.y, -d.x) / 12
#pragma unroll
  for (int i = 0; i < IA; ++i) {
    const int it = tid + i * kThreads;
    if (it < M * R2) {
      const int m = it % M, j2 = it / M;
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1) {
        const int x = R2 * j1 + j2;
        const float2 p1 = lds[((x + 1) & (N - 1)) * M + m], m1 = lds[((x - 1) & (N - 1)) * M + m];
        const float2 p2 = lds[((x + 2) & (N - 1)) * M + m], m2 = lds[((x - 2) & (N - 1)) * M + m];
        const float2 d = make_float2(8.f * (p1.x - m1.x) - (p2.x - m2.x), 8.f * (p1.y - m1.y) - (p2.y - m2.y));
        constexpr float k12 = 1.f / 12.f;
        w[i][j1] = make_float2(w[i][j1].x + k12 * d.y, w[i][j1].y - k12 * d.x);
      }
    }
  }
  __syncthreads();   // the staging copy is read before the exchange reuses it
  // forward stage A
#pragma unroll
  for (int i = 0; i < IA; ++i) {
    const int it = tid + i * kThreads;
    if (it < M * R2) {
      const int m = it % M, j2 = it / M;
      dft<R1, -1>(w[i]);
#pragma unroll
      for (int l1 = 0; l1 < R1; ++l1) lds[l1 * SA + j2 * M + m] = l1 == 0 ? w[i][l1] : cmul(w[i][l1], tws[l1 * R2 + j2]);
    }
  }
  __syncthreads();
  // forward stage B (kx = l1 + R1 l2), times -i g: (a + i b)(-i g) = g b - i g a
  float2 Z[IB][R2];
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    const int it = tid + i * kThreads;
    if (it < M * R1) {
      const int m = it % M, l1 = it / M;
#pragma unroll
      for (int l2 = 0; l2 < R2; ++l2) Z[i][l2] = lds[l1 * SA + l2 * M + m];
      dft<R2, -1>(Z[i]);
#pragma unroll
      for (int l2 = 0; l2 < R2; ++l2) Z[i][l2] = make_float2(fac[i][l2] * Z[i][l2].y, -fac[i][l2] * Z[i][l2].x);
    }
  }
  __syncthreads();
  // inverse x transform of Z; outputs x = lp + R2 l2p
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    const int it = tid + i * kThreads;
    if (it < M * R1) {
      const int m = it % M, l1 = it / M;
      dft<R2, 1>(Z[i]);
#pragma unroll
      for (int lp = 0; lp < R2; ++lp)
        lds[lp * SB + l1 * M + m] = lp == 0 ? Z[i][0] : cmulc(Z[i][lp], tws[l1 * R2 + lp]);
    }
  }
  __syncthreads();
  float2* dst = (mode == 0 ? op.out_c[0] : op.out_q[0]) + off;
#pragma unroll
  for (int i = 0; i < IA; ++i) {
    const int it = tid + i * kThreads;
    if (it < M * R2) {
      const int m = it % M, lp = it / M;
      float2 v[R1];
#pragma unroll
      for (int l1 = 0; l1 < R1; ++l1) v[l1] = lds[lp * SB + l1 * M + m];
      dft<R1, 1>(v);
      if (c0 + m < g.ncols) {
#pragma unroll
        for (int l2p = 0; l2p < R1; ++l2p) dst[row_off<true>(lp + R2 * l2p, g.sn) + m * 8] = v[l2p];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

template <int N, int DIR, bool BLK>
void launch_cols(float2* const* dm, float2* const* dq, int nf, ColGeom gm, int nbm, ColGeom gp, int nbp,
                 const float2* tw, hipStream_t s, const BatchArg& bat = BatchArg()) {
  constexpr int M = BLK ? Cols<N>::M : YTile<N>::M;
  constexpr int TH = BLK ? kThreads : YTile<N>::TH;
  ColPass p;
  for (int i = 0; i < 3; ++i) {
    p.main[i] = dm[i < nf ? i : 0];
    p.plane[i] = dq[i < nf ? i : 0];
  }
  gm.ntc = cdiv(gm.ncols, M);
  gp.ntc = cdiv(gp.ncols, M);
  p.gm = gm;
  p.gp = gp;
  p.nb_main = nbm * gm.ntc;
  p.ntiles = p.nb_main + nbp * gp.ntc;
  p.bat = bat;
  dim3 grid(p.ntiles, nf, bat.n);
  hipLaunchKernelGGL((k_fft_cols<N, M, DIR, BLK, TH>), grid, dim3(TH), 0, s, p, tw);
}

// y pass over the main arrays and the Nyquist planes of nf fields
template <int N, int DIR>
void ypass(const FftTables& t, Field* f, int nf, hipStream_t s, const BatchArg& bat = BatchArg()) {
  float2* dm[3];
  float2* dq[3];
  for (int i = 0; i < nf; ++i) { dm[i] = f[i].c(); dq[i] = f[i].q; }
  // main c[xb][y][kz][xi]: (b = xb, n = y, c = kz*8 + xi): sb = 4N^2, sn = 4N, ncols = 4N
  // Nyquist plane q[xb][y][xi]: (b = xb, n = y, c = xi): sb = 8N, sn = 8, ncols = 8
  launch_cols<N, DIR, false>(dm, dq, nf, ColGeom{4L * N * N, 4L * N, 4 * N, 0}, N / 8,
                             ColGeom{8L * N, 8, 8, 0}, N / 8, t.tw_n, s, bat);
}

template <int N, int DIR>
void xpass(const FftTables& t, Field* f, int nf, hipStream_t s) {
  float2* dm[3];
  float2* dq[3];
  for (int i = 0; i < nf; ++i) { dm[i] = f[i].c(); dq[i] = f[i].q; }
  // main c[xb][y][kz][xi]: (b = y, n = x, c = kz): sb = 4N, row(x) = xb*4N^2 + xi, column stride 8
  // Nyquist plane q[xb][y][xi]: (b = 0, n = x, c = y): row(x) = xb*8N + xi, column stride 8
  launch_cols<N, DIR, true>(dm, dq, nf, ColGeom{4L * N, 4L * N * N, N / 2, 0}, N, ColGeom{0, 8L * N, N, 0}, 1,
                            t.tw_n, s);
}

template <int N>
void zr2c(const FftTables& t, Field* f, int nf, hipStream_t s, const BatchArg& bat = BatchArg()) {
  using G = ZGeom<N>;
  dim3 grid((N * N) / G::L, nf, bat.n);
  hipLaunchKernelGGL((k_r2c_z<N>), grid, dim3(kThreads), 0, s, f[0].r, nf > 1 ? f[1].r : f[0].r,
                     nf > 2 ? f[2].r : f[0].r, f[0].q, nf > 1 ? f[1].q : f[0].q, nf > 2 ? f[2].q : f[0].q,
                     t.tw_h, t.tw_n, bat);
}

template <int N>
void zc2r3(const FftTables& t, const Field* f, float* out, hipStream_t s, const BatchArg& bat = BatchArg()) {
  dim3 grid(3 * (N * N) / Z3Geom<N>::L, 1, bat.n);
  hipLaunchKernelGGL((k_c2r_z3<N>), grid, dim3(kThreads), 0, s, f[0].r, (long)(f[1].r - f[0].r), f[0].q,
                     (long)(f[1].q - f[0].q), out, t.tw_h, t.tw_n, bat);
}

template <int N>
void zc2r(const FftTables& t, Field* f, int nf, hipStream_t s) {
  using G = ZGeom<N>;
  dim3 grid((N * N) / G::L, nf);
  hipLaunchKernelGGL((k_c2r_z<N>), grid, dim3(kThreads), 0, s, f[0].r, nf > 1 ? f[1].r : f[0].r,
                     nf > 2 ? f[2].r : f[0].r, f[0].q, nf > 1 ? f[1].q : f[0].q, nf > 2 ? f[2].q : f[0].q,
                     t.tw_h, t.tw_n);
}

template <int N>
void xfused(const FftTables& t, const Field& in, const SpecOp& op, hipStream_t s) {
  constexpr int M = Cols<N>::M;
  FusedArgs a;
  a.op = op;
  a.t = t;
  a.in_main = in.c();
  a.in_nyq = in.q;
  a.gm = ColGeom{4L * N, 4L * N * N, N / 2, cdiv(N / 2, M)};
  a.gp = ColGeom{0, 8L * N, N, cdiv(N, M)};
  a.nb_main = N * a.gm.ntc;
  const dim3 grid(a.nb_main + a.gp.ntc);
  a.pbasis = 0;
  a.first = a.last = 1;
  a.park_main = nullptr;
  a.park_nyq = nullptr;
  const bool fan_in = op_fan_in(op.kind);
  const int nterm = fan_in ? op.n_in : op.n_out;
  int pmask = 0, first_in = -1;
  for (int o = 0; o < nterm; ++o) pmask |= 1 << op_term(op.kind, o).p;
  if (fan_in && Split<N>::R2 == 1) {   // whole columns in registers: all bases in one launch
    hipLaunchKernelGGL((k_fft_x_fused<N, M, true>), grid, dim3(kThreads), 0, s, a);
    return;
  }
  const int pfirst = __builtin_ctz(pmask), plast = 31 - __builtin_clz(pmask);
  if (fan_in) {
    for (int o = 0; o < nterm && first_in < 0; ++o)
      if (op_term(op.kind, o).p == pfirst) first_in = o;
    a.park_main = op.in_c[first_in];
    a.park_nyq = op.in_q[first_in];
  }
  for (int p = pfirst; p <= plast; ++p) {
    if (!(pmask >> p & 1)) continue;
    a.pbasis = p;
    a.first = p == pfirst;
    a.last = p == plast;
    if (fan_in)
      hipLaunchKernelGGL((k_fft_x_fused<N, M, true>), grid, dim3(kThreads), 0, s, a);
    else
      hipLaunchKernelGGL((k_fft_x_fused<N, M, false>), grid, dim3(kThreads), 0, s, a);
  }
}

// The force's x pass: for N >= 64 (OP_FORCE_XS) one launch of
// k_fft_x_force, for N <= 32 (OP_FORCE, whole columns in registers) the
// fused register pass.
template <int N>
void xforce(const FftTables& t, const Field& in, const SpecOp& op, hipStream_t s, const BatchArg& bat = BatchArg()) {
  constexpr int M = Cols<N>::M;
  if constexpr (Split<N>::R2 == 1) {
    xfused<N>(t, in, op, s);
  } else {
    FusedArgs a;
    a.op = op;
    a.t = t;
    a.in_main = in.c();
    a.in_nyq = in.q;
    a.gm = ColGeom{4L * N, 4L * N * N, N / 2, cdiv(N / 2, M)};
    a.gp = ColGeom{0, 8L * N, N, cdiv(N, M)};
    a.nb_main = N * a.gm.ntc;
    a.first = a.last = 1;
    a.park_main = nullptr;
    a.park_nyq = nullptr;
    a.pbasis = 0;
    a.bat = bat;
    const dim3 grid(a.nb_main + a.gp.ntc, 1, bat.n);
    hipLaunchKernelGGL((k_fft_x_force<N, M>), grid, dim3(kThreads), 0, s, a);
  }
}

// The transposed force's x pass (one launch of k_fft_x_force_t) over
// f[0..2] = the forward-(z, y) spectra of the x, y, z inputs; the result
// replaces f[0], f[1] and f[2] are left as they were.
template <int N>
void xforce_t(const FftTables& t, Field* f, const SpecOp& op, hipStream_t s) {
  if constexpr (Split<N>::R2 > 1) {
    constexpr int M = Cols<N>::M;
    FusedArgs a;
    a.op = op;
    a.t = t;
    a.gm = ColGeom{4L * N, 4L * N * N, N / 2, cdiv(N / 2, M)};
    a.gp = ColGeom{0, 8L * N, N, cdiv(N, M)};
    a.nb_main = N * a.gm.ntc;
    a.first = a.last = 1;
    a.park_main = nullptr;
    a.park_nyq = nullptr;
    a.pbasis = 0;
    for (int d = 0; d < 3; ++d) {
      a.op.in_c[d] = f[d].c();
      a.op.in_q[d] = f[d].q;
    }
    a.op.out_c[0] = f[0].c();
    a.op.out_q[0] = f[0].q;
    a.in_main = f[0].c();
    a.in_nyq = f[0].q;
    const dim3 grid(a.nb_main + a.gp.ntc);
    if (op.deconv || op.split)
      hipLaunchKernelGGL((k_fft_x_force_t<N, M, true>), grid, dim3(kThreads), 0, s, a);
    else
      hipLaunchKernelGGL((k_fft_x_force_t<N, M, false>), grid, dim3(kThreads), 0, s, a);
  }
}

template <int N>
void yforce(const FftTables& t, Field* f, hipStream_t s, const BatchArg& bat = BatchArg()) {
  if constexpr (Split<N>::R2 > 1) {
    constexpr int M = YTile<N>::M, TH = YTile<N>::TH;
    ColPass p;
    const int order[3] = {0, 2, 1};   // F_x, shared factor (F_z), F_y
    for (int i = 0; i < 3; ++i) {
      p.main[i] = f[order[i]].c();
      p.plane[i] = f[order[i]].q;
    }
    // geometry of ypass: main c[xb][y][kz][xi], Nyquist plane q[xb][y][xi]
    p.gm = ColGeom{4L * N * N, 4L * N, 4 * N, cdiv(4 * N, M)};
    p.gp = ColGeom{8L * N, 8, 8, cdiv(8, M)};
    p.nb_main = (N / 8) * p.gm.ntc;
    p.bat = bat;
    const dim3 grid(p.nb_main + (N / 8) * p.gp.ntc, 2, bat.n);
    hipLaunchKernelGGL((k_fft_cols_force<N, M, TH>), grid, dim3(TH), 0, s, p, t.tw_n, t.dxy, t.dz);
  }
}

// chunks of at most 3 fields per launch (blockIdx.y selects the field)
template <class Fn>
void by3(Field* f, int nf, Fn fn) {
  for (int i = 0; i < nf; i += 3) fn(f + i, nf - i < 3 ? nf - i : 3);
}

}  // namespace

#define PM_FFT_SWITCH(n, CALL)                            \
  switch (n) {                                            \
    case 8: CALL(8); break;                               \
    case 16: CALL(16); break;                             \
    case 32: CALL(32); break;                             \
    case 64: CALL(64); break;                             \
    case 128: CALL(128); break;                           \
    case 256: CALL(256); break;                           \
    case 512: CALL(512); break;                           \
    case 1024: CALL(1024); break;                         \
    default: break;                                       \
  }

void fft_r2c_zy(const FftTables& t, Field* f, int nf, hipStream_t s) {
  by3(f, nf, [&](Field* g, int k) {
#define CALL(N) zr2c<N>(t, g, k, s); ypass<N, -1>(t, g, k, s)
    PM_FFT_SWITCH(t.n, CALL)
#undef CALL
  });
}

void fft_z_r2c(const FftTables& t, Field* f, int nf, hipStream_t s, const BatchArg& bat) {
  by3(f, nf, [&](Field* g, int k) {
#define CALL(N) zr2c<N>(t, g, k, s, bat)
    PM_FFT_SWITCH(t.n, CALL)
#undef CALL
  });
}

void fft_y(const FftTables& t, Field* f, int nf, int dir, hipStream_t s, const BatchArg& bat) {
  by3(f, nf, [&](Field* g, int k) {
#define CALL(N) (dir < 0 ? ypass<N, -1>(t, g, k, s, bat) : ypass<N, 1>(t, g, k, s, bat))
    PM_FFT_SWITCH(t.n, CALL)
#undef CALL
  });
}

void fft_z_c2r(const FftTables& t, Field* f, int nf, hipStream_t s) {
  by3(f, nf, [&](Field* g, int k) {
#define CALL(N) zc2r<N>(t, g, k, s)
    PM_FFT_SWITCH(t.n, CALL)
#undef CALL
  });
}

void fft_x_forward(const FftTables& t, Field* f, int nf, hipStream_t s) {
  by3(f, nf, [&](Field* g, int k) {
#define CALL(N) xpass<N, -1>(t, g, k, s)
    PM_FFT_SWITCH(t.n, CALL)
#undef CALL
  });
}

void fft_x_inverse(const FftTables& t, Field* f, int nf, hipStream_t s) {
  by3(f, nf, [&](Field* g, int k) {
#define CALL(N) xpass<N, 1>(t, g, k, s)
    PM_FFT_SWITCH(t.n, CALL)
#undef CALL
  });
}

void fft_x_fused(const FftTables& t, const Field& in, const SpecOp& op, hipStream_t s) {
#define CALL(N) xfused<N>(t, in, op, s)
  PM_FFT_SWITCH(t.n, CALL)
#undef CALL
}

void fft_x_force(const FftTables& t, const Field& in, const SpecOp& op, hipStream_t s, const BatchArg& bat) {
#define CALL(N) xforce<N>(t, in, op, s, bat)
  PM_FFT_SWITCH(t.n, CALL)
#undef CALL
}

void fft_x_force_t(const FftTables& t, Field* f, const SpecOp& op, hipStream_t s) {
  if (t.n < 64) {   // whole columns in registers: the fused fan-in pass
    fft_x_fused(t, f[0], op, s);
    return;
  }
#define CALL(N) xforce_t<N>(t, f, op, s)
  PM_FFT_SWITCH(t.n, CALL)
#undef CALL
}

void fft_y_force(const FftTables& t, Field* f, hipStream_t s, const BatchArg& bat) {
#define CALL(N) yforce<N>(t, f, s, bat)
  PM_FFT_SWITCH(t.n, CALL)
#undef CALL
}

void fft_z_c2r_interleaved3(const FftTables& t, const Field* f, float* out, hipStream_t s, const BatchArg& bat) {
#define CALL(N) zc2r3<N>(t, f, out, s, bat)
  PM_FFT_SWITCH(t.n, CALL)
#undef CALL
}

void fft_c2r_yz(const FftTables& t, Field* f, int nf, hipStream_t s) {
  by3(f, nf, [&](Field* g, int k) {
#define CALL(N) ypass<N, 1>(t, g, k, s); zc2r<N>(t, g, k, s)
    PM_FFT_SWITCH(t.n, CALL)
#undef CALL
  });
}

}  // namespace pmk
