// Particle-side kernels of the PM step for gfx950: white noise, LPT particle
// assembly, counting sort by tile, LDS-tiled CIC paint, LDS-tiled CIC readout
// fused with the kick and drift updates, and the binned power spectrum.
//
// Tiles.  The mesh is cut into T^3-cell tiles.  A particle whose CIC base
// cell floor(x) lies in tile t gets key (8*t + c)*8 + b, where the class bit
// c_d is set when floor(x_d) is the last cell of the tile along d, i.e. when
// the particle also deposits into the next tile along d, and b names the
// half-tile block of floor(x).  A counting sort by key groups the particles
// of every tile in 8 contiguous (tile, class) bins, each ordered by block.
//  - Paint: the workgroup of tile t accumulates, in LDS, its own particles
//    and those particles of the 7 lower neighbour tiles whose class says they
//    reach into t, keeping only the corners inside t.  Every mesh cell is
//    written once, by its owner, with no global float atomics.
//  - Readout: one sorted particle per thread gathers its 8 corners from the
//    interleaved force mesh; sorted neighbours share cache lines.
// Meshes use the x-blocked layout of layout.h.
#include "particles.h"
#include "pm_device.h"

namespace pmk {
namespace {

constexpr int kThreads = 256;

// ---- white noise ------------------------------------------------------------
// SplitMix64 output of the counter seed*2^40 + i, Box-Muller (cosine branch).
// The counter is the site index (x*n + y)*n + z; blocked != 0 writes the
// x-blocked layout (element e holds site blk_real_xyz(e)).
__global__ void k_noise(uint64_t seed, long n3, int ln, int blocked, float* __restrict__ out) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += stride) {
    long site = i;
    if (blocked) {
      int x, y, zc;
      blk_real_xyz(i, ln, x, y, zc);
      site = ((((long)x << ln) + y) << ln) + zc;
    }
    uint64_t z = seed * (1ull << 40) + (uint64_t)site + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u1 = ((double)(z >> 32) + 1.0) * 2.3283064365386963e-10;
    const double u2 = (double)(z & 0xFFFFFFFFull) * 2.3283064365386963e-10;
    out[i] = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
  }
}

// ---- LPT -----------------------------------------------------------------------
// delta2 = phi_xx phi_yy + phi_xx phi_zz + phi_yy phi_zz - phi_xy^2 - phi_xz^2 - phi_yz^2
__global__ void k_lpt_delta2(const float* __restrict__ xx, const float* __restrict__ yy,
                             const float* __restrict__ zz, const float* __restrict__ xy,
                             const float* __restrict__ xz, const float* __restrict__ yz, long n,
                             float* __restrict__ out) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float a = xx[i], b = yy[i], c = zz[i], d = xy[i], e = xz[i], f = yz[i];
    out[i] = a * b + a * c + b * c - d * d - e * e - f * f;
  }
}

// x = B q + shift + B (D1 s1 + D2 s2) (wrapped); p = B a0^2 E (f1 D1 s1 + f2 D2 s2)
// np is a power of two: the lattice site comes from shifts (a 64-bit
// division per particle costs more than the particle's memory traffic), and
// position and momentum are stored as one 12-byte access each.
__global__ void k_lpt_particles(LptParticleArgs a) {
  const int ln = __builtin_ctz(a.np);
  const long n3 = 1L << (3 * ln);
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += stride) {
    const int q[3] = {(int)(i >> (2 * ln)), (int)((i >> ln) & (a.np - 1)), (int)(i & (a.np - 1))};
    const long e = blk_real(q[0], q[1], q[2], a.np);   // lattice fields are x-blocked
    float x[3], p[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float s1 = a.s1[d][e];
      const float s2 = a.has_s2 ? a.s2[d][e] : 0.f;
      const float dx = a.cx1 * s1 + a.cx2 * s2;
      x[d] = wrap_pos((float)(a.ratio * q[d]) + a.shift + dx, a.nmesh);
      p[d] = a.cp1 * s1 + a.cp2 * s2;
      if (a.psi1) {
        a.psi1[3 * i + d] = (float)a.ratio * s1;
        a.psi2[3 * i + d] = (float)a.ratio * s2;
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) a.pos[3 * i + d] = x[d];
#pragma unroll
    for (int d = 0; d < 3; ++d) a.mom[3 * i + d] = p[d];
  }
}

// ---- counting sort -------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* __restrict__ p, long n, uint32_t v, BatchArg bat) {
  const long bo = batch_bytes(bat);
  if (bo < 0) return;
  p = byte_adv(p, bo);
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Sort key of each particle, counted per key (one atomic per group of equal
// keys in the wave); particles in lattice order (lat_ln >= 0) are visited
// brick by brick, so that a wave holds a few keys instead of eight tiles'.
__global__ __launch_bounds__(kThreads) void k_keys(const float* __restrict__ pos, long np, TileGeom g,
                                                   uint32_t* __restrict__ key, uint32_t* __restrict__ count,
                                                   int lat_ln) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < np;
  const long i = valid && lat_ln >= 0 ? lattice_order(t, lat_ln) : t;
  uint32_t k = 0;
  if (valid) {
    int ix, iy, iz;
    float t;
    cic_base(pos[3 * i + 0], g.n, ix, t);
    cic_base(pos[3 * i + 1], g.n, iy, t);
    cic_base(pos[3 * i + 2], g.n, iz, t);
    k = tile_key(ix, iy, iz, g);
  }
  agg_count(count, k, valid);
  if (valid) key[i] = k;
}

// Exclusive scan of count[0..n) into off[0..n], off[n] = total.
constexpr int kScanItems = 8;
constexpr int kScanBlock = kThreads * kScanItems;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < kThreads; o <<= 1) {
    const uint32_t add = tid >= o ? sh[tid - o] : 0u;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  total = sh[kThreads - 1];
  const uint32_t incl = sh[tid];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kThreads) void k_scan_local(const uint32_t* __restrict__ cnt, long n,
                                                         uint32_t* __restrict__ off, uint32_t* __restrict__ bsum,
                                                         BatchArg bat) {
  __shared__ uint32_t sh[kThreads];
  const long bo = batch_bytes(bat);
  if (bo < 0) return;
  cnt = byte_adv(cnt, bo);
  off = byte_adv(off, bo);
  bsum = byte_adv(bsum, bo);
  const long base = (long)blockIdx.x * kScanBlock + (long)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = base + j < n ? cnt[base + j] : 0u;
    s += v[j];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, sh, total);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) off[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_top(uint32_t* __restrict__ bsum, int nb, BatchArg bat) {
  __shared__ uint32_t sh[kThreads];
  const long bo = batch_bytes(bat);
  if (bo < 0) return;
  bsum = byte_adv(bsum, bo);
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nb; c0 += kThreads) {
    const int i = c0 + threadIdx.x;
    const uint32_t v = i < nb ? bsum[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, sh, total);
    if (i < nb) bsum[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

// adds the block carries and copies the offsets into the (consumed) counts:
// the scatter's per-key cursors
__global__ __launch_bounds__(kThreads) void k_scan_add(uint32_t* __restrict__ off, uint32_t* __restrict__ cursor,
                                                       long n, const uint32_t* __restrict__ bsum, int nb,
                                                       BatchArg bat) {
  const long bo = batch_bytes(bat);
  if (bo < 0) return;
  off = byte_adv(off, bo);
  cursor = byte_adv(cursor, bo);
  bsum = byte_adv(bsum, bo);
  const long base = (long)blockIdx.x * kScanBlock;
  const uint32_t add = bsum[blockIdx.x];
  for (int j = threadIdx.x; j < kScanBlock; j += kThreads)
    if (base + j < n) {
      const uint32_t v = off[base + j] + add;
      off[base + j] = v;
      cursor[base + j] = v;
    }
  if (blockIdx.x == 0 && threadIdx.x == 0) off[n] = bsum[nb];
}

// Each particle's destination is reserved at its key's cursor (one atomic
// per group of equal keys in the wave; the order inside a key is the order
// in which the groups arrive, which no result depends on: paint sums in
// integers and the readout is per particle).  Every load of a particle
// (key, state, id) is issued before the atomic, and pinned: left to the
// compiler, the state loads follow it and add a third round trip to the
// chain.  A source in lattice order (a first sort, lat_ln >= 0) is walked
// brick by brick (lattice_order), so that a wave's particles share keys.
__global__ void k_scatter(ScatterArgs a) {
  if (a.bat.d) {
    const long bo = batch_bytes(a.bat);
    if (bo < 0) return;
    a.pos = byte_adv(a.pos, bo);
    a.mom = byte_adv(a.mom, bo);
    a.id = byte_adv(a.id, bo);
    a.key = byte_adv(a.key, bo);
    a.cursor = byte_adv(a.cursor, bo);
    a.pos_out = byte_adv(a.pos_out, bo);
    a.mom_out = byte_adv(a.mom_out, bo);
    a.id_out = byte_adv(a.id_out, bo);
  }
  // consecutive blocks of particles on one XCD: their destinations form
  // runs that continue from block to block, and the partial cache lines at
  // the ends of the runs then merge in one L2.  The loop bound is uniform
  // over the block: the whole wave takes part in the key grouping.
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i0 = (long)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x; i0 < a.np; i0 += stride) {
    const long t = i0 + threadIdx.x;
    const bool valid = t < a.np;
    const long tc = valid ? t : a.np - 1;
    const long ic = a.lat_ln >= 0 ? lattice_order(tc, a.lat_ln) : tc;
    const uint32_t key = a.key[ic];
    float x[3], p[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = a.pos[3 * ic + d];
    if (a.mom) {
#pragma unroll
      for (int d = 0; d < 3; ++d) p[d] = a.mom[3 * ic + d];
    }
    const uint32_t id = (a.id_out && a.id) ? a.id[ic] : (uint32_t)ic;
    asm volatile("" : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(p[0]), "+v"(p[1]), "+v"(p[2]));
    const uint32_t d = agg_rank(a.cursor, key, valid);
    if (!valid) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) a.pos_out[3 * (long)d + c] = x[c];
    if (a.mom) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.mom_out[3 * (long)d + c] = p[c];
    }
    if (a.id_out) a.id_out[d] = id;
  }
}

// ---- paint ---------------------------------------------------------------------
// LDS accumulator order of a tile: tile_li (z fastest, z swizzled so that
// the deposits of a wave spread over the banks); the store walks the cells
// in the order of the x-blocked mesh (x%8 fastest), so that its global
// stores are contiguous.  STD writes the plain [x][y][z] layout instead
// (caller-visible meshes).
//
// The tile accumulates in 64-bit fixed point (ds_add_u64): LDS float atomics
// run about 25x slower than integer ones on gfx950 (measured), and integer
// sums are exact and independent of the order of the deposits, so the
// painted mesh is bitwise deterministic.
//  - unit masses: weight * 2^31 per deposit, exact to 2^-31; 2^33 unit
//    deposits fit in one cell;
//  - WT (signed per-particle masses m_p = wts[3 id_p + comp] * k, the
//    adjoint's cotangent channels): the float value w m_p S per deposit,
//    with S = 2^(40 - e) and 2^e > max |m_p| (from *maxbits), so every
//    |deposit| < 2^40 is an integer held exactly and 2^23 of them fit.
struct PaintWeights {
  const uint32_t* id = nullptr;     // sorted particle ids
  const float* wts = nullptr;       // [np][3] in particle-id order
  int comp = 0;                     // < 0: component blockIdx.y, into out + blockIdx.y * out_stride
  long out_stride = 0;
  float k = 1.f;
  const uint32_t* maxbits = nullptr;   // bits of max |wts| (non-negative float)
};

// Threads per paint workgroup: the 64-bit tile accumulator (32 KB of LDS)
// allows four workgroups per CU, and 512 threads each make that the full
// eight waves per SIMD to hide the latency of the range and particle loads.
constexpr int kPaintThreads = 512;
// workgroups of the persistent paint (a multiple of 8)
constexpr int kPaintPersistentGroups = 1024;

template <bool STD, bool WT>
__global__ __launch_bounds__(kPaintThreads) void k_paint(const float* __restrict__ pos, const uint32_t* __restrict__ off,
                                                    TileGeom g, float* __restrict__ out, float scale, float offset,
                                                    PaintWeights pw, BatchArg bat) {
  __shared__ __align__(16) unsigned long long acc[kTileCells];
  __shared__ RangeTable rt;
  {
    const long bo = batch_bytes(bat);
    if (bo < 0) return;
    pos = byte_adv(pos, bo);
    off = byte_adv(off, bo);
    out = byte_adv(out, bo);
  }
  if (WT && pw.comp < 0) {   // uniform: one component per blockIdx.y
    pw.comp = (int)blockIdx.y;
    out += blockIdx.y * pw.out_stride;
  }
  const int TX = g.tx, TY = g.ty, TZ = g.tz, n = g.n;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  int tx, ty, tz;
  tile_coords(tile, g, tx, ty, tz);
  const int ox = tx * TX, oy = ty * TY, oz = tz * TZ;
  {   // zero the accumulator with 16-byte LDS writes
    uint4* a4 = reinterpret_cast<uint4*>(acc);
    for (int c = threadIdx.x; c < (tile_cells(g) >> 1); c += kPaintThreads) a4[c] = make_uint4(0u, 0u, 0u, 0u);
  }
  float S = 1.f;   // WT: fixed-point scale, a power of two
  if (WT) {
    const float mx = __uint_as_float(*pw.maxbits) * fabsf(pw.k);
    if (mx > 0.f && mx < INFINITY) {
      int e;
      frexpf(mx, &e);   // mx < 2^e
      S = ldexpf(1.f, 40 - e);
    }
  }
  build_ranges(rt, off, tx, ty, tz, g);
  const uint32_t total = rt.pre[27];
  // particles per thread whose loads are in flight together (the weighted
  // form has a third dependent load, the weight by id)
  constexpr int kBatch = WT ? 4 : 2;
  for (uint32_t base = 0; base < total; base += kPaintThreads * kBatch) {
    // all range searches (LDS) first, then all loads, so that the kBatch
    // loads of a thread are in flight together; positions past the end are
    // clamped onto the last particle (a valid address) and skipped below
    uint32_t jj[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const uint32_t idx = base + threadIdx.x + u * kPaintThreads;
      jj[u] = range_particle(rt, idx < total ? idx : total - 1);
    }
    float px[kBatch][3];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
#pragma unroll
      for (int d = 0; d < 3; ++d) px[u][d] = pos[3 * (long)jj[u] + d];
    float mp[kBatch];
    if (WT) {
      uint32_t pid[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) pid[u] = pw.id[jj[u]];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) mp[u] = pw.wts[3 * (long)pid[u] + pw.comp] * pw.k;
    }
    // pin the loads here: each particle's use sits in its own branch, and
    // sunk into those branches the loads would run one round trip at a time
#pragma unroll
    for (int u = 0; u < kBatch; ++u) asm volatile("" : "+v"(px[u][0]), "+v"(px[u][1]), "+v"(px[u][2]));
    if (WT) {
#pragma unroll
      for (int u = 0; u < kBatch; ++u) asm volatile("" : "+v"(mp[u]));
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
    if (base + threadIdx.x + u * kPaintThreads >= total) continue;
    int ix, iy, iz;
    float fx, fy, fz;
    cic_base(px[u][0], n, ix, fx);
    cic_base(px[u][1], n, iy, fy);
    cic_base(px[u][2], n, iz, fz);
    // local base cell in [-1, T-1] (-1: the particle sits in the lower neighbour)
    int lx = (ix - ox) & (n - 1), ly = (iy - oy) & (n - 1), lz = (iz - oz) & (n - 1);
    if (lx > TX) lx -= n;
    if (ly > TY) ly -= n;
    if (lz > TZ) lz -= n;
    const float wx[2] = {1.f - fx, fx}, wy[2] = {1.f - fy, fy}, wz[2] = {1.f - fz, fz};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int cx = lx + a;
      if (cx < 0 || cx >= TX) continue;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int cy = ly + b;
        if (cy < 0 || cy >= TY) continue;
        const float wxy = wx[a] * wy[b];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int cz = lz + c;
          if (cz < 0 || cz >= TZ) continue;
          unsigned long long q;
          if (WT) {
            q = (unsigned long long)__float2ll_rn(wxy * wz[c] * mp[u] * S);
          } else {
            // w <= 1, so w * 2^31 <= 2^31 fits in 32 bits
            q = (unsigned long long)(uint32_t)(wxy * wz[c] * 2147483648.0f);
          }
          atomicAdd(&acc[tile_li(cx, cy, cz, g)], q);
        }
      }
    }
    }
  }
  __syncthreads();
  auto cell_value = [&](int cx, int cy, int cz) {
    const unsigned long long v = acc[tile_li(cx, cy, cz, g)];
    const double rho = WT ? (double)(long long)v / (double)S : (double)v * 0x1p-31;
    return (float)(rho * (double)scale + (double)offset);
  };
  if (!STD && (TX & 7) == 0) {
    // whole 8-cell x runs: four consecutive x of one (y, z) per thread, one
    // 16-byte store each (the walk's x%8 is fastest, so c4 * 4 starts at
    // x%8 = 0 or 4 and the address is 16-byte aligned)
    for (int c4 = threadIdx.x; c4 < (store_walk_len(g) >> 2); c4 += kPaintThreads) {
      int cx, cy, cz;
      store_walk(c4 << 2, g, cx, cy, cz);
      const float4 v = make_float4(cell_value(cx, cy, cz), cell_value(cx + 1, cy, cz), cell_value(cx + 2, cy, cz),
                                   cell_value(cx + 3, cy, cz));
      *reinterpret_cast<float4*>(out + blk_real(ox + cx, oy + cy, oz + cz, n)) = v;
    }
    return;
  }
  for (int c = threadIdx.x; c < store_walk_len(g); c += kPaintThreads) {
    int cx, cy, cz;
    store_walk(c, g, cx, cy, cz);
    if (cx >= TX) continue;
    const int x = ox + cx, y = oy + cy, z = oz + cz;
    const unsigned long long v = acc[tile_li(cx, cy, cz, g)];
    const double rho = WT ? (double)(long long)v / (double)S : (double)v * 0x1p-31;
    out[STD ? ((long)x * n + y) * n + z : blk_real(x, y, z, n)] = (float)(rho * (double)scale + (double)offset);
  }
}

// Persistent form of the plain paint (unit masses, x-blocked mesh, tiles at
// least 8 cells wide along x): each workgroup walks its own run of tiles and
// overlaps the global loads of the next tile with the work on the current
// one.  While it deposits tile k, wave 0 has the bin offsets of tile k+1 in
// flight; while it stores tile k (and clears the accumulator cell by cell as
// it reads it), every thread has its first particles of tile k+1 in flight.
// A one-tile-per-workgroup launch waits for both round trips on every tile.
// The cells and sums are those of k_paint; the tiles are 16^3 cells.  STD
// stores the plain [x][y][z] layout (caller-visible meshes), four
// consecutive z per 16-byte store.
template <bool STD>
__global__ __launch_bounds__(kPaintThreads) void k_paint_p(const float* __restrict__ pos,
                                                           const uint32_t* __restrict__ off, TileGeom g,
                                                           float* __restrict__ out, float scale, float offset,
                                                           BatchArg bat) {
  __shared__ __align__(16) unsigned long long acc[kTileCells];
  __shared__ RangeTable rt[2];
  {
    const long bo = batch_bytes(bat);
    if (bo < 0) return;
    pos = byte_adv(pos, bo);
    off = byte_adv(off, bo);
    out = byte_adv(out, bo);
  }
  const int n = g.n;
  // tiles: XCD x (= blockIdx.x % 8) takes the contiguous eighth of the
  // tiles [x cnt, (x + 1) cnt) and its nslot workgroups take every nslot-th
  // of them (gridDim.x is a multiple of 8, at most ntiles)
  const int cnt = g.ntiles >> 3, nslot = (int)gridDim.x >> 3;
  const int c0 = ((int)blockIdx.x & 7) * cnt;
  int k = (int)blockIdx.x >> 3;
  if (k >= cnt) return;   // uniform over the workgroup
  {
    uint4* a4 = reinterpret_cast<uint4*>(acc);
    for (int c = threadIdx.x; c < (tile_cells(g) >> 1); c += kPaintThreads) a4[c] = make_uint4(0u, 0u, 0u, 0u);
  }
  constexpr int kBatch = 2;
  constexpr int kRound = kPaintThreads * kBatch;
  auto coords = [&](int tile, int& tx, int& ty, int& tz) { tile_coords(tile, g, tx, ty, tz); };
  // particles of a tile: indices past the end are clamped onto its last
  // particle (particle 0 for an empty tile) and skipped at deposit time.
  // The loads are unconditional, so that every path leaves the same loads
  // in flight and the waits before the deposits count only these.
  auto issue = [&](const RangeTable& t, uint32_t total, uint32_t base, float (&px)[kBatch][3]) {
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const uint32_t idx = base + threadIdx.x + u * kPaintThreads;
      const uint32_t j = total ? range_particle(t, idx < total ? idx : total - 1) : 0u;
#pragma unroll
      for (int d = 0; d < 3; ++d) px[u][d] = pos[3 * (long)j + d];
    }
  };
  auto deposit = [&](const float (&px)[kBatch][3], uint32_t total, uint32_t base, int ox, int oy, int oz) {
    const int TX = g.tx, TY = g.ty, TZ = g.tz;
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (base + threadIdx.x + u * kPaintThreads >= total) continue;
      int ix, iy, iz;
      float fx, fy, fz;
      cic_base(px[u][0], n, ix, fx);
      cic_base(px[u][1], n, iy, fy);
      cic_base(px[u][2], n, iz, fz);
      int lx = (ix - ox) & (n - 1), ly = (iy - oy) & (n - 1), lz = (iz - oz) & (n - 1);
      if (lx > TX) lx -= n;
      if (ly > TY) ly -= n;
      if (lz > TZ) lz -= n;
      const float wx[2] = {1.f - fx, fx}, wy[2] = {1.f - fy, fy}, wz[2] = {1.f - fz, fz};
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int cx = lx + a;
        if (cx < 0 || cx >= TX) continue;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int cy = ly + b;
          if (cy < 0 || cy >= TY) continue;
          const float wxy = wx[a] * wy[b];
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const int cz = lz + c;
            if (cz < 0 || cz >= TZ) continue;
            atomicAdd(&acc[tile_li(cx, cy, cz, g)], (unsigned long long)(uint32_t)(wxy * wz[c] * 2147483648.0f));
          }
        }
      }
    }
  };

  int cur = 0;
  int tx, ty, tz;
  coords(c0 + k, tx, ty, tz);
  build_ranges(rt[0], off, tx, ty, tz, g);
  uint32_t total = rt[0].pre[27];
  float px[kBatch][3];
  issue(rt[0], total, 0, px);
  for (;;) {
    const int kn = k + nslot;
    const bool more = kn < cnt;   // uniform
    // the next tile's bin offsets, loaded by every lane (lane r of each wave
    // reads range min(r, 26); the last tile reloads its own), used by wave 0
    int nx, ny, nz;
    coords(c0 + (more ? kn : k), nx, ny, nz);
    uint32_t b0, b1;
    {
      const int r = (int)(threadIdx.x & 63);
      range_loads(off, nx, ny, nz, g, r < 27 ? r : 26, b0, b1);
    }
    // deposits of tile k: the first round from the particles already loaded
    const int ox = tx * g.tx, oy = ty * g.ty, oz = tz * g.tz;
#pragma unroll
    for (int u = 0; u < kBatch; ++u) asm volatile("" : "+v"(px[u][0]), "+v"(px[u][1]), "+v"(px[u][2]));
    deposit(px, total, 0, ox, oy, oz);
    for (uint32_t base = kRound; base < total; base += kRound) {   // heavy tiles
      issue(rt[cur], total, base, px);
#pragma unroll
      for (int u = 0; u < kBatch; ++u) asm volatile("" : "+v"(px[u][0]), "+v"(px[u][1]), "+v"(px[u][2]));
      deposit(px, total, base, ox, oy, oz);
    }
    if (more && threadIdx.x < 64) range_publish(rt[cur ^ 1], threadIdx.x, b0, b1);
    __syncthreads();   // deposits done, the next table published
    // (after the last tile: particle 0, unused)
    const uint32_t ntotal = more ? rt[cur ^ 1].pre[27] : 0u;
    issue(rt[cur ^ 1], ntotal, 0, px);
    // store tile k four cells at a time (16-byte stores, x%8 fastest) and
    // clear each cell as it is read: a fixed count per thread, so that the
    // wait for the next particles need not wait for these stores
    static_assert((kTileCells / 4) % kPaintThreads == 0, "whole store rounds");
#pragma unroll
    for (int r4 = 0; r4 < kTileCells / 4 / kPaintThreads; ++r4) {
      const int c4 = threadIdx.x + r4 * kPaintThreads;
      // x-blocked: four consecutive x of one (y, z) in the walk's order;
      // STD ([x][y][z], caller-visible): four consecutive z of one (x, y)
      int cx, cy, cz;
      if (STD) {
        cz = (c4 & 3) << 2;
        cy = (c4 >> 2) & 15;
        cx = c4 >> 6;
      } else {
        store_walk(c4 << 2, g, cx, cy, cz);
      }
      float v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        unsigned long long& cell = acc[STD ? tile_li(cx, cy, cz + i, g) : tile_li(cx + i, cy, cz, g)];
        v[i] = (float)((double)cell * 0x1p-31 * (double)scale + (double)offset);
        cell = 0ull;
      }
      const long o = STD ? ((long)(ox + cx) * n + (oy + cy)) * n + (oz + cz) : blk_real(ox + cx, oy + cy, oz + cz, n);
      *reinterpret_cast<float4*>(out + o) = make_float4(v[0], v[1], v[2], v[3]);
    }
    if (!more) break;
    __syncthreads();   // the accumulator is clear and the old table free
    k = kn;
    cur ^= 1;
    total = ntotal;
    tx = nx;
    ty = ny;
    tz = nz;
  }
}

// ---- readout + kick + drift ---------------------------------------------------------
// One tile-sorted particle per thread: CIC gather of the 8 corners from the
// interleaved force mesh (one 12-byte load per corner; sorted neighbours
// share cache lines), kicks, drift, wrap, and the sort key of the new
// position, counted per key.  All loads are issued before any is used
// (every lane computes, on a clamped index, and only the stores are
// predicated).  The counts are added per group of equal keys in the wave
// (agg_count: one global atomic per group, not waited for); the scatter
// reserves the destinations.  Nothing waits on a workgroup barrier.  (Two
// particles per thread measured slower: the tile span per wave grows in
// voids.)
constexpr int kReadoutPPT = 1;

// Instantiations by the flags they keep (the others compile away, fewer
// registers and branches): VAR 0, a single simulation's steps and force
// evaluations (no batch descriptors, no LPT frame, no RO_TO_ALT); VAR 1, the
// batched step (descriptors, RO_KICK, RO_DRIFT, RO_KEYS, RO_TO_ALT and the
// descriptors' checkpoints only); VAR 2, everything (the LPT frame).
template <int VAR>
__global__ __launch_bounds__(kThreads) void k_readout(ReadoutArgs a) {
  constexpr bool EXT = VAR != 0;
  constexpr int kKeep = VAR == 0 ? ~(RO_COLA | RO_COLA_OUT | RO_TO_ALT)
                                 : (VAR == 1 ? (RO_KICK | RO_DRIFT | RO_KEYS | RO_TO_ALT | RO_CKPT) : ~0);
  constexpr int PPT = kReadoutPPT;
  const TileGeom& g = a.g;
  const int n = g.n;
  const long chunk = xcd_tile(blockIdx.x, gridDim.x);
  const long j0 = chunk * (long)(kThreads * PPT);
  const bool keys = (a.flags & RO_KEYS) != 0;
  float kick_a = a.kick_a, kick_b = a.kick_b, drift = a.drift;
  float *ckpt_x = a.ckpt_x, *ckpt_p = a.ckpt_p;
  a.flags &= kKeep;
  if (EXT && a.bat.d) {   // uniform: this block's member, its factors and checkpoints
    const long bo = batch_bytes(a.bat);
    if (bo < 0) return;
    const pm_req_desc& dsc = a.bat.d[blockIdx.z];
    a.pos = byte_adv(a.pos, bo);
    a.mom = byte_adv(a.mom, bo);
    a.id = byte_adv(a.id, bo);
    a.fi = byte_adv(a.fi, bo);
    a.key_out = byte_adv(a.key_out, bo);
    a.count = byte_adv(a.count, bo);
    a.pos_alt = byte_adv(a.pos_alt, bo);
    a.mom_alt = byte_adv(a.mom_alt, bo);
    a.id_alt = byte_adv(a.id_alt, bo);
    kick_a = dsc.kick_close;
    kick_b = dsc.kick_open;
    drift = dsc.drift;
    ckpt_x = dsc.ckpt_x;
    ckpt_p = dsc.ckpt_p;
    a.flags = ((a.flags & ~RO_CKPT) | ((dsc.flags & PM_REQ_CKPT) && ckpt_x && ckpt_p ? RO_CKPT : 0)) & kKeep;
  }
  float4 cola = a.cola;
  if (a.steps) {   // uniform: the factors of step *step_i
    const uint32_t si = *a.step_i;
    const float4 f = a.steps[si];
    kick_a = f.x;
    kick_b = f.y;
    drift = f.z;
    if (VAR == 2 && a.cola_steps) cola = a.cola_steps[si];
    if (a.flags & RO_CKPT) {
      ckpt_x = *a.ckpt_base + 2 * (long)si * a.ckpt_stride;
      ckpt_p = ckpt_x + a.ckpt_stride;
    }
  }
  long jj[PPT];
  bool valid[PPT];
  float x[PPT][3], p[PPT][3];
  uint32_t id[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    jj[u] = j0 + threadIdx.x + u * kThreads;
    valid[u] = jj[u] < a.np;
    const long jc = valid[u] ? jj[u] : a.np - 1;
    // position and momentum as one 12-byte load each
#pragma unroll
    for (int d = 0; d < 3; ++d) x[u][d] = a.pos[3 * jc + d];
#pragma unroll
    for (int d = 0; d < 3; ++d) p[u][d] = 0.f;
    if (a.mom) {
#pragma unroll
      for (int d = 0; d < 3; ++d) p[u][d] = a.mom[3 * jc + d];
    }
    // ids are needed only for writes by id (not on ordinary steps)
    id[u] = (a.id && (a.flags & (RO_FORCE_BYID | RO_XP_BYID | RO_CKPT | RO_TO_ALT | RO_COLA))) ? a.id[jc]
                                                                                        : (uint32_t)jc;
  }
  // all 8 x PPT corner loads first, pinned, then the weighted sums
  float cv[PPT][8][3], wgt[PPT][8];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    int ix, iy, iz;
    float fx, fy, fz;
    cic_base(x[u][0], n, ix, fx);
    cic_base(x[u][1], n, iy, fy);
    cic_base(x[u][2], n, iz, fz);
    const int jx = (ix + 1) & (n - 1), jy = (iy + 1) & (n - 1), jz = (iz + 1) & (n - 1);
    // corner (x, y, z) at fi + 3 * blk_real(x, y, z): x and x+1 of one block
    // are adjacent 12-byte cells
    const int xs[2] = {ix, jx}, ys[2] = {iy, jy}, zs[2] = {iz, jz};
    const float wx[2] = {1.f - fx, fx}, wy[2] = {1.f - fy, fy}, wz[2] = {1.f - fz, fz};
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) {
      const int e = c8 & 1, b = (c8 >> 1) & 1, c = c8 >> 2;
      const float* cp = a.fi + 3 * blk_real(xs[e], ys[b], zs[c], n);
#pragma unroll
      for (int d = 0; d < 3; ++d) cv[u][c8][d] = cp[d];
      wgt[u][c8] = wx[e] * wy[b] * wz[c];
    }
  }
#pragma unroll
  for (int u = 0; u < PPT; ++u)
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) asm volatile("" : "+v"(cv[u][c8][0]), "+v"(cv[u][c8][1]), "+v"(cv[u][c8][2]));
  float F[PPT][3];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
#pragma unroll
    for (int d = 0; d < 3; ++d) F[u][d] = 0.f;
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8)
#pragma unroll
      for (int d = 0; d < 3; ++d) F[u][d] += wgt[u][c8] * cv[u][c8][d];
  }
  const float nf = (float)n;
  // LPT frame: the fields of the particle (by id; loaded after the corner
  // gathers so that those go first)
  float ps1[PPT][3], ps2[PPT][3];
  if (a.flags & RO_COLA) {
#pragma unroll
    for (int u = 0; u < PPT; ++u)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        ps1[u][d] = a.psi1[3 * (long)id[u] + d];
        ps2[u][d] = a.psi2[3 * (long)id[u] + d];
      }
  }
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const long j = jj[u];
    if (valid[u] && (a.flags & RO_FORCE_BYID)) {
#pragma unroll
      for (int d = 0; d < 3; ++d) a.force_out[3 * (long)id[u] + d] = F[u][d];
    }
    if (a.flags & RO_COLA) {   // residual force from the LPT trajectory
#pragma unroll
      for (int d = 0; d < 3; ++d) F[u][d] -= cola.x * ps1[u][d] + cola.y * ps2[u][d];
    }
    if (a.flags & RO_KICK) {
#pragma unroll
      for (int d = 0; d < 3; ++d) p[u][d] += F[u][d] * kick_a;
    }
    if (valid[u] && (a.flags & RO_CKPT)) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        ckpt_x[3 * (long)id[u] + d] = x[u][d];
        ckpt_p[3 * (long)id[u] + d] = p[u][d];
      }
    }
    if (a.flags & RO_KICK) {
#pragma unroll
      for (int d = 0; d < 3; ++d) p[u][d] += F[u][d] * kick_b;
    }
    if (a.flags & RO_DRIFT) {
      if (a.flags & RO_COLA) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
          x[u][d] = wrap_pos(x[u][d] + p[u][d] * drift + cola.z * ps1[u][d] + cola.w * ps2[u][d], nf);
      } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) x[u][d] = wrap_pos(x[u][d] + p[u][d] * drift, nf);
      }
    }
    if (!valid[u]) continue;
    if (a.flags & RO_WRITE_SORTED) {
#pragma unroll
      for (int d = 0; d < 3; ++d) a.pos[3 * j + d] = x[u][d];
      if (a.mom) {
#pragma unroll
        for (int d = 0; d < 3; ++d) a.mom[3 * j + d] = p[u][d];
      }
    }
    if (a.flags & RO_TO_ALT) {
#pragma unroll
      for (int d = 0; d < 3; ++d) a.pos_alt[3 * j + d] = x[u][d];
#pragma unroll
      for (int d = 0; d < 3; ++d) a.mom_alt[3 * j + d] = p[u][d];
      a.id_alt[j] = id[u];
    }
    if (a.flags & RO_XP_BYID) {
#pragma unroll
      for (int d = 0; d < 3; ++d) a.pos_out[3 * (long)id[u] + d] = x[u][d];
      if (a.flags & RO_COLA_OUT) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
          a.mom_out[3 * (long)id[u] + d] = p[u][d] + a.cola_out.x * ps1[u][d] + a.cola_out.y * ps2[u][d];
      } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) a.mom_out[3 * (long)id[u] + d] = p[u][d];
      }
    }
  }
  if (!keys) return;
  // sort key of the new position, counted: the wave's lanes with equal keys
  // are grouped with ballots and each group adds its size with one global
  // atomic (a sorted wave holds a few keys)
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    uint32_t key = 0u;
    if (valid[u]) {
      int kx, ky, kz;
      float t;
      cic_base(x[u][0], n, kx, t);
      cic_base(x[u][1], n, ky, t);
      cic_base(x[u][2], n, kz, t);
      key = tile_key(kx, ky, kz, g);
      a.key_out[jj[u]] = key;
    }
    agg_count(a.count, key, valid[u]);
  }
}

__global__ void k_frame_shift(float* __restrict__ mom, const uint32_t* __restrict__ id,
                              const float* __restrict__ psi1, const float* __restrict__ psi2, long np, float u1,
                              float u2) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < np; j += stride) {
    const long i = id[j];
#pragma unroll
    for (int d = 0; d < 3; ++d) mom[3 * j + d] += u1 * psi1[3 * i + d] + u2 * psi2[3 * i + d];
  }
}

__global__ void k_step_inc(uint32_t* ctr) {
  if (threadIdx.x == 0) atomicAdd(ctr, 1u);
}

// elementwise kick + drift with a given per-particle force (first half of a
// standalone KDK step)
__global__ void k_kick_drift(float* __restrict__ pos, float* __restrict__ mom, const float* __restrict__ f,
                             long np, float kick, float drift, float nmesh) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float p = mom[3 * i + d] + f[3 * i + d] * kick;
      mom[3 * i + d] = p;
      pos[3 * i + d] = wrap_pos(pos[3 * i + d] + p * drift, nmesh);
    }
  }
}

// ---- power spectrum --------------------------------------------------------------
constexpr int kPowerBins = 512;
constexpr int kPowerBlocks = 1024;

__global__ __launch_bounds__(kThreads) void k_power_bins(PowerArgs a) {
  __shared__ double sw[kPowerBins], sk[kPowerBins], sp[kPowerBins];
  for (int i = threadIdx.x; i < a.n_bins; i += kThreads) sw[i] = sk[i] = sp[i] = 0.0;
  __syncthreads();
  const int n = a.n, h = n / 2;
  const int ln = __builtin_ctz(n), lh = ln - 1;
  const long nmain = (long)n * n * h;
  const long ntot = nmain + (long)n * n;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < ntot; i += stride) {
    int kx, ky, kz;
    float2 v;
    if (i < nmain) {   // x-blocked c[kx/8][ky][kz][kx%8]; n, h = n/2 powers of two
      const long r = i >> 3;
      kz = (int)(r & (h - 1));
      ky = (int)((r >> lh) & (n - 1));
      kx = (int)((r >> (lh + ln)) << 3) + (int)(i & 7);
      v = a.c[i];
    } else {           // q[kx/8][ky][kx%8]
      const long j = i - nmain, r = j >> 3;
      ky = (int)(r & (n - 1));
      kx = (int)((r >> ln) << 3) + (int)(j & 7);
      kz = h;
      v = a.q[j];
    }
    const int fx = kx < h ? kx : kx - n, fy = ky < h ? ky : ky - n;
    if (a.n_max > 0 && (abs(fx) >= a.n_max || abs(fy) >= a.n_max || kz >= a.n_max)) continue;
    const int n2 = fx * fx + fy * fy + kz * kz;
    const double mag = sqrt((double)n2);
    const int bin = (int)floor(mag + 0.5);
    if (bin < 1 || bin > a.n_bins) continue;
    const double w = (kz == 0 || kz == h) ? 1.0 : 2.0;
    double p = (double)v.x * v.x + (double)v.y * v.y;
    if (a.deconv) {
      const double win = (double)a.wxy[kx] * a.wxy[ky] * a.wz[kz];
      p /= win * win;
    }
    atomicAdd(&sw[bin - 1], w);
    atomicAdd(&sk[bin - 1], w * mag);
    atomicAdd(&sp[bin - 1], w * p);
  }
  __syncthreads();
  double* out = a.partial + (long)blockIdx.x * 3 * a.n_bins;
  for (int i = threadIdx.x; i < a.n_bins; i += kThreads) {
    out[i] = sw[i];
    out[a.n_bins + i] = sk[i];
    out[2 * a.n_bins + i] = sp[i];
  }
}

__global__ void k_power_reduce(const double* __restrict__ partial, int nblocks, int n_bins, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n_bins) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[(long)b * 3 * n_bins + i];
  out[i] = s;
}

// [n][n][n/2] + Nyquist plane  <->  [n][n][n/2+1] (numpy rfftn layout)
__global__ void k_spec_pack(const float2* __restrict__ c, const float2* __restrict__ q, float2* __restrict__ out,
                            int n, float scale, int to_numpy) {
  const int h = n / 2;
  const long total = (long)n * n * (h + 1);
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int kz = (int)(i % (h + 1));
    const long line = i / (h + 1);
    const int kx = (int)(line / n), ky = (int)(line % n);
    const long ec = blk_spec(kx, ky, kz < h ? kz : 0, n), eq = blk_nyq(kx, ky, n);
    if (to_numpy) {
      const float2 v = kz < h ? c[ec] : q[eq];
      out[i] = make_float2(v.x * scale, v.y * scale);
    } else {
      float2* dst = kz < h ? const_cast<float2*>(c) + ec : const_cast<float2*>(q) + eq;
      const float2 v = out[i];
      *dst = make_float2(v.x * scale, v.y * scale);
    }
  }
}

// bits of max_i |v_i| (non-negative floats order like their bit patterns);
// NaNs are ignored by fmaxf
// (16-byte loads; one atomic per workgroup: the atomics on the one word
// are serialized, so their number, not the loads, set the time of a small
// launch)
__global__ __launch_bounds__(kThreads) void k_absmax(const float* __restrict__ v, long n, uint32_t* __restrict__ bits) {
  __shared__ float wm[kThreads / 64];
  float m = 0.f;
  const long stride = (long)gridDim.x * blockDim.x;
  const long first = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n4 = (reinterpret_cast<uintptr_t>(v) & 15) ? 0 : n >> 2;
  const float4* v4 = reinterpret_cast<const float4*>(v);
  for (long i = first; i < n4; i += stride) {
    const float4 t = v4[i];
    m = fmaxf(m, fmaxf(fmaxf(fabsf(t.x), fabsf(t.y)), fmaxf(fabsf(t.z), fabsf(t.w))));
  }
  for (long i = 4 * n4 + first; i < n; i += stride) m = fmaxf(m, fabsf(v[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) m = fmaxf(m, wm[w]);
    atomicMax(bits, __float_as_uint(m));
  }
}

// plain [x][y][z] <-> x-blocked real mesh (caller-visible buffers); the
// output index runs over threads so that the stores are contiguous
__global__ void k_relayout(const float* __restrict__ in, float* __restrict__ out, int ln, int to_blocked) {
  const long n3 = 1L << (3 * ln);
  const long stride = (long)gridDim.x * blockDim.x;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n3; e += stride) {
    int x, y, z;
    if (to_blocked) {
      blk_real_xyz(e, ln, x, y, z);
      out[e] = in[((((long)x << ln) + y) << ln) + z];
    } else {
      z = (int)(e & ((1L << ln) - 1));
      y = (int)((e >> ln) & ((1L << ln) - 1));
      x = (int)(e >> (2 * ln));
      out[e] = in[blk_real(x, y, z, 1 << ln)];
    }
  }
}

__global__ void k_scale(float* __restrict__ p, long n, float s) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] *= s;
}

inline int grid_for(long n, int per = kThreads, int cap = 65536) {
  long g = (n + per - 1) / per;
  if (g < 1) g = 1;
  return (int)(g > cap ? cap : g);
}

}  // namespace

TileGeom make_tile_geom(int n) {
  TileGeom g;
  g.n = n;
  g.tx = g.ty = g.tz = n / 2 < 16 ? n / 2 : 16;
  g.ntx = n / g.tx;
  g.nty = n / g.ty;
  g.ntz = n / g.tz;
  g.ntiles = g.ntx * g.nty * g.ntz;
  g.lx = __builtin_ctz(g.tx);
  g.ly = __builtin_ctz(g.ty);
  g.lz = __builtin_ctz(g.tz);
  g.lnx = __builtin_ctz(g.ntx);
  g.lny = __builtin_ctz(g.nty);
  g.lnz = __builtin_ctz(g.ntz);
  return g;
}

void launch_noise(uint64_t seed, int n_side, float* out, bool blocked, hipStream_t s) {
  const long n3 = (long)n_side * n_side * n_side;
  hipLaunchKernelGGL(k_noise, dim3(grid_for(n3)), dim3(kThreads), 0, s, seed, n3, __builtin_ctz(n_side),
                     blocked ? 1 : 0, out);
}

void launch_relayout(const float* in, float* out, int n_side, bool to_blocked, hipStream_t s) {
  const long n3 = (long)n_side * n_side * n_side;
  hipLaunchKernelGGL(k_relayout, dim3(grid_for(n3)), dim3(kThreads), 0, s, in, out, __builtin_ctz(n_side),
                     to_blocked ? 1 : 0);
}

void launch_lpt_delta2(float* const* phi6, long n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_lpt_delta2, dim3(grid_for(n)), dim3(kThreads), 0, s, phi6[0], phi6[1], phi6[2], phi6[3],
                     phi6[4], phi6[5], n, out);
}

void launch_lpt_particles(const LptParticleArgs& a, hipStream_t s) {
  const long n3 = (long)a.np * a.np * a.np;
  hipLaunchKernelGGL(k_lpt_particles, dim3(grid_for(n3)), dim3(kThreads), 0, s, a);
}

void launch_fill_u32(uint32_t* p, long n, uint32_t v, hipStream_t s, const BatchArg& bat) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n), 1, bat.n), dim3(kThreads), 0, s, p, n, v, bat);
}

void launch_keys(const float* pos, long np, const TileGeom& g, uint32_t* key, uint32_t* count,
                 hipStream_t s, int lat_ln) {
  const int grid = (int)((np + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_keys, dim3(grid), dim3(kThreads), 0, s, pos, np, g, key, count, lat_ln);
}

long scan_scratch_words(long n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

void launch_scan(uint32_t* count, long n, uint32_t* off, uint32_t* bsum, hipStream_t s, const BatchArg& bat) {
  const int nb = (int)((n + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(k_scan_local, dim3(nb, 1, bat.n), dim3(kThreads), 0, s, count, n, off, bsum, bat);
  hipLaunchKernelGGL(k_scan_top, dim3(1, 1, bat.n), dim3(kThreads), 0, s, bsum, nb, bat);
  hipLaunchKernelGGL(k_scan_add, dim3(nb, 1, bat.n), dim3(kThreads), 0, s, off, count, n, bsum, nb, bat);
}

void launch_scatter(const ScatterArgs& a, hipStream_t s) {
  // one particle per thread: the key -> cursor -> store chain of each
  // particle is latency bound, so many short waves overlap it best
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(a.np, kThreads, 1 << 30), 1, a.bat.n), dim3(kThreads), 0, s, a);
}

void launch_paint(const float* pos_sorted, const uint32_t* off, const TileGeom& g, float* out, float scale,
                  float offset, bool std_layout, hipStream_t s, const BatchArg& bat) {
  const PaintWeights pw;
  if (g.tx * g.ty * g.tz == kTileCells && g.ntiles >= 8) {
    // persistent: up to four workgroups per CU of 256 CUs, a multiple of 8
    const int nwg = g.ntiles < kPaintPersistentGroups ? g.ntiles : kPaintPersistentGroups;
    if (std_layout)
      hipLaunchKernelGGL(k_paint_p<true>, dim3(nwg, 1, bat.n), dim3(kPaintThreads), 0, s, pos_sorted, off, g, out,
                         scale, offset, bat);
    else
      hipLaunchKernelGGL(k_paint_p<false>, dim3(nwg, 1, bat.n), dim3(kPaintThreads), 0, s, pos_sorted, off, g, out,
                         scale, offset, bat);
    return;
  }
  const dim3 grid(g.ntiles, 1, bat.n);
  if (std_layout)
    hipLaunchKernelGGL((k_paint<true, false>), grid, dim3(kPaintThreads), 0, s, pos_sorted, off, g, out, scale,
                       offset, pw, bat);
  else
    hipLaunchKernelGGL((k_paint<false, false>), grid, dim3(kPaintThreads), 0, s, pos_sorted, off, g, out,
                       scale, offset, pw, bat);
}

void launch_absmax(const float* v, long n, uint32_t* bits, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kThreads), 0, s, bits, 1L, 0u, BatchArg());
  // at least 64 elements per thread, at most 1024 workgroups (atomics)
  hipLaunchKernelGGL(k_absmax, dim3(grid_for(n, kThreads * 64, 1024)), dim3(kThreads), 0, s, v, n, bits);
}

void launch_paint_weighted(const float* pos_sorted, const uint32_t* id_sorted, const uint32_t* off, const TileGeom& g,
                           const float* wts, int comp, float k, const uint32_t* maxbits, float* out, hipStream_t s,
                           long out_stride) {
  PaintWeights pw;
  pw.id = id_sorted;
  pw.wts = wts;
  pw.comp = comp;
  pw.out_stride = out_stride;
  pw.k = k;
  pw.maxbits = maxbits;
  hipLaunchKernelGGL((k_paint<false, true>), dim3(g.ntiles, comp < 0 ? 3 : 1), dim3(kPaintThreads), 0, s, pos_sorted,
                     off, g, out, 1.f, 0.f, pw, BatchArg());
}

void launch_readout(const ReadoutArgs& a, hipStream_t s) {
  const long per = (long)kThreads * kReadoutPPT;
  const int grid = (int)((a.np + per - 1) / per);
  const int batched = RO_KICK | RO_DRIFT | RO_KEYS | RO_TO_ALT | RO_CKPT;
  if (a.bat.d && !(a.flags & ~batched))
    hipLaunchKernelGGL(k_readout<1>, dim3(grid, 1, a.bat.n), dim3(kThreads), 0, s, a);
  else if (a.bat.d || (a.flags & (RO_COLA | RO_COLA_OUT | RO_TO_ALT)))
    hipLaunchKernelGGL(k_readout<2>, dim3(grid, 1, a.bat.n), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_readout<0>, dim3(grid), dim3(kThreads), 0, s, a);
}

void launch_frame_shift(float* mom, const uint32_t* id, const float* psi1, const float* psi2, long np, float u1,
                        float u2, hipStream_t s) {
  hipLaunchKernelGGL(k_frame_shift, dim3(grid_for(np)), dim3(kThreads), 0, s, mom, id, psi1, psi2, np, u1, u2);
}

void launch_step_inc(uint32_t* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, s, ctr);
}

void launch_kick_drift(float* pos, float* mom, const float* f, long np, float kick, float drift, float nmesh,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_kick_drift, dim3(grid_for(np)), dim3(kThreads), 0, s, pos, mom, f, np, kick, drift, nmesh);
}

void launch_spec_to_numpy(const float2* c, const float2* q, float2* out, int n, float scale, hipStream_t s) {
  const long total = (long)n * n * (n / 2 + 1);
  hipLaunchKernelGGL(k_spec_pack, dim3(grid_for(total)), dim3(kThreads), 0, s, c, q, out, n, scale, 1);
}

void launch_spec_from_numpy(const float2* in, float2* c, float2* q, int n, float scale, hipStream_t s) {
  const long total = (long)n * n * (n / 2 + 1);
  hipLaunchKernelGGL(k_spec_pack, dim3(grid_for(total)), dim3(kThreads), 0, s, c, q, const_cast<float2*>(in), n,
                     scale, 0);
}

void launch_scale(float* p, long n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(kThreads), 0, s, p, n, v);
}

int power_max_bins() { return kPowerBins; }
long power_partial_doubles(int n_bins) { return (long)kPowerBlocks * 3 * n_bins; }

void launch_power(const PowerArgs& a, double* out3, hipStream_t s) {
  hipLaunchKernelGGL(k_power_bins, dim3(kPowerBlocks), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(k_power_reduce, dim3((3 * a.n_bins + 255) / 256), dim3(256), 0, s, a.partial, kPowerBlocks,
                     a.n_bins, out3);
}

}  // namespace pmk
