// C-ABI entry points of the PM library (declared in include/pm.h): config
// validation, workspace layout, host float64 tables and the orchestration of
// the HIP kernels for painting, force, KDK steps, full runs, initial
// conditions and power spectra.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cosmo.h"
#include "particles.h"
#include "pyramid.h"
#include "recon.h"
#include "pm.h"
#include "pm_internal.h"

using pmk::Field;
using pmk::FftTables;

static_assert(sizeof(pm_req_desc) == 48, "pm_req_desc is 48 bytes in the ABI");

namespace {

// Host-side roctx range around the enqueueing of one phase of the path (a
// KDK step, the initial conditions, a reverse step): rocprofv3
// --marker-trace shows them beside the kernels they launched.
struct Range {
  explicit Range(const char* what) { roctxRangePushA(what); }
  Range(const char* what, int i) {
    char buf[48];
    std::snprintf(buf, sizeof(buf), "%s %d", what, i);
    roctxRangePushA(buf);
  }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

constexpr double kPi = 3.14159265358979323846;
constexpr size_t kAlign = 256;
constexpr int kMaxSteps = 65536;   // steps per run (the device step table)

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }

size_t field_bytes(long n) { return align_up((size_t)n * n * n * 4) + align_up((size_t)n * n * 8); }

size_t fft_table_bytes(long n) {
  return align_up(n * 8) + align_up(n / 2 * 8) + 4 * align_up(n * 4) + 4 * align_up((n / 2 + 1) * 4);
}

pmk::TileGeom make_tiles(int n) { return pmk::make_tile_geom(n); }

// Byte layout of the workspace (offsets from its base).
struct Layout {
  size_t tab_mesh = 0, tab_lat = 0, pk_lat = 0;
  size_t mesh[3] = {0, 0, 0};
  size_t force_i = 0;
  size_t pos_s[2] = {0, 0}, mom_s[2] = {0, 0}, id_s[2] = {0, 0};
  size_t key = 0;
  size_t count = 0, off = 0, bsum = 0;
  size_t pw_partial = 0, pw_out = 0;
  size_t misc = 0;   // small device words (the adjoint paint's max |weight|)
  size_t steps = 0;  // a run's step loop: counter, checkpoint base, factor table
  size_t red = 0;    // float64 partial sums of the chi^2 reduction
  size_t desc = 0;   // a batch plan's device descriptor table (member 0's)
  size_t cola = 0;   // COLA: per-step LPT-frame factors {c1, c2, dD1, dD2}
  size_t tab_coarse = 0, coarse[3] = {0, 0, 0}, force_c = 0;   // pyramid coarse grid
  size_t lat0 = 0;   // LPT lattice fields alias the mesh + particle region
  size_t total = 0;
  long n_keys = 0, cap = 0;
  int n_bins_max = 0;
};

int validate(const pm_config* c, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return PM_EINVAL;
  };
  if (!c) return bad("config is NULL");
  if (!(c->box_size > 0)) return bad("box_size must be > 0");
  if (!is_pow2(c->n_mesh) || c->n_mesh < 8 || c->n_mesh > 1024) return bad("n_mesh must be a power of 2 in [8, 1024]");
  if (!is_pow2(c->n_part) || c->n_part < 8 || c->n_part > c->n_mesh) return bad("n_part must be a power of 2 in [8, n_mesh]");
  if (c->n_mesh % c->n_part) return bad("n_mesh must be a multiple of n_part");
  if (!(c->cosmo.omega_m > 0 && c->cosmo.omega_m <= 1)) return bad("omega_m must be in (0, 1]");
  if (c->cosmo.pk_kind < 0 || c->cosmo.pk_kind > 2) return bad("unknown pk_kind");
  if (c->cosmo.pk_kind == PM_PK_EH_NOWIGGLE &&
      !(c->cosmo.h > 0 && c->cosmo.omega_b >= 0 && c->cosmo.omega_b < c->cosmo.omega_m && c->cosmo.t_cmb > 0))
    return bad("no-wiggle P(k) needs h > 0, 0 <= omega_b < omega_m, t_cmb > 0");
  if (c->cosmo.pk_kind == PM_PK_TABLE) {
    if (c->cosmo.pk_n < 2 || !c->cosmo.pk_k || !c->cosmo.pk_p) return bad("table P(k) needs pk_n >= 2 points");
    for (int i = 0; i < c->cosmo.pk_n; ++i) {
      if (!(c->cosmo.pk_k[i] > 0) || !(c->cosmo.pk_p[i] >= 0) || !std::isfinite(c->cosmo.pk_k[i]) ||
          !std::isfinite(c->cosmo.pk_p[i]))
        return bad("table P(k) needs finite k > 0 and P >= 0");
      if (i && !(c->cosmo.pk_k[i] > c->cosmo.pk_k[i - 1])) return bad("table k must increase");
    }
  }
  if (c->cosmo.pk_amp == 0 && c->cosmo.pk_kind != PM_PK_TABLE && !(c->cosmo.sigma8 > 0))
    return bad("sigma8 must be > 0 when pk_amp is 0");
  if (c->lpt_order != 1 && c->lpt_order != 2) return bad("lpt_order must be 1 or 2");
  if (c->deconv_order < 0 || c->deconv_order > 2) return bad("deconv_order must be 0, 1 or 2");
  if (c->split_mode < 0 || c->split_mode > 2) return bad("unknown split_mode");
  if (c->split_mode != PM_SPLIT_NONE && !(c->split_rs > 0)) return bad("split_rs must be > 0");
  if (!(c->lattice_shift >= 0 && c->lattice_shift < 1)) return bad("lattice_shift must be in [0, 1)");
  const long np3 = (long)c->n_part * c->n_part * c->n_part;
  if (c->max_particles < 0) return bad("max_particles must be >= 0");
  if (c->max_particles > 0 && c->max_particles < np3) return bad("max_particles must be 0 or >= n_part^3");
  if ((c->max_particles > 0 ? c->max_particles : np3) > (1L << 31) - 1) return bad("too many particles");
  if (c->pyramid_levels < 0 || c->pyramid_levels > 4) return bad("pyramid_levels must be in [0, 4]");
  if (c->batch < 0 || c->batch > PM_MAX_BATCH) return bad("batch must be in [0, PM_MAX_BATCH]");
  if (c->batch > 1 && (c->n_mesh < 64 || c->pyramid_levels > 0))
    return bad("a batch plan needs n_mesh >= 64 and no pyramid");
  if (c->integrator < PM_INT_FASTPM || c->integrator > PM_INT_COLA) return bad("unknown integrator");
  if (c->integrator == PM_INT_COLA && c->batch > 1) return bad("a batch plan takes no COLA integrator");
  if (c->pyramid_levels > 0) {
    if ((c->n_mesh >> c->pyramid_levels) < 8) return bad("the pyramid's coarse grid needs >= 8 cells per side");
    if (c->deconv_order != 0 || c->split_mode != PM_SPLIT_NONE)
      return bad("the pyramid force takes neither deconvolution nor a force split");
  }
  return PM_OK;
}

Layout make_layout(const pm_config* c) {
  Layout L;
  const long ng = c->n_mesh, np = c->n_part;
  const long np3 = np * np * np;
  L.cap = c->max_particles > 0 ? c->max_particles : np3;
  L.n_keys = (long)make_tiles((int)ng).ntiles * 64;   // tile x class x half-tile block
  L.n_bins_max = (int)(ng / 2);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align_up(bytes);
    return at;
  };
  L.tab_mesh = take(fft_table_bytes(ng));
  L.tab_lat = take(fft_table_bytes(np));
  L.pk_lat = take((size_t)(3 * (np / 2) * (np / 2) + 1) * 4);
  L.count = take((size_t)(L.n_keys + 1) * 4);
  L.off = take((size_t)(L.n_keys + 1) * 4);
  L.bsum = take((size_t)(pmk::scan_scratch_words(L.n_keys) + 1) * 4);
  L.pw_partial = take((size_t)pmk::power_partial_doubles(L.n_bins_max) * 8);
  L.pw_out = take((size_t)3 * L.n_bins_max * 8);
  L.misc = take(256);
  L.steps = take(256 + (size_t)kMaxSteps * 16);
  L.red = take((size_t)(pmk::kReducePartials + 2) * 8);
  L.desc = take((size_t)PM_MAX_BATCH * sizeof(pm_req_desc));
  L.cola = take((size_t)kMaxSteps * 16);
  const long nc = c->pyramid_levels > 0 ? ng >> c->pyramid_levels : 0;
  if (nc) L.tab_coarse = take(fft_table_bytes(nc));
  const size_t region = o;
  for (int i = 0; i < 3; ++i) L.mesh[i] = take(field_bytes(ng));
  L.force_i = take((size_t)ng * ng * ng * 12);
  for (int i = 0; i < 2; ++i) L.pos_s[i] = take((size_t)L.cap * 12);
  for (int i = 0; i < 2; ++i) L.mom_s[i] = take((size_t)L.cap * 12);
  for (int i = 0; i < 2; ++i) L.id_s[i] = take((size_t)L.cap * 4);
  L.key = take((size_t)L.cap * 4);
  if (nc) {
    for (int i = 0; i < 3; ++i) L.coarse[i] = take(field_bytes(nc));
    L.force_c = take((size_t)nc * nc * nc * 12);
  }
  // initial conditions (and their adjoint) use up to 13 lattice fields
  // inside the (then idle) mesh and particle region
  L.lat0 = region;
  const size_t lat_end = region + 13 * field_bytes(np);
  if (lat_end > o) o = lat_end;
  L.total = o;
  return L;
}

void build_fft_tables(long n, double rs, std::vector<char>& host, size_t base_off, FftTables& t, char* dev) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align_up(bytes);
    return at;
  };
  const size_t o_twn = take(n * 8), o_twh = take(n / 2 * 8);
  const size_t o_d = take(n * 4), o_k = take(n * 4), o_w = take(n * 4), o_s = take(n * 4);
  const size_t o_dz = take((n / 2 + 1) * 4), o_kz = take((n / 2 + 1) * 4), o_wz = take((n / 2 + 1) * 4),
               o_sz = take((n / 2 + 1) * 4);
  char* h = host.data() + base_off;
  float2* twn = reinterpret_cast<float2*>(h + o_twn);
  float2* twh = reinterpret_cast<float2*>(h + o_twh);
  for (long k = 0; k < n; ++k) twn[k] = make_float2((float)std::cos(2 * kPi * k / n), (float)-std::sin(2 * kPi * k / n));
  for (long k = 0; k < n / 2; ++k)
    twh[k] = make_float2((float)std::cos(2 * kPi * k / (n / 2)), (float)-std::sin(2 * kPi * k / (n / 2)));
  auto fill = [&](float* d, float* kk, float* w, float* s, long len, bool signed_freq) {
    for (long i = 0; i < len; ++i) {
      const double f = signed_freq ? (i < n / 2 ? (double)i : (double)(i - n)) : (double)i;
      const double om = 2 * kPi * f / n;
      d[i] = (float)((8.0 * std::sin(om) - std::sin(2.0 * om)) / 6.0);
      const double s2 = 2.0 * std::sin(om / 2.0);
      kk[i] = (float)(s2 * s2);
      const double sc = om == 0 ? 1.0 : std::sin(om / 2.0) / (om / 2.0);
      w[i] = (float)(sc * sc);
      s[i] = (float)std::exp(-om * om * rs * rs);
    }
  };
  fill(reinterpret_cast<float*>(h + o_d), reinterpret_cast<float*>(h + o_k), reinterpret_cast<float*>(h + o_w),
       reinterpret_cast<float*>(h + o_s), n, true);
  fill(reinterpret_cast<float*>(h + o_dz), reinterpret_cast<float*>(h + o_kz), reinterpret_cast<float*>(h + o_wz),
       reinterpret_cast<float*>(h + o_sz), n / 2 + 1, false);
  char* d = dev + base_off;
  t.n = (int)n;
  t.tw_n = reinterpret_cast<float2*>(d + o_twn);
  t.tw_h = reinterpret_cast<float2*>(d + o_twh);
  t.dxy = reinterpret_cast<float*>(d + o_d);
  t.kxy = reinterpret_cast<float*>(d + o_k);
  t.wxy = reinterpret_cast<float*>(d + o_w);
  t.sxy = reinterpret_cast<float*>(d + o_s);
  t.dz = reinterpret_cast<float*>(d + o_dz);
  t.kz = reinterpret_cast<float*>(d + o_kz);
  t.wz = reinterpret_cast<float*>(d + o_wz);
  t.sz = reinterpret_cast<float*>(d + o_sz);
}

// Kernel classes timed by the optional event profiler.
enum ProfCls : int {
  PC_FILL, PC_KEYS, PC_SCAN, PC_SCATTER, PC_PAINT, PC_FFT_R2C_Z, PC_FFT_Y_FWD, PC_FFT_X_FORCE, PC_FFT_Y_INV,
  PC_FFT_C2R_Z, PC_READOUT, PC_PYR_REDUCE, PC_PYR_COARSE, PC_PYR_EXPAND, PC_NCLS
};
const char* const kProfNames[PC_NCLS] = {"fill",       "keys",      "scan",        "scatter",
                                         "paint",      "fft_z_r2c", "fft_y_fwd",   "fft_x_force",
                                         "fft_y_inv",  "fft_z_c2r", "readout_kdk", "pyr_reduce",
                                         "pyr_coarse_force", "pyr_expand"};

struct Profiler {
  bool on = false;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  ~Profiler() {
    for (auto e : pool) (void)hipEventDestroy(e);   // teardown: nothing to report to
  }
};

}  // namespace

struct pm_ctx {
  pm_config cfg{};
  hipStream_t stream = nullptr;
  std::string err;
  pmk::Cosmo cosmo;
  std::vector<double> pk_k_copy, pk_p_copy;
  char* ws = nullptr;
  Layout L;
  int ng = 0, npart = 0, ratio = 1;
  long np3 = 0;
  pmk::TileGeom tg;
  FftTables tm, tl;
  Field mesh[3];
  float* force_i = nullptr;   // interleaved force mesh, x-blocked [n/8][n][n][8][3]
  float* cur_force = nullptr; // the force mesh the next readout reads (force_i or a checkpoint slot)
  // caller-owned force-mesh checkpoints of a run: slot j holds the force
  // mesh at a[j] (layout of force_i), so that the adjoint reads instead of
  // recomputing them
  float* fck = nullptr;
  long fck_slots = 0;
  float* fck_slot(int j) const { return fck + (size_t)j * ng * ng * ng * 3; }
  // pyramid: coarse grid of nc = ng / 2^levels cells per side
  int nc = 0;
  FftTables tc;
  Field coarse[3];
  const FftTables& tl_c() const { return tc; }
  float* force_c = nullptr;   // interleaved coarse force, fine-cell units
  uint32_t* misc = nullptr;   // small device words
  // the step loop of a run: step counter, checkpoint base and per-step
  // factors in device memory, and the captured graphs of one step starting
  // from either ping-pong buffer
  uint32_t* step_ctr = nullptr;
  float** ckpt_base_dev = nullptr;
  float4* step_tab = nullptr;
  double* red = nullptr;      // chi^2 partial sums (kReducePartials) + result
  bool use_graphs = false;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  long g_np = -1;
  bool g_ckpt = false;
  void drop_graphs() {
    for (auto& g : gexec)
      if (g) {
        (void)hipGraphExecDestroy(g);   // nothing to report to: the graph is rebuilt on demand
        g = nullptr;
      }
  }
  // COLA frame: caller's Psi1, Psi2 ([np][3] by particle id) and the
  // device table of per-step frame factors
  float* psi1 = nullptr;
  float* psi2 = nullptr;
  float4* cola_tab = nullptr;
  bool cola() const { return cfg.integrator == PM_INT_COLA; }
  // kick/drift factors of the configured integrator
  void factors(const double* a, int n_a, double* k1, double* dr, double* k2) const {
    cosmo.step_factors(cfg.integrator, a, n_a, k1, dr, k2);
  }
  // COLA frame coefficients at a: (c1, c2) of the LPT force, (q1, q2) of the
  // LPT momentum, (D1, D2)
  void cola_coeffs(double a, double* c, double* q, double* d) const {
    double g[6];
    cosmo.growth(a, g);
    const double d2 = cfg.lpt_order >= 2 ? g[2] : 0.0;
    c[0] = 1.5 * cfg.cosmo.omega_m * g[0];
    c[1] = 1.5 * cfg.cosmo.omega_m * (d2 - g[0] * g[0]);
    q[0] = a * a * g[4] * g[1] * g[0];
    q[1] = a * a * g[4] * g[3] * d2;
    d[0] = g[0];
    d[1] = d2;
  }
  // batch plans: member slots at a fixed stride of the workspace (member 0
  // is the plan itself; members 1.. are owned by it)
  int batch = 1;
  size_t mstride = 0;
  pm_ctx* plan = nullptr;             // members 1..: their plan
  std::vector<pm_ctx*> members;       // plan: members[0] == this
  pm_req_desc* desc_dev = nullptr;    // plan: device descriptor table (PM_MAX_BATCH entries)
  std::vector<pm_req_desc> desc_host;
  // plan: captured batched steps, one per number of running members (the
  // descriptors of the running members are packed at the front of the
  // table, so that a step launches no workgroups for idle slots)
  std::vector<hipGraphExec_t> bgraphs;
  void drop_bgraphs() {
    for (auto& g : bgraphs)
      if (g) {
        (void)hipGraphExecDestroy(g);   // rebuilt on demand
        g = nullptr;
      }
  }
  ~pm_ctx() {
    drop_graphs();
    drop_bgraphs();   // teardown: nothing to report to
    for (size_t m = 1; m < members.size(); ++m) delete members[m];
  }
  float* pos_s[2] = {};
  float* mom_s[2] = {};
  uint32_t* id_s[2] = {};
  uint32_t *key = nullptr, *count = nullptr, *off = nullptr, *bsum = nullptr;
  double *pw_partial = nullptr, *pw_out = nullptr;
  float* pk_lat = nullptr;
  Profiler prof;

  // state of a resumable run (pm_run_begin / advance / end)
  struct RunState {
    bool active = false;
    int ns = 0, step = 0, cur = 0;
    std::vector<double> k1, dr, k2;
    std::vector<float4> tab;   // host copy of the device step table
    float *pos = nullptr, *mom = nullptr, *ckpt = nullptr;
    bool fck = false;          // force meshes go to the checkpoint slots
    std::vector<float4> cola_tab;                 // COLA: host copy of the frame factors
    double cola_end[2] = {0, 0}, cola_qend[2] = {0, 0};
  } run;

  // run f (which enqueues one kernel class) between two events when profiling
  template <class F>
  void timed(int cls, F&& f) {
    if (!prof.on || prof.recs.size() >= 65536) {
      f();
      return;
    }
    hipEvent_t a = prof.get(), b = prof.get();
    if (!a || !b) {
      f();
      return;
    }
    // a pair whose record failed is dropped (the work itself still runs)
    const bool ok_a = hipEventRecord(a, stream) == hipSuccess;
    f();
    const bool ok_b = hipEventRecord(b, stream) == hipSuccess;
    if (ok_a && ok_b) prof.recs.push_back({cls, a, b});
  }

  int fail(int code, const std::string& m) {
    err = m;
    return code;
  }
  int check(const char* where) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
    return PM_OK;
  }
  Field lat(int i) const {
    Field f;
    char* b = ws + L.lat0 + (size_t)i * field_bytes(npart);
    f.r = reinterpret_cast<float*>(b);
    f.q = reinterpret_cast<float2*>(b + align_up((size_t)npart * npart * npart * 4));
    return f;
  }

  // counting sort of np particles (caller order) into sorted buffer dst
  // (a first sort: its input is in the caller's order, lattice order when
  // it holds n_part^3 particles, which the key and scatter passes walk brick
  // by brick)
  void sort(const float* pos, const float* mom, const uint32_t* id, long np, int dst) {
    const int lat_ln = np == np3 ? __builtin_ctz((unsigned)npart) : -1;
    timed(PC_FILL, [&] { pmk::launch_fill_u32(count, L.n_keys, 0u, stream); });
    timed(PC_KEYS, [&] { pmk::launch_keys(pos, np, tg, key, count, stream, lat_ln); });
    finish_sort(pos, mom, id, np, dst, lat_ln);
  }
  // scan + scatter once the keys and their counts are known
  void finish_sort(const float* pos, const float* mom, const uint32_t* id, long np, int dst, int lat_ln = -1) {
    timed(PC_SCAN, [&] { pmk::launch_scan(count, L.n_keys, off, bsum, stream); });
    pmk::ScatterArgs a;
    a.np = np;
    a.pos = pos;
    a.mom = mom;
    a.id = id;
    a.key = key;
    a.cursor = count;   // the scan left a copy of the offsets there
    a.pos_out = pos_s[dst];
    a.mom_out = mom ? mom_s[dst] : nullptr;
    a.id_out = id_s[dst];
    a.lat_ln = lat_ln;
    timed(PC_SCATTER, [&] { pmk::launch_scatter(a, stream); });
  }
  // overdensity of the sorted particles; std_layout: caller-visible [x][y][z]
  // mesh instead of the internal x-blocked one
  void paint(int cur, long np, float* out, bool std_layout = false) {
    const double scale = (double)ng * ng * ng / (double)np;
    timed(PC_PAINT, [&] { pmk::launch_paint(pos_s[cur], off, tg, out, (float)scale, -1.f, std_layout, stream); });
  }
  // force meshes of an n^3 grid (tables t, fields f[0..2], overdensity in
  // f[0].r, overwritten) into the interleaved mesh out; scale multiplies the
  // force (the inverse transform's 1/n^3 and any change of cell units); the
  // stages are timed by class when cls < 0, else as one class
  void force_on(const FftTables& t, Field* f, float* out, long n, double scale, int deconv, int split, int cls,
                const pmk::BatchArg& bat = pmk::BatchArg()) {
    auto tm_ = [&](int c, auto&& fn) { timed(cls < 0 ? c : cls, fn); };
    tm_(PC_FFT_R2C_Z, [&] { pmk::fft_z_r2c(t, &f[0], 1, stream, bat); });
    tm_(PC_FFT_Y_FWD, [&] { pmk::fft_y(t, &f[0], 1, -1, stream, bat); });
    pmk::SpecOp op;
    op.scale = (float)scale;
    op.deconv = deconv;
    op.split = split;
    // from 64^3 up F_y and F_z share one x transform (i g X) and get their
    // D(w_y), D(w_z) in the y pass; smaller meshes take the fused x pass
    const bool xs = n >= 64;
    op.kind = xs ? pmk::OP_FORCE_XS : pmk::OP_FORCE;
    op.n_out = xs ? 2 : 3;
    const int dst[3] = {0, xs ? 2 : 1, 2};
    for (int i = 0; i < op.n_out; ++i) {
      op.out_c[i] = f[dst[i]].c();
      op.out_q[i] = f[dst[i]].q;
    }
    tm_(PC_FFT_X_FORCE, [&] { pmk::fft_x_force(t, f[0], op, stream, bat); });
    if (xs)
      tm_(PC_FFT_Y_INV, [&] { pmk::fft_y_force(t, f, stream, bat); });
    else
      tm_(PC_FFT_Y_INV, [&] { pmk::fft_y(t, f, 3, 1, stream); });   // below 64^3: never batched
    tm_(PC_FFT_C2R_Z, [&] { pmk::fft_z_c2r_interleaved3(t, f, out, stream, bat); });
  }

  // REDUCE (expand = false) or EXPAND of ch channels over `levels` levels,
  // as three one-axis passes per level; intermediates alternate between the
  // halves of each channel's scratch (scr[c], 2 * half floats).  When the
  // three channel buffers are consecutive (scr[c] = scr[0] + c * stride,
  // stride >= 2 * half), three-channel intermediates are interleaved instead,
  // alternating between the two 3 * half-float halves of that region, so
  // that every tap of a pass is one 12-byte access.  The last pass writes
  // `out` with `mode`.
  void pyr_chain(bool expand, int ch, pmk::PyrField in, const pmk::PyrField& out, int levels, float* const* scr,
                 size_t half, int mode, const float* aux, float alpha) {
    const bool il = ch == 3 && scr[1] - scr[0] >= (ptrdiff_t)(2 * half) && scr[2] - scr[1] == scr[1] - scr[0];
    int k = 0;
    for (int lv = 0; lv < levels; ++lv)
      for (int ax = 0; ax < 3; ++ax) {
        const bool last = lv == levels - 1 && ax == 2;
        pmk::PyrField nx;
        if (last) {
          nx = out;
        } else {
          nx.kind = il ? pmk::PYR_INTERLEAVED : pmk::PYR_SEPARATE;
          nx.nx = in.nx;
          nx.ny = in.ny;
          nx.nz = in.nz;
          int* d = ax == 0 ? &nx.nx : (ax == 1 ? &nx.ny : &nx.nz);
          *d = expand ? *d * 2 : *d / 2;
          if (il)
            nx.p[0] = scr[0] + (k & 1) * 3 * half;
          else
            for (int c = 0; c < ch; ++c) nx.p[c] = scr[c] + (k & 1) * half;
        }
        pmk::launch_pyr_pass(expand, ax, ch, in, nx, last ? mode : pmk::PYR_STORE, aux, alpha, stream);
        in = nx;
        ++k;
      }
  }

  // force meshes from the overdensity in mesh[0].r (overwritten) into out
  // (default force_i); the next readout reads them
  void force_meshes(float* out = nullptr) {
    out = out ? out : force_i;
    cur_force = out;
    const double g = 1.5 * cfg.cosmo.omega_m;
    if (!nc) {
      force_on(tm, mesh, out, ng, g / ((double)ng * ng * ng), cfg.deconv_order, cfg.split_mode, -1);
      return;
    }
    // Algorithm 3 with one device holding the periodic mesh:
    //   F = EXPAND(F_L) + F_S - EXPAND(REDUCE(F_S)) = F_S + EXPAND(F_L - REDUCE(F_S))
    // (EXPAND is linear); F_L is the coarse-grid force of REDUCE(delta),
    // converted to fine cells by 2^levels.
    const int lv = cfg.pyramid_levels;
    const size_t half = (size_t)ng * ng * ng / 2;
    pmk::PyrField fine1, coarse1;
    fine1.kind = pmk::PYR_SEPARATE;
    fine1.p[0] = mesh[0].r;
    fine1.nx = fine1.ny = fine1.nz = (int)ng;
    coarse1.kind = pmk::PYR_SEPARATE;
    coarse1.p[0] = coarse[0].r;
    coarse1.nx = coarse1.ny = coarse1.nz = nc;
    float* scr_d[1] = {mesh[1].r};
    timed(PC_PYR_REDUCE, [&] { pyr_chain(false, 1, fine1, coarse1, lv, scr_d, half, pmk::PYR_STORE, nullptr, 0.f); });
    force_on(tc, coarse, force_c, nc, g / ((double)nc * nc * nc) * (double)(1 << lv), 0, 0, PC_PYR_COARSE);
    force_on(tm, mesh, out, ng, g / ((double)ng * ng * ng), 0, 0, -1);
    // D = F_L - REDUCE(F_S) on the coarse grid (three channels in the now
    // idle coarse fields), then F_S += EXPAND(D)
    pmk::PyrField fs, dc;
    fs.kind = pmk::PYR_INTERLEAVED;
    fs.p[0] = out;
    fs.nx = fs.ny = fs.nz = (int)ng;
    dc.kind = pmk::PYR_SEPARATE;
    for (int c = 0; c < 3; ++c) dc.p[c] = coarse[c].r;
    dc.nx = dc.ny = dc.nz = nc;
    float* scr3[3] = {mesh[0].r, mesh[1].r, mesh[2].r};
    timed(PC_PYR_REDUCE, [&] { pyr_chain(false, 3, fs, dc, lv, scr3, half, pmk::PYR_COMBINE, force_c, 1.f); });
    timed(PC_PYR_EXPAND, [&] { pyr_chain(true, 3, dc, fs, lv, scr3, half, pmk::PYR_ADD, nullptr, 0.f); });
  }
  void readout(const pmk::ReadoutArgs& a) {
    timed(PC_READOUT, [&] { pmk::launch_readout(a, stream); });
  }
  // One KDK step of the members listed in the device descriptors d[0..n):
  // every kernel is launched once with blockIdx.z over the descriptors and
  // member 0's workspace pointers (the kernels shift them by member *
  // mstride).  Between steps a member's sorted state is in buffer 0; the
  // readout writes the updated state to buffer 1 in the same order and the
  // scatter sorts it back into buffer 0.  The static tables are member 0's
  // (every member holds the same ones).
  void batched_step(const pm_req_desc* d, int n) {
    Range rg("pm_kdk_step_batched", n);
    pmk::BatchArg bat;
    bat.d = d;
    bat.stride = (long)mstride;
    bat.n = n;
    const long np = np3;
    timed(PC_FILL, [&] { pmk::launch_fill_u32(count, L.n_keys, 0u, stream, bat); });
    pmk::ReadoutArgs a = readout_args(0, np);
    a.fi = force_i;
    a.flags = pmk::RO_KICK | pmk::RO_DRIFT | pmk::RO_KEYS | pmk::RO_TO_ALT;
    a.pos_alt = pos_s[1];
    a.mom_alt = mom_s[1];
    a.id_alt = id_s[1];
    a.bat = bat;
    readout(a);
    timed(PC_SCAN, [&] { pmk::launch_scan(count, L.n_keys, off, bsum, stream, bat); });
    pmk::ScatterArgs sa;
    sa.np = np;
    sa.pos = pos_s[1];
    sa.mom = mom_s[1];
    sa.id = id_s[1];
    sa.key = key;
    sa.cursor = count;
    sa.pos_out = pos_s[0];
    sa.mom_out = mom_s[0];
    sa.id_out = id_s[0];
    sa.bat = bat;
    timed(PC_SCATTER, [&] { pmk::launch_scatter(sa, stream); });
    const double scale = (double)ng * ng * ng / (double)np;
    timed(PC_PAINT, [&] {
      pmk::launch_paint(pos_s[0], off, tg, mesh[0].r, (float)scale, -1.f, false, stream, bat);
    });
    const double g = 1.5 * cfg.cosmo.omega_m;
    force_on(tm, mesh, force_i, ng, g / ((double)ng * ng * ng), cfg.deconv_order, cfg.split_mode, -1, bat);
  }
  pmk::ReadoutArgs readout_args(int cur, long np) {
    pmk::ReadoutArgs a;
    a.g = tg;
    a.np = np;
    a.pos = pos_s[cur];
    a.mom = mom_s[cur];
    a.id = id_s[cur];
    a.fi = cur_force ? cur_force : force_i;
    a.key_out = key;
    a.count = count;
    return a;
  }
};

extern "C" {

const char* pm_strerror(int s) {
  switch (s) {
    case PM_OK: return "ok";
    case PM_EINVAL: return "invalid argument";
    case PM_ENOMEM: return "workspace too small";
    case PM_EHIP: return "HIP runtime error";
    case PM_ESTATE: return "invalid state";
    default: return "unknown status";
  }
}

const char* pm_last_error(const pm_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

namespace {
int batch_of(const pm_config* cfg) { return cfg->batch > 1 ? cfg->batch : 1; }

// One simulation's context over the workspace at ws (layout L); the static
// tables are uploaded with `stream` (and waited for).
int create_one(const pm_config* cfg, char* ws, const Layout& L, void* stream, pm_ctx** out);
}  // namespace

size_t pm_workspace_bytes(const pm_config* cfg) {
  if (validate(cfg, nullptr) != PM_OK) return 0;
  return make_layout(cfg).total * (size_t)batch_of(cfg);
}

int pm_create(const pm_config* cfg, void* d_workspace, size_t bytes, void* stream, pm_ctx** out) {
  if (!out) return PM_EINVAL;
  *out = nullptr;
  std::string why;
  if (validate(cfg, &why) != PM_OK) {
    std::fprintf(stderr, "pm_create: %s\n", why.c_str());
    return PM_EINVAL;
  }
  if (!d_workspace || ((uintptr_t)d_workspace % kAlign)) return PM_EINVAL;
  const Layout L = make_layout(cfg);
  const int nb = batch_of(cfg);
  if (bytes / (size_t)nb < L.total) return PM_ENOMEM;
  char* ws = reinterpret_cast<char*>(d_workspace);
  pm_ctx* plan = nullptr;
  int st = create_one(cfg, ws, L, stream, &plan);
  if (st != PM_OK) return st;
  if (nb > 1) {
    plan->batch = nb;
    plan->mstride = L.total;
    plan->desc_dev = reinterpret_cast<pm_req_desc*>(ws + L.desc);
    plan->desc_host.assign(nb, pm_req_desc{});
    plan->members.push_back(plan);
    for (int m = 1; m < nb; ++m) {
      pm_ctx* c = nullptr;
      st = create_one(cfg, ws + (size_t)m * L.total, L, stream, &c);
      if (st != PM_OK) {
        delete plan;
        return st;
      }
      c->plan = plan;
      plan->members.push_back(c);
    }
  }
  *out = plan;
  return PM_OK;
}

namespace {
int create_one(const pm_config* cfg, char* ws, const Layout& L, void* stream, pm_ctx** out) {
  pm_ctx* c = new (std::nothrow) pm_ctx;
  if (!c) return PM_ENOMEM;
  c->cfg = *cfg;
  if (cfg->cosmo.pk_kind == PM_PK_TABLE) {   // own a copy of the caller's table
    c->pk_k_copy.assign(cfg->cosmo.pk_k, cfg->cosmo.pk_k + cfg->cosmo.pk_n);
    c->pk_p_copy.assign(cfg->cosmo.pk_p, cfg->cosmo.pk_p + cfg->cosmo.pk_n);
    c->cfg.cosmo.pk_k = c->pk_k_copy.data();
    c->cfg.cosmo.pk_p = c->pk_p_copy.data();
  }
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->ws = ws;
  c->L = L;
  c->ng = cfg->n_mesh;
  c->npart = cfg->n_part;
  c->ratio = cfg->n_mesh / cfg->n_part;
  c->np3 = (long)cfg->n_part * cfg->n_part * cfg->n_part;
  c->cosmo.init(c->cfg.cosmo);
  c->tg = make_tiles(c->ng);
  char* w = c->ws;
  for (int i = 0; i < 3; ++i) {
    c->mesh[i].r = reinterpret_cast<float*>(w + L.mesh[i]);
    c->mesh[i].q = reinterpret_cast<float2*>(w + L.mesh[i] + align_up((size_t)c->ng * c->ng * c->ng * 4));
  }
  // the interleaved c2r addresses the three meshes by one stride
  if (c->mesh[2].r - c->mesh[1].r != c->mesh[1].r - c->mesh[0].r ||
      c->mesh[2].q - c->mesh[1].q != c->mesh[1].q - c->mesh[0].q) {
    std::fprintf(stderr, "pm_create: mesh fields are not equally spaced\n");
    delete c;
    return PM_EINVAL;
  }
  c->force_i = reinterpret_cast<float*>(w + L.force_i);
  c->misc = reinterpret_cast<uint32_t*>(w + L.misc);
  c->step_ctr = reinterpret_cast<uint32_t*>(w + L.steps);
  c->ckpt_base_dev = reinterpret_cast<float**>(w + L.steps + 64);
  c->step_tab = reinterpret_cast<float4*>(w + L.steps + 256);
  c->red = reinterpret_cast<double*>(w + L.red);
  c->cola_tab = reinterpret_cast<float4*>(w + L.cola);
  c->nc = cfg->pyramid_levels > 0 ? c->ng >> cfg->pyramid_levels : 0;
  if (c->nc) {
    for (int i = 0; i < 3; ++i) {
      c->coarse[i].r = reinterpret_cast<float*>(w + L.coarse[i]);
      c->coarse[i].q = reinterpret_cast<float2*>(w + L.coarse[i] + align_up((size_t)c->nc * c->nc * c->nc * 4));
    }
    c->force_c = reinterpret_cast<float*>(w + L.force_c);
  }
  for (int i = 0; i < 2; ++i) {
    c->pos_s[i] = reinterpret_cast<float*>(w + L.pos_s[i]);
    c->mom_s[i] = reinterpret_cast<float*>(w + L.mom_s[i]);
    c->id_s[i] = reinterpret_cast<uint32_t*>(w + L.id_s[i]);
  }
  c->key = reinterpret_cast<uint32_t*>(w + L.key);
  c->count = reinterpret_cast<uint32_t*>(w + L.count);
  c->off = reinterpret_cast<uint32_t*>(w + L.off);
  c->bsum = reinterpret_cast<uint32_t*>(w + L.bsum);
  c->pw_partial = reinterpret_cast<double*>(w + L.pw_partial);
  c->pw_out = reinterpret_cast<double*>(w + L.pw_out);
  c->pk_lat = reinterpret_cast<float*>(w + L.pk_lat);

  // static tables, built on the host in float64 and uploaded once
  std::vector<char> host(L.mesh[0], 0);
  const double rs = cfg->split_mode != PM_SPLIT_NONE ? cfg->split_rs : 0.0;
  build_fft_tables(c->ng, rs, host, L.tab_mesh, c->tm, w);
  build_fft_tables(c->npart, 0.0, host, L.tab_lat, c->tl, w);
  if (c->nc) build_fft_tables(c->nc, 0.0, host, L.tab_coarse, c->tc, w);
  {
    float* pk = reinterpret_cast<float*>(host.data() + L.pk_lat);
    const long h = c->npart / 2;
    const double box = cfg->box_size;
    const double vcell = std::pow(box / c->npart, 3);
    const double n3 = (double)c->np3;
    for (long n2 = 0; n2 <= 3 * h * h; ++n2) {
      const double k = 2 * kPi * std::sqrt((double)n2) / box;
      pk[n2] = n2 == 0 ? 0.f : (float)(std::sqrt(c->cosmo.pk(k) / vcell) / n3);
    }
  }
  hipError_t e = hipMemcpyAsync(w, host.data(), L.mesh[0], hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    std::fprintf(stderr, "pm_create: %s\n", hipGetErrorString(e));
    delete c;
    return PM_EHIP;
  }
  *out = c;
  return PM_OK;
}
}  // namespace

int pm_destroy(pm_ctx* ctx) {
  if (ctx && ctx->plan) return PM_EINVAL;   // a member belongs to its plan
  delete ctx;
  return PM_OK;
}

int pm_set_stream(pm_ctx* ctx, void* stream) {
  if (!ctx) return PM_EINVAL;
  if (ctx->plan) return ctx->fail(PM_EINVAL, "set the stream on the plan, not on a member");
  for (pm_ctx* m : ctx->members) m->stream = reinterpret_cast<hipStream_t>(stream);
  ctx->stream = reinterpret_cast<hipStream_t>(stream);
  ctx->drop_bgraphs();   // a captured step belongs to its stream's capture: rebuilt on the next advance
  return PM_OK;
}

int pm_sync(pm_ctx* ctx) {
  if (!ctx) return PM_EINVAL;
  const hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return ctx->fail(PM_EHIP, std::string("sync: ") + hipGetErrorString(e));
  return ctx->check("sync");
}

int pm_growth(const pm_ctx* ctx, double a, double* out6) {
  if (!ctx || !out6 || !(a > 0)) return PM_EINVAL;
  ctx->cosmo.growth(a, out6);
  return PM_OK;
}

int pm_kdk_factors(const pm_ctx* ctx, const double* h_a, int n_a, double* h_k1, double* h_dr, double* h_k2) {
  if (!ctx || !h_a || !h_k1 || !h_dr || !h_k2 || n_a < 2) return PM_EINVAL;
  for (int i = 0; i < n_a; ++i)
    if (!(h_a[i] > 0) || (i && !(h_a[i] > h_a[i - 1]))) return PM_EINVAL;
  ctx->factors(h_a, n_a, h_k1, h_dr, h_k2);
  return PM_OK;
}

int pm_noise(pm_ctx* ctx, uint64_t seed, float* d_noise) {
  if (!ctx || !d_noise) return PM_EINVAL;
  pmk::launch_noise(seed, ctx->npart, d_noise, false, ctx->stream);
  return ctx->check("pm_noise");
}

int pm_init_lpt(pm_ctx* ctx, uint64_t seed, double a0, const float* d_noise_in, float* d_noise_out, float* d_pos,
                float* d_mom) {
  if (!ctx || !d_pos || !d_mom || !(a0 > 0)) return PM_EINVAL;
  Range rg("pm_init_lpt");
  pm_ctx& c = *ctx;
  const long n3 = c.np3;
  Field f[10];
  for (int i = 0; i < 10; ++i) f[i] = c.lat(i);
  // the lattice fields are x-blocked; the caller's noise is [x][y][z]
  if (d_noise_in)
    pmk::launch_relayout(d_noise_in, f[0].r, c.npart, true, c.stream);
  else
    pmk::launch_noise(seed, c.npart, f[0].r, true, c.stream);
  if (d_noise_out) pmk::launch_relayout(f[0].r, d_noise_out, c.npart, false, c.stream);
  const int order = c.cfg.lpt_order;
  pmk::fft_r2c_zy(c.tl, &f[0], 1, c.stream);
  pmk::SpecOp op;
  op.kind = pmk::OP_LPT1;
  op.n_out = order >= 2 ? 9 : 3;
  op.pk = c.pk_lat;
  for (int i = 0; i < op.n_out; ++i) {
    op.out_c[i] = f[1 + i].c();
    op.out_q[i] = f[1 + i].q;
  }
  pmk::fft_x_fused(c.tl, f[0], op, c.stream);
  pmk::fft_c2r_yz(c.tl, &f[1], op.n_out, c.stream);
  if (order >= 2) {
    float* phi[6] = {f[4].r, f[5].r, f[6].r, f[7].r, f[8].r, f[9].r};
    pmk::launch_lpt_delta2(phi, n3, f[0].r, c.stream);
    pmk::fft_r2c_zy(c.tl, &f[0], 1, c.stream);
    pmk::SpecOp op2;
    op2.kind = pmk::OP_LPT2;
    op2.n_out = 3;
    op2.scale = (float)(1.0 / (double)n3);
    for (int i = 0; i < 3; ++i) {
      op2.out_c[i] = f[4 + i].c();
      op2.out_q[i] = f[4 + i].q;
    }
    pmk::fft_x_fused(c.tl, f[0], op2, c.stream);
    pmk::fft_c2r_yz(c.tl, &f[4], 3, c.stream);
  }
  double g[6];
  c.cosmo.growth(a0, g);
  const double d1 = g[0], f1 = g[1], d2 = order >= 2 ? g[2] : 0.0, f2 = g[3], e = g[4];
  const double b = c.ratio;
  pmk::LptParticleArgs a;
  a.np = c.npart;
  a.ratio = c.ratio;
  a.shift = (float)c.cfg.lattice_shift;
  a.nmesh = (float)c.ng;
  a.cx1 = (float)(b * d1);
  a.cx2 = (float)(b * d2);
  a.cp1 = (float)(b * a0 * a0 * e * f1 * d1);
  a.cp2 = (float)(b * a0 * a0 * e * f2 * d2);
  for (int d = 0; d < 3; ++d) {
    a.s1[d] = f[1 + d].r;
    a.s2[d] = f[4 + d].r;
  }
  a.has_s2 = order >= 2 ? 1 : 0;
  a.pos = d_pos;
  a.mom = d_mom;
  a.psi1 = c.psi1;   // the LPT frame, when set: B s1, B s2
  a.psi2 = c.psi2;
  pmk::launch_lpt_particles(a, c.stream);
  return c.check("pm_init_lpt");
}

int pm_paint(pm_ctx* ctx, const float* d_pos, int64_t np, float* d_delta) {
  if (!ctx || !d_pos || !d_delta || np < 1 || np > ctx->L.cap) return PM_EINVAL;
  pm_ctx& c = *ctx;
  c.sort(d_pos, nullptr, nullptr, np, 0);
  c.paint(0, np, d_delta, true);
  return c.check("pm_paint");
}

int pm_force(pm_ctx* ctx, const float* d_pos, int64_t np, float* d_force) {
  if (!ctx || !d_pos || !d_force || np < 1 || np > ctx->L.cap) return PM_EINVAL;
  pm_ctx& c = *ctx;
  c.sort(d_pos, nullptr, nullptr, np, 0);
  c.paint(0, np, c.mesh[0].r);
  c.force_meshes();
  pmk::ReadoutArgs a = c.readout_args(0, np);
  a.mom = nullptr;
  a.flags = pmk::RO_FORCE_BYID;
  a.force_out = d_force;
  c.readout(a);
  return c.check("pm_force");
}

int pm_kdk_step(pm_ctx* ctx, float* d_pos, float* d_mom, float* d_force, double a0, double a1) {
  if (!ctx || !d_pos || !d_mom || !d_force || !(a0 > 0) || !(a1 > a0)) return PM_EINVAL;
  pm_ctx& c = *ctx;
  const double aa[2] = {a0, a1};
  double k1, dr, k2;
  if (c.cola()) return c.fail(PM_EINVAL, "pm_kdk_step: the COLA integrator runs through pm_run");
  c.factors(aa, 2, &k1, &dr, &k2);
  pmk::launch_kick_drift(d_pos, d_mom, d_force, c.np3, (float)k1, (float)dr, (float)c.ng, c.stream);
  c.sort(d_pos, d_mom, nullptr, c.np3, 0);
  c.paint(0, c.np3, c.mesh[0].r);
  c.force_meshes();
  pmk::ReadoutArgs a = c.readout_args(0, c.np3);
  a.flags = pmk::RO_KICK | pmk::RO_XP_BYID | pmk::RO_FORCE_BYID;
  a.kick_a = (float)k2;
  a.kick_b = 0.f;
  a.pos_out = d_pos;
  a.mom_out = d_mom;
  a.force_out = d_force;
  c.readout(a);
  return c.check("pm_kdk_step");
}

int pm_run_begin(pm_ctx* ctx, const double* h_a, int n_a, float* d_pos, float* d_mom, float* d_ckpt) {
  if (!ctx || !h_a || n_a < 1 || !d_pos || !d_mom) return PM_EINVAL;
  pm_ctx& c = *ctx;
  for (int i = 0; i < n_a; ++i)
    if (!(h_a[i] > 0) || (i && !(h_a[i] > h_a[i - 1]))) return c.fail(PM_EINVAL, "a must be > 0 and increasing");
  auto& r = c.run;
  r = pm_ctx::RunState();
  r.ns = n_a - 1;
  r.k1.resize(r.ns);
  r.dr.resize(r.ns);
  r.k2.resize(r.ns);
  if (r.ns > kMaxSteps) return c.fail(PM_EINVAL, "at most 65536 steps per run");
  if (c.cola()) {
    if (!c.psi1) return c.fail(PM_ESTATE, "pm_run_begin: the COLA integrator needs pm_set_lpt_frame");
    if (d_ckpt) return c.fail(PM_EINVAL, "pm_run_begin: no checkpoints with the COLA integrator");
  }
  c.factors(h_a, n_a, r.k1.data(), r.dr.data(), r.k2.data());
  r.tab.resize(r.ns);
  for (int i = 0; i < r.ns; ++i)
    r.tab[i] = make_float4(i ? (float)r.k2[i - 1] : 0.f, (float)r.k1[i], (float)r.dr[i], 0.f);
  r.pos = d_pos;
  r.mom = d_mom;
  r.ckpt = d_ckpt;
  r.cur = 0;
  r.step = 0;
  const long np = c.np3;
  if (r.ns > 0) {
    hipError_t e = hipMemcpyAsync(c.step_tab, r.tab.data(), (size_t)r.ns * sizeof(float4), hipMemcpyHostToDevice,
                                  c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c.ckpt_base_dev, &r.ckpt, sizeof(float*), hipMemcpyHostToDevice, c.stream);
    if (e != hipSuccess) return c.fail(PM_EHIP, std::string("pm_run_begin: ") + hipGetErrorString(e));
  }
  pmk::launch_fill_u32(c.step_ctr, 1, 0u, c.stream);
  r.fck = c.fck && n_a <= c.fck_slots;
  Range rg("pm_run_begin");
  c.sort(d_pos, d_mom, nullptr, np, r.cur);
  if (c.cola()) {
    // the frame's factors per step: LPT force at a_i, LPT drift a_i -> a_i+1;
    // the end's factors, and the start's residual momentum p - p_LPT(a0)
    r.cola_tab.resize(r.ns > 0 ? r.ns : 1);
    double cc[2], q[2], d[2], cn[2], qn[2], dn[2];
    for (int i = 0; i < r.ns; ++i) {
      c.cola_coeffs(h_a[i], cc, q, d);
      c.cola_coeffs(h_a[i + 1], cn, qn, dn);
      r.cola_tab[i] = make_float4((float)cc[0], (float)cc[1], (float)(dn[0] - d[0]), (float)(dn[1] - d[1]));
    }
    c.cola_coeffs(h_a[n_a - 1], r.cola_end, r.cola_qend, d);
    if (r.ns > 0) {
      const hipError_t e = hipMemcpyAsync(c.cola_tab, r.cola_tab.data(), (size_t)r.ns * sizeof(float4),
                                          hipMemcpyHostToDevice, c.stream);
      if (e != hipSuccess) return c.fail(PM_EHIP, std::string("pm_run_begin: ") + hipGetErrorString(e));
    }
    c.cola_coeffs(h_a[0], cc, q, d);
    pmk::launch_frame_shift(c.mom_s[r.cur], c.id_s[r.cur], c.psi1, c.psi2, np, (float)-q[0], (float)-q[1],
                            c.stream);
  }
  c.paint(r.cur, np, c.mesh[0].r);
  c.force_meshes(r.fck ? c.fck_slot(0) : nullptr);
  r.active = true;
  return c.check("pm_run_begin");
}

int pm_run_advance(pm_ctx* ctx, int max_steps, int* h_remaining) {
  if (!ctx || max_steps < 0) return PM_EINVAL;
  pm_ctx& c = *ctx;
  auto& r = c.run;
  if (!r.active) return c.fail(PM_ESTATE, "no run in progress");
  const long np = c.np3;
  // one step from ping-pong buffer cur; its factors and checkpoint slot come
  // from the device step table at the device step counter
  auto enqueue_step = [&](int cur, int i) {
    Range rg("pm_kdk_step", i);
    c.timed(PC_FILL, [&] { pmk::launch_fill_u32(c.count, c.L.n_keys, 0u, c.stream); });
    pmk::ReadoutArgs a = c.readout_args(cur, np);
    a.flags = pmk::RO_KICK | pmk::RO_DRIFT | pmk::RO_WRITE_SORTED | pmk::RO_KEYS | (r.ckpt ? pmk::RO_CKPT : 0);
    if (c.cola()) {
      a.flags |= pmk::RO_COLA;
      a.psi1 = c.psi1;
      a.psi2 = c.psi2;
      a.cola_steps = c.cola_tab;
    }
    a.steps = c.step_tab;
    a.step_i = c.step_ctr;
    a.ckpt_base = c.ckpt_base_dev;
    a.ckpt_stride = np * 3;
    c.readout(a);
    c.finish_sort(c.pos_s[cur], c.mom_s[cur], c.id_s[cur], np, 1 - cur);
    c.paint(1 - cur, np, c.mesh[0].r);
    c.force_meshes(r.fck ? c.fck_slot(i + 1) : nullptr);
    pmk::launch_step_inc(c.step_ctr, c.stream);
  };
  // (force checkpoints move the output every step: launched eagerly)
  const bool graphs = c.use_graphs && !c.prof.on && !r.fck;
  if (graphs && (c.g_np != np || c.g_ckpt != (r.ckpt != nullptr))) {
    c.drop_graphs();
    c.g_np = np;
    c.g_ckpt = r.ckpt != nullptr;
  }
  for (int k = 0; k < max_steps && r.step < r.ns; ++k) {
    if (graphs) {
      hipGraphExec_t& ge = c.gexec[r.cur];
      if (!ge) {
        if (hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed) != hipSuccess)
          return c.fail(PM_EHIP, "pm_run_advance: stream capture could not start (graphs need a non-default stream)");
        enqueue_step(r.cur, r.step);
        hipGraph_t g = nullptr;
        const hipError_t e1 = hipStreamEndCapture(c.stream, &g);
        const hipError_t e2 = e1 == hipSuccess ? hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) : e1;
        if (g) (void)hipGraphDestroy(g);   // the instantiated graph keeps what it needs
        if (e2 != hipSuccess) {
          ge = nullptr;
          return c.fail(PM_EHIP, std::string("pm_run_advance: graph capture failed: ") + hipGetErrorString(e2));
        }
      }
      const hipError_t e = hipGraphLaunch(ge, c.stream);
      if (e != hipSuccess) return c.fail(PM_EHIP, std::string("pm_run_advance: ") + hipGetErrorString(e));
    } else {
      enqueue_step(r.cur, r.step);
    }
    r.cur = 1 - r.cur;
    ++r.step;
  }
  if (h_remaining) *h_remaining = r.ns - r.step;
  return c.check("pm_run_advance");
}

int pm_run_end(pm_ctx* ctx, float* d_delta_final) {
  if (!ctx) return PM_EINVAL;
  pm_ctx& c = *ctx;
  auto& r = c.run;
  if (!r.active) return c.fail(PM_ESTATE, "no run in progress");
  if (r.step != r.ns) return c.fail(PM_ESTATE, "pm_run_end before the last step");
  const long np = c.np3;
  const size_t ck = (size_t)np * 3;
  Range rg("pm_run_end");
  if (d_delta_final) c.paint(r.cur, np, d_delta_final, true);
  pmk::ReadoutArgs a = c.readout_args(r.cur, np);
  a.flags = pmk::RO_KICK | pmk::RO_XP_BYID;
  a.kick_a = r.ns ? (float)r.k2[r.ns - 1] : 0.f;
  a.kick_b = 0.f;
  a.pos_out = r.pos;
  a.mom_out = r.mom;
  if (c.cola()) {   // residual kick at the last a, then back to the full momentum
    a.flags |= pmk::RO_COLA | pmk::RO_COLA_OUT;
    a.psi1 = c.psi1;
    a.psi2 = c.psi2;
    a.cola = make_float4((float)r.cola_end[0], (float)r.cola_end[1], 0.f, 0.f);
    a.cola_out = make_float2((float)r.cola_qend[0], (float)r.cola_qend[1]);
  }
  if (r.ckpt) {
    a.flags |= pmk::RO_CKPT;
    a.ckpt_x = r.ckpt + (2 * (size_t)r.ns) * ck;
    a.ckpt_p = r.ckpt + (2 * (size_t)r.ns + 1) * ck;
  }
  c.readout(a);
  r.active = false;
  return c.check("pm_run_end");
}

int pm_run(pm_ctx* ctx, const double* h_a, int n_a, float* d_pos, float* d_mom, float* d_ckpt,
           float* d_delta_final) {
  int st = pm_run_begin(ctx, h_a, n_a, d_pos, d_mom, d_ckpt);
  if (st != PM_OK) return st;
  int rem = 0;
  st = pm_run_advance(ctx, n_a, &rem);
  if (st != PM_OK) return st;
  return pm_run_end(ctx, d_delta_final);
}

int pm_kdk_step_batched(pm_ctx* plan, const pm_req_desc* d_descs, int n) {
  if (!plan) return PM_EINVAL;
  if (plan->batch < 2 || plan->plan) return plan->fail(PM_EINVAL, "pm_kdk_step_batched: not a batch plan");
  if (!d_descs || n < 1 || n > plan->batch) return plan->fail(PM_EINVAL, "pm_kdk_step_batched: bad descriptors");
  plan->batched_step(d_descs, n);
  return plan->check("pm_kdk_step_batched");
}

int pm_batch_member(pm_ctx* plan, int m, pm_ctx** out) {
  if (!plan || !out || plan->plan || plan->batch < 2 || m < 0 || m >= plan->batch) return PM_EINVAL;
  *out = plan->members[m];
  return PM_OK;
}

int pm_batch_begin(pm_ctx* plan, int m, const double* h_a, int n_a, float* d_pos, float* d_mom, float* d_ckpt) {
  if (!plan || plan->plan || plan->batch < 2 || m < 0 || m >= plan->batch) return PM_EINVAL;
  pm_ctx* c = plan->members[m];
  if (c->run.active) return plan->fail(PM_ESTATE, "pm_batch_begin: the member already runs");
  if (c->fck) return plan->fail(PM_ESTATE, "pm_batch_begin: members take no force checkpoints");
  const int st = pm_run_begin(c, h_a, n_a, d_pos, d_mom, d_ckpt);   // sorts into buffer 0
  if (st != PM_OK) return plan->fail(st, std::string("pm_batch_begin: ") + c->err);
  return PM_OK;
}

int pm_batch_advance(pm_ctx* plan, int* h_stepped) {
  if (!plan || plan->plan || plan->batch < 2) return PM_EINVAL;
  pm_ctx& p = *plan;
  int k = 0;   // running members, their descriptors packed at the front
  for (int m = 0; m < p.batch; ++m) {
    auto& r = p.members[m]->run;
    if (!r.active || r.step >= r.ns) continue;
    pm_req_desc& d = p.desc_host[k];
    d = pm_req_desc{};
    const int i = r.step;
    const size_t ck = (size_t)p.np3 * 3;
    d.member = m;
    d.kick_close = r.tab[i].x;
    d.kick_open = r.tab[i].y;
    d.drift = r.tab[i].z;
    if (r.ckpt) {
      d.flags = PM_REQ_CKPT;
      d.ckpt_x = r.ckpt + (2 * (size_t)i) * ck;
      d.ckpt_p = r.ckpt + (2 * (size_t)i + 1) * ck;
    }
    ++k;
  }
  if (h_stepped) *h_stepped = k;
  if (!k) return PM_OK;
  // pageable source: the copy has left desc_host when the call returns
  hipError_t e = hipMemcpyAsync(p.desc_dev, p.desc_host.data(), (size_t)k * sizeof(pm_req_desc),
                                hipMemcpyHostToDevice, p.stream);
  if (e != hipSuccess) return p.fail(PM_EHIP, std::string("pm_batch_advance: ") + hipGetErrorString(e));
  if (p.use_graphs && !p.prof.on) {
    if (p.bgraphs.size() < (size_t)p.batch + 1) p.bgraphs.resize((size_t)p.batch + 1, nullptr);
    hipGraphExec_t& ge = p.bgraphs[k];
    if (!ge) {
      if (hipStreamBeginCapture(p.stream, hipStreamCaptureModeRelaxed) != hipSuccess)
        return p.fail(PM_EHIP, "pm_batch_advance: stream capture could not start (graphs need a non-default stream)");
      p.batched_step(p.desc_dev, k);
      hipGraph_t g = nullptr;
      const hipError_t e1 = hipStreamEndCapture(p.stream, &g);
      const hipError_t e2 = e1 == hipSuccess ? hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) : e1;
      if (g) (void)hipGraphDestroy(g);   // the instantiated graph keeps what it needs
      if (e2 != hipSuccess) {
        ge = nullptr;
        return p.fail(PM_EHIP, std::string("pm_batch_advance: graph capture failed: ") + hipGetErrorString(e2));
      }
    }
    e = hipGraphLaunch(ge, p.stream);
    if (e != hipSuccess) return p.fail(PM_EHIP, std::string("pm_batch_advance: ") + hipGetErrorString(e));
  } else {
    p.batched_step(p.desc_dev, k);
  }
  for (int i = 0; i < k; ++i) ++p.members[p.desc_host[i].member]->run.step;
  return p.check("pm_batch_advance");
}

int pm_batch_remaining(pm_ctx* plan, int m) {
  if (!plan || plan->plan || plan->batch < 2 || m < 0 || m >= plan->batch) return PM_EINVAL;
  const auto& r = plan->members[m]->run;
  if (!r.active) return PM_ESTATE;
  return r.ns - r.step;
}

int pm_batch_end(pm_ctx* plan, int m, float* d_delta_final) {
  if (!plan || plan->plan || plan->batch < 2 || m < 0 || m >= plan->batch) return PM_EINVAL;
  pm_ctx* c = plan->members[m];
  if (!c->run.active) return plan->fail(PM_ESTATE, "pm_batch_end: the member does not run");
  c->run.step = c->run.ns;   // steps taken through pm_kdk_step_batched are not counted here
  const int st = pm_run_end(c, d_delta_final);
  if (st != PM_OK) return plan->fail(st, std::string("pm_batch_end: ") + c->err);
  return PM_OK;
}

int pm_run_adjoint(pm_ctx* ctx, const double* h_a, int n_a, const float* d_ckpt, const float* d_noise,
                   const float* d_grad_delta_final, float* d_grad_pos, float* d_grad_mom, float* d_grad_noise) {
  if (!ctx || !h_a || n_a < 1 || !d_ckpt || !d_grad_pos || !d_grad_mom) return PM_EINVAL;
  pm_ctx& c = *ctx;
  if (d_grad_noise && !d_noise) return c.fail(PM_EINVAL, "d_grad_noise needs d_noise");
  for (int i = 0; i < n_a; ++i)
    if (!(h_a[i] > 0) || (i && !(h_a[i] > h_a[i - 1]))) return c.fail(PM_EINVAL, "a must be > 0 and increasing");
  const int ns = n_a - 1;
  if (c.cola()) return c.fail(PM_EINVAL, "pm_run_adjoint: no adjoint of the COLA integrator");
  std::vector<double> k1(ns), dr(ns), k2(ns);
  c.factors(h_a, n_a, k1.data(), dr.data(), k2.data());
  const long np = c.np3;
  const size_t ck = (size_t)np * 3;
  float* xbar = d_grad_pos;
  float* pbar = d_grad_mom;
  auto ckpt_x = [&](int i) { return d_ckpt + 2 * (size_t)i * ck; };
  const double s = (double)c.ng * c.ng * c.ng / (double)np;
  // loss on the final overdensity: x_bar += paint^T-gradient of s * delta_bar
  if (d_grad_delta_final) {
    c.sort(ckpt_x(ns), nullptr, nullptr, np, 0);
    pmk::launch_readout_grad1(c.pos_s[0], c.id_s[0], np, c.ng, d_grad_delta_final, (float)s, xbar, true,
                              c.stream);
  }
  // reverse sweep over the force evaluation points x_ns ... x_0; the force
  // meshes come from the forward's checkpoints when it kept them
  const bool use_fck = c.fck && n_a <= c.fck_slots;
  for (int j = ns; j >= 0; --j) {
    Range rg("pm_adjoint_step", j);
    const double kj = (j < ns ? k1[j] : 0.0) + (j > 0 ? k2[j - 1] : 0.0);
    if (kj != 0.0) {
      c.sort(ckpt_x(j), nullptr, nullptr, np, 0);
      const float* fmesh = c.force_i;
      if (use_fck) {
        fmesh = c.fck_slot(j);
      } else {
        c.paint(0, np, c.mesh[0].r);
        c.force_meshes();
      }
      // term A: positions at which the force meshes are read out; it joins
      // term B's pass at the end of the step unless the pyramid below uses
      // the force mesh as scratch
      const bool fuse_ab = !c.nc || use_fck;
      if (!fuse_ab)
        pmk::launch_readout_grad3(c.pos_s[0], c.id_s[0], np, c.ng, fmesh, pbar, (float)kj, xbar, c.stream);
      // term B: positions that paint the density, through G^T
      pmk::launch_absmax(pbar, 3 * np, c.misc, c.stream);
      // the three channels in one launch (the meshes are equally spaced)
      pmk::launch_paint_weighted(c.pos_s[0], c.id_s[0], c.off, c.tg, pbar, -1, (float)kj, c.misc, c.mesh[0].r,
                                 c.stream, (long)(c.mesh[1].r - c.mesh[0].r));
      // pyramid force: F_d^T m = G_d^T (m - E R m) + 2^f E G_c,d^T R m
      // (R = REDUCE, E = EXPAND); the interleaved force mesh, read by term A
      // above, is free scratch here
      const size_t n3 = (size_t)c.ng * c.ng * c.ng;
      float* scr3[3] = {c.force_i, c.force_i + n3, c.force_i + 2 * n3};
      pmk::PyrField mf, cf;
      if (c.nc) {
        mf.kind = cf.kind = pmk::PYR_SEPARATE;
        mf.nx = mf.ny = mf.nz = c.ng;
        cf.nx = cf.ny = cf.nz = c.nc;
        for (int d = 0; d < 3; ++d) {
          mf.p[d] = c.mesh[d].r;
          cf.p[d] = c.coarse[d].r;
        }
        const int lv = c.cfg.pyramid_levels;
        c.pyr_chain(false, 3, mf, cf, lv, scr3, n3 / 2, pmk::PYR_STORE, nullptr, 0.f);   // R m
        c.pyr_chain(true, 3, cf, mf, lv, scr3, n3 / 2, pmk::PYR_SUB, nullptr, 0.f);     // m - E R m
      }
      pmk::fft_r2c_zy(c.tm, c.mesh, 3, c.stream);
      pmk::SpecOp op;
      op.kind = pmk::OP_FORCE_T;
      op.n_in = 3;
      op.n_out = 1;
      op.scale = (float)(1.5 * c.cfg.cosmo.omega_m / (double)np);
      op.deconv = c.cfg.deconv_order;
      op.split = c.cfg.split_mode;
      for (int d = 0; d < 3; ++d) {
        op.in_c[d] = c.mesh[d].c();
        op.in_q[d] = c.mesh[d].q;
      }
      op.out_c[0] = c.mesh[0].c();
      op.out_q[0] = c.mesh[0].q;
      pmk::fft_x_force_t(c.tm, c.mesh, op, c.stream);
      pmk::fft_c2r_yz(c.tm, &c.mesh[0], 1, c.stream);
      if (c.nc) {
        // coarse part: G_c^T over R m with the coarse transform's 1/nc^3 and
        // the coarse force's 2^f, then expanded onto the fine result
        const int lv = c.cfg.pyramid_levels;
        pmk::fft_r2c_zy(c.tl_c(), c.coarse, 3, c.stream);
        pmk::SpecOp oc = op;
        oc.deconv = 0;
        oc.split = 0;
        oc.scale = (float)(1.5 * c.cfg.cosmo.omega_m * s * (double)(1 << lv) / ((double)c.nc * c.nc * c.nc));
        for (int d = 0; d < 3; ++d) {
          oc.in_c[d] = c.coarse[d].c();
          oc.in_q[d] = c.coarse[d].q;
        }
        oc.out_c[0] = c.coarse[0].c();
        oc.out_q[0] = c.coarse[0].q;
        pmk::fft_x_force_t(c.tl_c(), c.coarse, oc, c.stream);
        pmk::fft_c2r_yz(c.tl_c(), &c.coarse[0], 1, c.stream);
        pmk::PyrField c1, f1;
        c1.kind = f1.kind = pmk::PYR_SEPARATE;
        c1.nx = c1.ny = c1.nz = c.nc;
        c1.p[0] = c.coarse[0].r;
        f1.nx = f1.ny = f1.nz = c.ng;
        f1.p[0] = c.mesh[0].r;
        c.pyr_chain(true, 1, c1, f1, lv, scr3, n3 / 2, pmk::PYR_ADD, nullptr, 0.f);
      }
      if (fuse_ab)
        pmk::launch_readout_grad31(c.pos_s[0], c.id_s[0], np, c.ng, fmesh, pbar, (float)kj, c.mesh[0].r, xbar,
                                   c.stream);
      else
        pmk::launch_readout_grad1(c.pos_s[0], c.id_s[0], np, c.ng, c.mesh[0].r, 1.f, xbar, false, c.stream);
    }
    if (j > 0) pmk::launch_axpy(pbar, xbar, (float)dr[j - 1], (long)ck, c.stream);
  }
  if (!d_grad_noise) return c.check("pm_run_adjoint");

  // Gen-IC: noise_bar from (x0_bar, p0_bar)
  const long n3 = np;
  const int order = c.cfg.lpt_order;
  Field f[13];
  for (int i = 0; i < 13; ++i) f[i] = c.lat(i);
  pmk::launch_relayout(d_noise, f[0].r, c.npart, true, c.stream);
  double g[6];
  c.cosmo.growth(h_a[0], g);
  const double a0 = h_a[0], b = c.ratio;
  const double d1 = g[0], f1 = g[1], d2 = order >= 2 ? g[2] : 0.0, f2 = g[3], e = g[4];
  float* s1b[3] = {f[7].r, f[8].r, f[9].r};
  float* s2b[3] = {f[10].r, f[11].r, f[12].r};
  pmk::launch_lpt_sbar(xbar, pbar, n3, (float)(b * d1), (float)(b * a0 * a0 * e * f1 * d1), (float)(b * d2),
                       (float)(b * a0 * a0 * e * f2 * d2), s1b, s2b, c.stream);
  int n_in = 3;
  if (order >= 2) {
    // phi_ij of the linear field
    pmk::fft_r2c_zy(c.tl, &f[0], 1, c.stream);
    pmk::SpecOp op;
    op.kind = pmk::OP_LPT_PHI;
    op.n_out = 6;
    op.pk = c.pk_lat;
    for (int i = 0; i < 6; ++i) {
      op.out_c[i] = f[1 + i].c();
      op.out_q[i] = f[1 + i].q;
    }
    pmk::fft_x_fused(c.tl, f[0], op, c.stream);
    pmk::fft_c2r_yz(c.tl, &f[1], 6, c.stream);
    // delta2_bar = sum_d S2_d^T s2_bar_d
    pmk::fft_r2c_zy(c.tl, &f[10], 3, c.stream);
    pmk::SpecOp o2;
    o2.kind = pmk::OP_LPT2_T;
    o2.n_in = 3;
    o2.scale = (float)(1.0 / (double)n3);
    for (int d = 0; d < 3; ++d) {
      o2.in_c[d] = f[10 + d].c();
      o2.in_q[d] = f[10 + d].q;
    }
    o2.out_c[0] = f[0].c();
    o2.out_q[0] = f[0].q;
    pmk::fft_x_fused(c.tl, f[0], o2, c.stream);
    pmk::fft_c2r_yz(c.tl, &f[0], 1, c.stream);
    float* phi[6] = {f[1].r, f[2].r, f[3].r, f[4].r, f[5].r, f[6].r};
    pmk::launch_lpt_phibar(phi, f[0].r, n3, c.stream);
    pmk::fft_r2c_zy(c.tl, &f[1], 6, c.stream);
    n_in = 9;
  }
  pmk::fft_r2c_zy(c.tl, &f[7], 3, c.stream);
  pmk::SpecOp o1;
  o1.kind = pmk::OP_LPT1_T;
  o1.n_in = n_in;
  o1.pk = c.pk_lat;
  for (int d = 0; d < 3; ++d) {
    o1.in_c[d] = f[7 + d].c();
    o1.in_q[d] = f[7 + d].q;
  }
  for (int i = 0; i < 6 && n_in == 9; ++i) {
    o1.in_c[3 + i] = f[1 + i].c();
    o1.in_q[3 + i] = f[1 + i].q;
  }
  o1.out_c[0] = f[0].c();
  o1.out_q[0] = f[0].q;
  pmk::fft_x_fused(c.tl, f[0], o1, c.stream);
  pmk::fft_c2r_yz(c.tl, &f[0], 1, c.stream);
  pmk::launch_relayout(f[0].r, d_grad_noise, c.npart, false, c.stream);
  return c.check("pm_run_adjoint");
}

// ---- MAP reconstruction (section 7) --------------------------------------
namespace {
struct ReconWork {
  float *ckpt, *fck, *pos, *mom, *resid, *gnoise;
  double *partials, *out;
  size_t total;
};

ReconWork recon_work(const pm_ctx& c, int n_a, char* base) {
  ReconWork w{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + o : nullptr;
    o += align_up(bytes);
    return p;
  };
  const size_t st = (size_t)c.np3 * 3 * sizeof(float);
  w.ckpt = reinterpret_cast<float*>(take((size_t)n_a * 2 * st));
  w.fck = reinterpret_cast<float*>(take((size_t)n_a * c.ng * c.ng * c.ng * 3 * sizeof(float)));
  w.pos = reinterpret_cast<float*>(take(st));
  w.mom = reinterpret_cast<float*>(take(st));
  w.resid = reinterpret_cast<float*>(take((size_t)c.ng * c.ng * c.ng * sizeof(float)));
  w.gnoise = reinterpret_cast<float*>(take((size_t)c.np3 * sizeof(float)));
  w.partials = reinterpret_cast<double*>(take(pmk::kReducePartials * sizeof(double)));
  w.out = reinterpret_cast<double*>(take(2 * sizeof(double)));
  w.total = o;
  return w;
}
}  // namespace

int pm_chi2(pm_ctx* ctx, const float* d_delta, const float* d_data, double sigma, float* d_grad, double* d_chi2) {
  if (!ctx || !d_delta || !d_data || !d_grad || !d_chi2) return PM_EINVAL;
  pm_ctx& c = *ctx;
  if (!(sigma > 0)) return c.fail(PM_EINVAL, "sigma must be > 0");
  const long ncell = (long)c.ng * c.ng * c.ng;
  pmk::launch_residual(d_delta, d_data, d_grad, ncell, (float)(1.0 / sigma), c.red, d_chi2, c.stream);
  return c.check("pm_chi2");
}

size_t pm_recon_work_bytes(const pm_ctx* ctx, int n_a) {
  if (!ctx || n_a < 2) return 0;
  return recon_work(*ctx, n_a, nullptr).total;
}

int pm_recon_step(pm_ctx* ctx, const double* h_a, int n_a, const float* d_data, double sigma, float* d_noise,
                  float* d_adam_m, float* d_adam_v, int t, double lr, double beta1, double beta2, double eps,
                  void* d_work, size_t work_bytes, double* h_loss2) {
  if (!ctx || !h_a || n_a < 2 || !d_data || !d_noise || !d_adam_m || !d_adam_v || !d_work || !h_loss2)
    return PM_EINVAL;
  pm_ctx& c = *ctx;
  if (!(sigma > 0) || t < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps >= 0))
    return c.fail(PM_EINVAL, "need sigma > 0, t >= 1, lr > 0, 0 <= beta < 1, eps >= 0");
  if ((uintptr_t)d_work % kAlign) return c.fail(PM_EINVAL, "d_work must be 256-byte aligned");
  if (c.cola()) return c.fail(PM_EINVAL, "pm_recon_step: no reconstruction with the COLA integrator");
  if (c.run.active) return c.fail(PM_ESTATE, "a resumable run is in progress");
  const ReconWork w = recon_work(c, n_a, static_cast<char*>(d_work));
  if (work_bytes < w.total) return c.fail(PM_ENOMEM, "reconstruction work buffer too small");
  int st = pm_init_lpt(ctx, 0, h_a[0], d_noise, nullptr, w.pos, w.mom);
  if (st != PM_OK) return st;
  // the run keeps its force meshes in the work buffer for the adjoint
  float* const user_fck = c.fck;
  const long user_slots = c.fck_slots;
  c.fck = w.fck;
  c.fck_slots = n_a;
  struct Restore {
    pm_ctx& c;
    float* f;
    long n;
    ~Restore() {
      c.fck = f;
      c.fck_slots = n;
    }
  } restore{c, user_fck, user_slots};
  st = pm_run(ctx, h_a, n_a, w.pos, w.mom, w.ckpt, w.resid);
  if (st != PM_OK) return st;
  const long ncell = (long)c.ng * c.ng * c.ng;
  pmk::launch_residual(w.resid, d_data, w.resid, ncell, (float)(1.0 / sigma), w.partials, w.out, c.stream);
  // the state buffers become the zeroed cotangent accumulators of the adjoint
  pmk::launch_fill_u32(reinterpret_cast<uint32_t*>(w.pos), c.np3 * 3, 0u, c.stream);
  pmk::launch_fill_u32(reinterpret_cast<uint32_t*>(w.mom), c.np3 * 3, 0u, c.stream);
  st = pm_run_adjoint(ctx, h_a, n_a, w.ckpt, d_noise, w.resid, w.pos, w.mom, w.gnoise);
  if (st != PM_OK) return st;
  pmk::launch_adam(d_noise, w.gnoise, d_adam_m, d_adam_v, c.np3, (float)lr, (float)beta1, (float)beta2, (float)eps,
                   (float)(1.0 / (1.0 - std::pow(beta1, t))), (float)(1.0 / (1.0 - std::pow(beta2, t))), w.partials,
                   w.out + 1, c.stream);
  hipError_t e = hipMemcpyAsync(h_loss2, w.out, 2 * sizeof(double), hipMemcpyDeviceToHost, c.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  if (e != hipSuccess) return c.fail(PM_EHIP, std::string("pm_recon_step: ") + hipGetErrorString(e));
  return c.check("pm_recon_step");
}

int pm_power(pm_ctx* ctx, const float* d_delta, int n_bins, int n_max, int deconv, double* h_k, double* h_pk,
             double* h_nmodes) {
  if (!ctx || !d_delta || !h_k || !h_pk || !h_nmodes) return PM_EINVAL;
  pm_ctx& c = *ctx;
  if (n_bins < 1 || n_bins > c.L.n_bins_max) return c.fail(PM_EINVAL, "n_bins must be in [1, n_mesh/2]");
  pmk::launch_relayout(d_delta, c.mesh[0].r, c.ng, true, c.stream);
  pmk::fft_r2c_zy(c.tm, &c.mesh[0], 1, c.stream);
  pmk::fft_x_forward(c.tm, &c.mesh[0], 1, c.stream);
  pmk::PowerArgs a;
  a.n = c.ng;
  a.n_bins = n_bins;
  a.n_max = n_max;
  a.deconv = deconv;
  a.c = c.mesh[0].c();
  a.q = c.mesh[0].q;
  a.wxy = c.tm.wxy;
  a.wz = c.tm.wz;
  a.partial = c.pw_partial;
  pmk::launch_power(a, c.pw_out, c.stream);
  std::vector<double> h(3 * (size_t)n_bins);
  hipError_t e = hipMemcpyAsync(h.data(), c.pw_out, h.size() * 8, hipMemcpyDeviceToHost, c.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  if (e != hipSuccess) return c.fail(PM_EHIP, std::string("pm_power: ") + hipGetErrorString(e));
  const double box = c.cfg.box_size;
  const double n3 = (double)c.ng * c.ng * c.ng;
  const double norm = box * box * box / (n3 * n3);
  for (int j = 0; j < n_bins; ++j) {
    const double sw = h[j], sk = h[n_bins + j], sp = h[2 * n_bins + j];
    h_nmodes[j] = sw;
    h_k[j] = sw > 0 ? sk / sw * 2 * kPi / box : 0.0;
    h_pk[j] = sw > 0 ? sp / sw * norm : 0.0;
  }
  return c.check("pm_power");
}

int pm_rfft(pm_ctx* ctx, const float* d_real, float* d_spec) {
  if (!ctx || !d_real || !d_spec) return PM_EINVAL;
  pm_ctx& c = *ctx;
  pmk::launch_relayout(d_real, c.mesh[0].r, c.ng, true, c.stream);
  pmk::fft_r2c_zy(c.tm, &c.mesh[0], 1, c.stream);
  pmk::fft_x_forward(c.tm, &c.mesh[0], 1, c.stream);
  pmk::launch_spec_to_numpy(c.mesh[0].c(), c.mesh[0].q, reinterpret_cast<float2*>(d_spec), c.ng, 1.f, c.stream);
  return c.check("pm_rfft");
}

int pm_irfft(pm_ctx* ctx, const float* d_spec, float* d_real) {
  if (!ctx || !d_real || !d_spec) return PM_EINVAL;
  pm_ctx& c = *ctx;
  const long n3 = (long)c.ng * c.ng * c.ng;
  pmk::launch_spec_from_numpy(reinterpret_cast<const float2*>(d_spec), c.mesh[0].c(), c.mesh[0].q, c.ng,
                              (float)(1.0 / (double)n3), c.stream);
  pmk::fft_x_inverse(c.tm, &c.mesh[0], 1, c.stream);
  pmk::fft_c2r_yz(c.tm, &c.mesh[0], 1, c.stream);
  pmk::launch_relayout(c.mesh[0].r, d_real, c.ng, false, c.stream);
  return c.check("pm_irfft");
}

int pm_set_force_ckpt(pm_ctx* ctx, float* d_fckpt, int64_t n_slots) {
  if (!ctx || n_slots < 0 || (d_fckpt && n_slots < 1)) return PM_EINVAL;
  if (ctx->run.active) return ctx->fail(PM_ESTATE, "a resumable run is in progress");
  ctx->fck = n_slots ? d_fckpt : nullptr;
  ctx->fck_slots = d_fckpt ? n_slots : 0;
  return PM_OK;
}

int pm_set_lpt_frame(pm_ctx* ctx, float* d_psi1, float* d_psi2) {
  if (!ctx) return PM_EINVAL;
  if (!d_psi1 != !d_psi2) return ctx->fail(PM_EINVAL, "pm_set_lpt_frame: both fields or neither");
  if (ctx->run.active) return ctx->fail(PM_ESTATE, "pm_set_lpt_frame during a run");
  ctx->psi1 = d_psi1;
  ctx->psi2 = d_psi2;
  ctx->drop_graphs();   // captured steps hold the frame's pointers
  return PM_OK;
}

int pm_use_graphs(pm_ctx* ctx, int enable) {
  if (!ctx) return PM_EINVAL;
  ctx->use_graphs = enable != 0;
  if (!ctx->use_graphs) {
    ctx->drop_graphs();
    ctx->drop_bgraphs();
  }
  return PM_OK;
}

int pm_profile(pm_ctx* ctx, int enable) {
  if (!ctx) return PM_EINVAL;
  ctx->prof.on = enable != 0;
  if (enable) {
    ctx->prof.recs.clear();
    ctx->prof.used = 0;
  }
  return PM_OK;
}

int pm_profile_read(pm_ctx* ctx, int max, char* h_names, double* h_total_ms, int* h_count) {
  if (!ctx || max < 0 || (max > 0 && (!h_names || !h_total_ms || !h_count))) return PM_EINVAL;
  pm_ctx& c = *ctx;
  const hipError_t e = hipStreamSynchronize(c.stream);
  if (e != hipSuccess) return c.fail(PM_EHIP, std::string("pm_profile_read: ") + hipGetErrorString(e));
  double tot[PC_NCLS] = {};
  int cnt[PC_NCLS] = {};
  for (const auto& r : c.prof.recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      tot[r.cls] += ms;
      cnt[r.cls] += 1;
    }
  }
  int k = 0;
  for (int i = 0; i < PC_NCLS; ++i) {
    if (!cnt[i]) continue;
    if (k < max) {
      std::snprintf(h_names + 32 * k, 32, "%s", kProfNames[i]);
      h_total_ms[k] = tot[i];
      h_count[k] = cnt[i];
    }
    ++k;
  }
  return k;
}

}  // extern "C"
