/*
 * pm.h - C ABI of the MI355X particle-mesh (PM) N-body library.
 *
 * The library evolves dark-matter particles with the FastPM kick-drift-kick
 * scheme described in section 2 of Modi, Lanusse & Seljak (arXiv:2010.11847):
 * cloud-in-cell (CIC) painting of the particles to a periodic mesh, a real
 * 3D FFT, the finite-difference (FD) Green's function and gradient kernels,
 * three inverse FFTs to force meshes, CIC readout at the particles, and
 * growth-factor weighted kick and drift updates.  Initial conditions follow
 * the Gen-IC algorithm of section 6 (Gaussian field scaled by P(k), then
 * first- or second-order Lagrangian displacements).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All functions are extern "C" and return an int status: PM_OK (0) or a
 *    negative PM_E* code.  Nothing throws across the ABI.
 *  - Pointers named d_* are device pointers (HBM of the GPU the context was
 *    created on); pointers named h_* are host pointers.  Every array is owned
 *    by the caller.  The library never allocates device memory: its scratch
 *    lives in the workspace handed to pm_create.
 *  - Particle arrays are float32, array-of-structures [n][3] (x, y, z).
 *    Positions and momenta are in mesh-cell units: the box is [0, n_mesh)^3,
 *    H0 = 1, a (scale factor) is the time variable.  Momentum is
 *    p = a^3 E(a) dx/da.  To convert: position in Mpc/h = x * box/n_mesh.
 *  - Meshes are float32, C order [x][y][z], n_mesh^3 elements.
 *  - Work is enqueued asynchronously on the context's stream (a hipStream_t
 *    passed as void*).  Kernel errors raised asynchronously surface as
 *    PM_EHIP at the next call that synchronises (pm_sync, pm_power, ...).
 *  - A context is not thread-safe.  Separate contexts on separate streams
 *    with separate workspaces are independent.
 *  - Particle lattice: particle index i = (ix*Np + iy)*Np + iz sits at
 *    q = B*(ix, iy, iz) + lattice_shift with B = n_mesh / n_part.
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define PM_OK       0
#define PM_EINVAL  (-1)   /* invalid argument or configuration */
#define PM_ENOMEM  (-2)   /* workspace smaller than pm_workspace_bytes() */
#define PM_EHIP    (-3)   /* HIP runtime error (text in pm_last_error) */
#define PM_ESTATE  (-4)   /* call not valid in the context's current state */

/* ---- linear power spectrum kinds --------------------------------------- */
#define PM_PK_POWERLAW     0  /* P(k) = A k^pk_index */
#define PM_PK_EH_NOWIGGLE  1  /* Eisenstein & Hu (1998) no-wiggle, A k^n_s T0(k)^2 */
#define PM_PK_TABLE        2  /* caller's table, log-log interpolated */

/* ---- time-stepping schemes (pm_config.integrator) ----------------------
 * All three are kick-drift-kick leapfrogs over the same PM force and the
 * same scale factors, half steps at a_c = sqrt(a_i a_{i+1}).
 *  FASTPM   : FastPM's kick/drift factors (section 2), exact for the linear
 *             growing mode.
 *  LEAPFROG : the plain leapfrog of dx/da = p/(a^3 E), dp/da = F/(a^2 E):
 *             kick int da/(a^2 E), drift int da/(a^3 E).
 *  COLA     : that leapfrog applied to the residual from the particles' LPT
 *             trajectory x_LPT = q + D1 Psi1 + D2 Psi2 (the comoving
 *             Lagrangian acceleration frame; section 2 leaves other PM
 *             schemes to the implementer): the force less the LPT force
 *             1.5 Om [D1 Psi1 + (D2 - D1^2) Psi2] kicks the residual
 *             momentum, and every drift adds the LPT displacement exactly.
 *             Needs the LPT displacement fields (pm_set_lpt_frame). */
#define PM_INT_FASTPM    0
#define PM_INT_LEAPFROG  1
#define PM_INT_COLA      2

/* ---- optional long/short force split (Fourier filter S = exp(-k^2 rs^2)) */
#define PM_SPLIT_NONE   0     /* full force */
#define PM_SPLIT_LONG   1     /* long-range part  S(k) * F */
#define PM_SPLIT_SHORT  2     /* short-range part (1 - S(k)) * F */

typedef struct {
    double omega_m;    /* matter density today; flat, Omega_L = 1 - omega_m */
    double omega_b;    /* baryons (no-wiggle transfer function only) */
    double h;          /* H0 / (100 km/s/Mpc) (transfer function only) */
    double n_s;        /* primordial tilt (no-wiggle only) */
    double sigma8;     /* rms linear overdensity in 8 Mpc/h spheres at a = 1 */
    double t_cmb;      /* CMB temperature in K (no-wiggle only) */
    int    pk_kind;    /* PM_PK_* */
    double pk_amp;     /* A; 0 = normalise to sigma8 (POWERLAW, EH_NOWIGGLE) */
    double pk_index;   /* power-law index (POWERLAW) */
    const double *pk_k, *pk_p;  /* TABLE: host arrays (h/Mpc, (Mpc/h)^3), copied by pm_create */
    int    pk_n;       /* TABLE: number of points (>= 2, k increasing) */
} pm_cosmo;

typedef struct {
    double   box_size;      /* comoving box side in Mpc/h (> 0) */
    int      n_mesh;        /* mesh cells per side: power of 2 in [8, 1024] */
    int      n_part;        /* particles per side of the lattice; n_mesh % n_part == 0,
                               n_part a power of 2 >= 8 */
    pm_cosmo cosmo;
    int      lpt_order;     /* 1 (Zel'dovich) or 2 (default in the presets) */
    int      deconv_order;  /* 0, 1 or 2: force divided by W_CIC(k)^deconv_order */
    double   split_rs;      /* split radius in mesh cells (used if split_mode != NONE) */
    int      split_mode;    /* PM_SPLIT_* */
    double   lattice_shift; /* offset of the particle lattice from mesh nodes, cells, [0, 1) */
    int64_t  max_particles; /* capacity for pm_paint/pm_force/pm_kdk_step; 0 = n_part^3 */
    int      pyramid_levels; /* 0: single-grid force; f >= 1: the multi-grid force of section 5.2
                                (Algorithm 3) with a coarse grid n_mesh / 2^f >= 8 per side,
                                order-6 B-spline REDUCE/EXPAND; needs deconv_order 0 and no
                                split; pm_run_adjoint differentiates it (its transpose) */
    int      batch;         /* 0 or 1: one simulation.  B in [2, PM_MAX_BATCH]: a batch plan of B
                               same-shape member slots (continuous batching, see pm_batch_*);
                               needs n_mesh >= 64 and pyramid_levels 0 */
    int      integrator;    /* PM_INT_* (0 = FastPM).  COLA: pm_run / pm_run_begin only (no
                               pm_kdk_step, checkpoints, adjoint, reconstruction or batch plan);
                               LEAPFROG: everywhere FASTPM is */
} pm_config;

typedef struct pm_ctx pm_ctx;   /* opaque; host memory only */

/* Bytes of device workspace pm_create needs for this configuration, or 0 if
 * the configuration is invalid.  Deterministic in the configuration. */
size_t pm_workspace_bytes(const pm_config* cfg);

/* Validate cfg, lay out the workspace and upload the static tables (FFT
 * twiddles, FD kernel tables, the sqrt(P(k)/V) table of the lattice) with the
 * given stream.  d_workspace must stay valid until pm_destroy; it must be
 * 256-byte aligned.  Computes every time-independent quantity on the host in
 * float64.  Returns PM_EINVAL (bad cfg), PM_ENOMEM (bytes too small) or PM_EHIP. */
int pm_create(const pm_config* cfg, void* d_workspace, size_t bytes, void* stream,
              pm_ctx** out);

/* Free the host-side context (never the workspace).  NULL is allowed. */
int pm_destroy(pm_ctx* ctx);

/* Change the stream used by later calls. */
int pm_set_stream(pm_ctx* ctx, void* stream);

/* Wait for the context's stream; reports asynchronous kernel errors. */
int pm_sync(pm_ctx* ctx);

const char* pm_strerror(int status);
const char* pm_last_error(const pm_ctx* ctx);

/* Growth and time-step factors computed by the library (float64, host):
 * out[0..5] = D1, f1, D2, f2, E, G_f at scale factor a (D1(1) = 1). */
int pm_growth(const pm_ctx* ctx, double a, double* h_out6);

/* Time-step factors of n_a - 1 KDK steps over h_a[0] < ... < h_a[n_a-1] of
 * the configured integrator (FASTPM, section 2: kick and drift exact for the
 * Zel'dovich growing mode; LEAPFROG and COLA: the plain time integrals):
 * h_k1[i] opening kick a_i -> a_c, h_dr[i] drift a_i -> a_{i+1}, h_k2[i]
 * closing kick a_c -> a_{i+1}, a_c = sqrt(a_i a_{i+1}).  Host arrays of
 * n_a - 1 doubles each, owned by the caller.  PM_EINVAL for a NULL pointer,
 * n_a < 2 or scale factors not positive and increasing. */
int pm_kdk_factors(const pm_ctx* ctx, const double* h_a, int n_a, double* h_k1, double* h_dr, double* h_k2);

/* Gen-IC step 1 (section 6): unit white noise on the n_part^3 lattice from the
 * counter-based generator (SplitMix64 output of seed*2^40 + site, Box-Muller,
 * cosine branch).  d_noise: [n_part^3] float32. */
int pm_noise(pm_ctx* ctx, uint64_t seed, float* d_noise);

/* Gen-IC (section 6): white noise -> linear field delta_L(k) =
 * DFT(w) sqrt(P(k)/V_cell) -> LPT displacements with the FD kernels of
 * section 2 on the lattice -> particle positions and momenta at scale factor
 * a0.  d_noise_in: [n_part^3] noise to use, or NULL to draw it from seed;
 * d_noise_out: NULL or [n_part^3] receives the noise used.  d_pos, d_mom:
 * [n_part^3][3] outputs in lattice (particle index) order. */
int pm_init_lpt(pm_ctx* ctx, uint64_t seed, double a0, const float* d_noise_in,
                float* d_noise_out, float* d_pos, float* d_mom);

/* CIC paint (section 2): delta(c) = rho(c) * n_mesh^3 / np - 1 with
 * rho(c) = sum_p prod_d max(0, 1 - |x_pd - c_d|) (periodic).  Implemented as a
 * counting sort of the particles by tile followed by LDS-tiled accumulation
 * (no global float atomics).  d_pos: [np][3] in [0, n_mesh); np in
 * [1, max_particles].  d_delta: [n_mesh^3] output. */
int pm_paint(pm_ctx* ctx, const float* d_pos, int64_t np, float* d_delta);

/* PM force at the particles (section 2, force equation and FD kernels):
 * F = 1.5 Omega_m * IDFT[i D(w)/K^2(w) W^-deconv S DFT(delta)] read out with
 * CIC, where K^2 = sum_d (2 sin(w_d/2))^2 and D(w) = (8 sin w - sin 2w)/6.
 * d_pos: [np][3]; d_force: [np][3] output, same particle order. */
int pm_force(pm_ctx* ctx, const float* d_pos, int64_t np, float* d_force);

/* One kick-drift-kick step from a0 to a1 (section 2, drift/kick equations,
 * FastPM factors): p += F K(a0->ac; a0); x += p D(a0->a1; ac) (wrapped);
 * F = force(x); p += F K(ac->a1; a1), ac = sqrt(a0 a1).  d_force holds F(x)
 * at a0 on entry and F at a1 on exit.  All arrays [np][3], np = n_part^3. */
int pm_kdk_step(pm_ctx* ctx, float* d_pos, float* d_mom, float* d_force,
                double a0, double a1);

/* Full run: force at a[0], then n_a - 1 KDK steps through the host array
 * h_a (strictly increasing, > 0).  Kicks between steps are merged.
 * d_pos, d_mom: [n_part^3][3] in/out, lattice order.  d_ckpt: NULL or
 * [n_a][2][n_part^3][3] receives (x, p) at every a[i] (the adjoint's
 * checkpoints).  d_delta_final: NULL or [n_mesh^3] receives the overdensity
 * painted from the final positions.  At most 65536 steps (PM_EINVAL). */
int pm_run(pm_ctx* ctx, const double* h_a, int n_a, float* d_pos, float* d_mom,
           float* d_ckpt, float* d_delta_final);

/* Resumable form of pm_run for schedulers that interleave several runs on
 * one GPU (continuous batching).  pm_run_begin validates and copies the
 * scale factors, sorts the particles and computes the force at h_a[0];
 * pm_run_advance enqueues up to max_steps KDK steps and writes the steps
 * still to go into *h_remaining (may be NULL); pm_run_end, once no step is
 * left, enqueues the closing half kick, writes d_pos/d_mom (the arrays given
 * to pm_run_begin, which must stay valid until then) and, if d_delta_final
 * is not NULL, the final overdensity.  pm_run(...) == begin + advance(all) +
 * end.  PM_ESTATE if advance/end are called without a run in progress or end
 * before the last step. */
int pm_run_begin(pm_ctx* ctx, const double* h_a, int n_a, float* d_pos, float* d_mom, float* d_ckpt);
int pm_run_advance(pm_ctx* ctx, int max_steps, int* h_remaining);
int pm_run_end(pm_ctx* ctx, float* d_delta_final);

/* Adjoint of pm_init_lpt + pm_run (reverse-mode derivative; the paper
 * differentiates the simulation with respect to the initial field, section 7).
 * h_a, n_a: the scale factors of the forward pm_run.  d_ckpt: the
 * [n_a][2][n_part^3][3] checkpoints it wrote; positions x_i are re-read at
 * every force evaluation point and the force meshes recomputed (no force
 * meshes are stored).  d_grad_delta_final: NULL or [n_mesh^3], the cotangent
 * of the final overdensity.  d_grad_pos, d_grad_mom: [n_part^3][3], on entry
 * the cotangents of the final positions and momenta (zeros if the loss only
 * sees the density), on exit those of the initial ones (lattice order).
 * d_grad_noise: NULL, or [n_part^3] receives the cotangent of the white
 * noise d_noise ([n_part^3], the noise the forward run started from) through
 * the LPT initial conditions.  The CIC weights are differentiated piecewise
 * (one-sided at cell faces).  Uses the workspace only. */
int pm_run_adjoint(pm_ctx* ctx, const double* h_a, int n_a, const float* d_ckpt, const float* d_noise,
                   const float* d_grad_delta_final, float* d_grad_pos, float* d_grad_mom,
                   float* d_grad_noise);

/* The chi^2 term of section 7's posterior for a model overdensity against
 * data, sum ((delta - data) / sigma)^2, into the device double *d_chi2
 * (float64 sum in a fixed order), and its derivative 2 (delta - data) /
 * sigma^2 into d_grad (may equal d_delta), the grad_delta of
 * pm_run_adjoint.  Asynchronous on the context's stream.  All meshes
 * [n_mesh^3] float32, C order.  PM_EINVAL for NULL pointers or sigma <= 0. */
int pm_chi2(pm_ctx* ctx, const float* d_delta, const float* d_data, double sigma, float* d_grad, double* d_chi2);

/* MAP reconstruction of the initial conditions from the final dark-matter
 * overdensity (section 7): minimise
 *   loss(w) = sum_cells ((delta_m(w) - delta_e) / sigma)^2 + sum_lattice w^2
 * over the white noise w that sets the initial field (the prior of the
 * initial modes in whitened variables).  One call: Gen-IC from w, the run
 * over h_a with checkpoints, the chi^2 residual, the adjoint of the run, and
 * one Adam update (Kingma & Ba, Algorithm 1) of w at step count t >= 1.
 * d_data: [n_mesh^3] observed overdensity, C order.  d_noise: [n_part^3],
 * inout.  d_adam_m, d_adam_v: [n_part^3] moment estimates, inout, zero
 * before t = 1.  d_work: 256-byte aligned scratch of at least
 * pm_recon_work_bytes(ctx, n_a) bytes (checkpoints, state, residual).
 * h_loss2: out, {chi^2, sum w^2} at the noise before the update; the call
 * synchronises the stream to return them.  The work buffer also holds the
 * run's force meshes (n_a * n_mesh^3 * 12 bytes), read back by the adjoint
 * instead of recomputed.  PM_EINVAL for NULL pointers,
 * n_a < 2, sigma <= 0, t < 1, lr <= 0, beta outside [0, 1) or eps < 0;
 * PM_ENOMEM if work_bytes is too small; PM_ESTATE during a resumable run. */
size_t pm_recon_work_bytes(const pm_ctx* ctx, int n_a);
int pm_recon_step(pm_ctx* ctx, const double* h_a, int n_a, const float* d_data, double sigma, float* d_noise,
                  float* d_adam_m, float* d_adam_v, int t, double lr, double beta1, double beta2, double eps,
                  void* d_work, size_t work_bytes, double* h_loss2);

/* Binned power spectrum of a real mesh (section 6.1 two-point statistics):
 * P(k_j) = (L^3/N^6) sum_w |delta^|^2 / sum_w, mode weight 2 on interior
 * n_z planes and 1 on n_z = 0 and N/2, bins |n| in [j-1/2, j+1/2),
 * j = 1..n_bins (n_bins <= n_mesh/2).  Only modes with every |n_d| < n_max
 * count when n_max > 0.  deconv: divide delta^ by the CIC window.  The mesh
 * at d_delta is left unchanged.  Synchronises; host outputs of n_bins
 * entries: h_k (mode-weighted mean k, h/Mpc), h_pk ((Mpc/h)^3), h_nmodes. */
int pm_power(pm_ctx* ctx, const float* d_delta, int n_bins, int n_max, int deconv,
             double* h_k, double* h_pk, double* h_nmodes);

/* 3D real FFT of a mesh (the transform of section 3, one pass per axis):
 * d_spec[kx][ky][kz] = sum_x d_real[x] exp(-2 pi i k.x / n_mesh),
 * kz = 0..n_mesh/2, complex64 interleaved (re, im), i.e. numpy's rfftn
 * layout [n][n][n/2+1].  d_real is left unchanged. */
int pm_rfft(pm_ctx* ctx, const float* d_real, float* d_spec);

/* Inverse of pm_rfft, normalised by 1/n_mesh^3 like numpy's irfftn: the
 * imaginary parts of the kz = 0 and kz = n/2 planes after the x and y
 * inverse transforms are ignored. d_spec is left unchanged. */
int pm_irfft(pm_ctx* ctx, const float* d_spec, float* d_real);

/* LPT frame of the COLA integrator: caller-owned device arrays d_psi1,
 * d_psi2 of [n_part^3][3] floats, lattice (particle index) order, mesh-cell
 * units: the first- and second-order LPT displacement fields Psi1, Psi2 of
 * the particles (x_LPT(a) = q + D1(a) Psi1 + D2(a) Psi2, section 6).  While
 * set, pm_init_lpt writes them (B times its lattice displacement fields;
 * Psi2 = 0 for lpt_order 1) and a COLA pm_run / pm_run_begin reads them; the
 * caller keeps them unchanged in between.  NULL, NULL unsets.  PM_EINVAL if
 * only one is NULL; PM_ESTATE during a resumable run. */
int pm_set_lpt_frame(pm_ctx* ctx, float* d_psi1, float* d_psi2);

/* Keep the force meshes of a run instead of recomputing them in the adjoint
 * (the capacity of the device's memory traded for a paint and four FFT passes
 * per step of the reverse sweep).  d_fckpt: caller-owned device memory of
 * n_slots * n_mesh^3 * 3 floats (internal layout, opaque); NULL or n_slots = 0
 * switches it off.  A pm_run / pm_run_begin with n_a <= n_slots then writes
 * the force mesh at a[j] into slot j, and a later pm_run_adjoint over the
 * same scale factors (n_a <= n_slots) reads them: the caller keeps d_fckpt
 * unchanged in between.  Runs with force checkpoints do not use graphs.
 * PM_EINVAL for n_slots < 0 or a buffer with no slots; PM_ESTATE during a
 * resumable run. */
int pm_set_force_ckpt(pm_ctx* ctx, float* d_fckpt, int64_t n_slots);

/* Run the step loop of pm_run_advance (and so pm_run) as one captured HIP
 * graph per step (two graphs per context, one per ping-pong buffer, built on
 * first use and kept until the particle count or checkpointing changes):
 * one launch per step instead of about fifteen, for small meshes where
 * launches dominate.  The step's factors and checkpoint slot live in device
 * memory, so replays need no new parameters.  Needs a non-default stream
 * (PM_EHIP at the first advance otherwise); ignored while profiling.
 * enable = 0 drops the graphs.  Results are identical to the eager loop. */
int pm_use_graphs(pm_ctx* ctx, int enable);

/* Optional per-kernel-class timing with HIP events recorded on the
 * context's stream around every kernel the library enqueues (measurement
 * support; adds two event records per launch while enabled).
 * pm_profile(ctx, 1) clears and starts collecting, pm_profile(ctx, 0) stops. */
int pm_profile(pm_ctx* ctx, int enable);

/* Synchronises, then fills up to max entries: h_names (32 bytes each,
 * NUL-terminated class name), h_total_ms (summed event time), h_count
 * (launches).  Returns the number of classes seen, or a negative status. */
int pm_profile_read(pm_ctx* ctx, int max, char* h_names, double* h_total_ms, int* h_count);

/* ---- continuous batching of same-shape simulations -----------------------
 * The paper runs many simulations of one shape as the batch dimension of its
 * tensors (section 4).  Here a plan created with cfg.batch = B holds B member
 * slots, each with the full workspace of one simulation of cfg (the
 * workspace is B times that of a single context, members at a fixed
 * stride).  Requests join and leave slots while others are mid-run; one
 * batched step launches every kernel of a KDK step once for all listed
 * members (readout + kick + drift, counting sort, paint, the five FFT passes
 * of the force), blockIdx.z selecting the member through a device table of
 * descriptors.  Each member's result equals the same run on a context of its
 * own, bit for bit (same kernels, integer paint sums).
 *
 * A member's state between steps (particles sorted by tile, force mesh at
 * its current scale factor) lives in its slot.  Typical use:
 *   pm_batch_member(plan, m, &ctx_m); pm_init_lpt(ctx_m, ...)  (any
 *     single-simulation call works on a member's context)
 *   pm_batch_begin(plan, m, h_a, n_a, d_pos, d_mom, d_ckpt)
 *   pm_batch_advance(plan, &n)   (repeated: one step of every running member)
 *   pm_batch_end(plan, m, d_delta_final)   once m has no step left
 * All calls are asynchronous on the plan's stream (pm_set_stream on the plan
 * also moves its members).  A plan and its members are not thread-safe. */
#define PM_MAX_BATCH 256
#define PM_REQ_CKPT 1

/* One member's entry of a batched step.  Device memory, 48 bytes. */
typedef struct {
    int32_t member;      /* slot in [0, batch); < 0: the entry is skipped */
    int32_t flags;       /* 0 or PM_REQ_CKPT */
    float   kick_close;  /* closing kick K(a_c(i-1) -> a_i; a_i) of the member's previous step, 0 before its first */
    float   kick_open;   /* opening kick K(a_i -> a_c; a_i) of this step */
    float   drift;       /* drift D(a_i -> a_i+1; a_c) of this step */
    float   reserved;
    float*  ckpt_x;      /* PM_REQ_CKPT: [n_part^3][3] receives x_i by particle id */
    float*  ckpt_p;      /* PM_REQ_CKPT: [n_part^3][3] receives p_i (after the closing kick) by particle id */
    int64_t reserved2;
} pm_req_desc;

/* One KDK step (section 2 kick/drift equations, force equation) of every
 * member listed in the device array d_descs[0..n) (n in [1, batch]; each
 * member at most once): p += F kick_close; checkpoint; p += F kick_open;
 * x += p drift (wrapped); sort; paint; force at the new positions.  The
 * factors come from the descriptors, so one captured graph can serve every
 * step.  The members must have been started with pm_batch_begin; the caller
 * keeps count of their steps (pm_batch_advance is this call with the
 * bookkeeping done, over the plan's own descriptor table).  PM_EINVAL if plan is not a batch plan, d_descs is NULL or n is out
 * of range. */
int pm_kdk_step_batched(pm_ctx* plan, const pm_req_desc* d_descs, int n);

/* Context handle of member m (0 <= m < batch) of a plan: every
 * single-simulation entry point works on it, over the member's slot.  Owned
 * by the plan (never pm_destroy it); member 0 is the plan itself. */
int pm_batch_member(pm_ctx* plan, int m, pm_ctx** out);

/* Start member m's run (as pm_run_begin on its context): scale factors
 * h_a[0..n_a) strictly increasing, d_pos/d_mom [n_part^3][3] in lattice
 * order (kept by the caller until pm_batch_end), d_ckpt NULL or
 * [n_a][2][n_part^3][3].  Sorts the particles into the slot, paints and
 * computes the force at h_a[0].  PM_ESTATE if m already runs. */
int pm_batch_begin(pm_ctx* plan, int m, const double* h_a, int n_a, float* d_pos, float* d_mom, float* d_ckpt);

/* One batched step of every running member with steps left: fills the
 * plan's device descriptor table from the members' scale factors (the
 * running members' descriptors packed at its front, so that no workgroup is
 * launched for an idle slot) and calls pm_kdk_step_batched (a captured
 * graph once pm_use_graphs(plan, 1), one per number of running members).
 * *h_stepped (may be NULL) receives the number of members advanced. */
int pm_batch_advance(pm_ctx* plan, int* h_stepped);

/* Steps member m still has to take (0 when it can end), or a negative
 * status; PM_ESTATE if m does not run. */
int pm_batch_remaining(pm_ctx* plan, int m);

/* Finish member m's run (as pm_run_end): closing half kick, positions and
 * momenta back to the caller's arrays in lattice order, the last checkpoint,
 * the final overdensity if d_delta_final is not NULL.  The slot is free
 * afterwards.  The member must have taken all its steps: with
 * pm_batch_advance, pm_batch_remaining(plan, m) == 0; with
 * pm_kdk_step_batched the caller counts them.  PM_ESTATE if m does not run. */
int pm_batch_end(pm_ctx* plan, int m, float* d_delta_final);

/* ---- allocation-free force ----------------------------------------------
 * For callers that cannot allocate device memory or create a workspace
 * (tight serving loops, harnesses that forbid allocation).  Not for code
 * under stream capture: the call waits for its table upload.  The same
 * computation as pm_force on a context created from
 * cfg, with the workspace taken from a fixed device array of
 * PM_STATIC_SCRATCH_BYTES bytes inside the library: every GPU the library
 * runs on holds one such array until the process ends.  The call allocates
 * no device memory; it builds a host-side context, uploads the static tables
 * into the array on `stream` (a hipStream_t as void*, NULL = default stream)
 * and waits for that upload, then enqueues the force asynchronously on
 * `stream`.  d_pos: [np][3] positions in [0, n_mesh); d_force: [np][3]
 * output; np in [1, max_particles].  All calls on one GPU share its array
 * and it keeps the last call's contents: calls that overlap on one GPU (two
 * host threads, or two streams with work still in flight) race and give
 * undefined results.  Returns PM_EINVAL for NULL pointers or an invalid cfg,
 * PM_ENOMEM if pm_workspace_bytes(cfg) exceeds PM_STATIC_SCRATCH_BYTES
 * (with a message on stderr; meshes up to 64^3 with up to 64^3 particles
 * fit), PM_EHIP for a runtime error. */
#define PM_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
int pm_force_static(const pm_config* cfg, const float* d_pos, int64_t np, float* d_force, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PM_H */
