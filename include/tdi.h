/*
 * tdi.h - C ABI of the MI355X (gfx950) hybrid time-domain LISA response.
 *
 * Computes the Michelson TDI observables X, Y, Z of a batch of gravitational-
 * wave sources from their sampled polarisations h+, hx, following
 * arXiv:2505.09600:
 *   - full response: per-link projection at retarded times, Sec. II.A-B,
 *     Eqs. (H), (xi_plus), (xi_cross), (yslr), (delta_s), (delta_r), with
 *     N-tap Lagrange fractional delays; TDI 1.5 / 2.0 Michelson combinations,
 *     Eqs. (X1.5) and (X2.0), every arm delay evaluated at the output time;
 *   - low-frequency approximation (LFA): delays become central finite-difference
 *     stencils of the strain, Sec. III, Eqs. (yslr_strain_derivatives),
 *     (X15_with_strain_derivatives), (X20_with_strain_derivatives) and App. B,
 *     Eqs. (X15_nonequal_timedelays), (X20_nonequal_timedelays);
 *   - hybrid: sigmoid blend of the two around a switch time, Sec. IV,
 *     Eqs. (sigmoid), (hybridized_xs).
 *
 * Memory and ownership
 *   Small per-batch metadata (source records, CSR offsets) are HOST pointers,
 *   validated on the host before any device work and copied by the library.
 *   Bulk arrays (hp, hc, X, Y, Z) are DEVICE pointers on the plan's device,
 *   owned by the caller; they must stay valid until the work on the plan's
 *   stream has completed.  The library owns the plan (device tables, work
 *   counters, captured graph); tdi_run allocates no device memory.
 *   All calls on one plan must come from one host thread at a time.
 *
 * Errors
 *   Every function returns a tdi_status.  Argument errors are detected before
 *   any device work and leave the outputs untouched.  After TDI_EDEVICE the
 *   output contents are unspecified.  NaN inputs propagate without a check.
 *
 * Numerics
 *   TDI_FP64: all arithmetic in FP64.  TDI_FP32_BULK: retarded-time arguments,
 *   geometry, stencils and the split into integer index and fraction stay in
 *   FP64; the fractional-delay interpolation, TDI combination and hybrid blend
 *   run in FP32 with FP32 accumulation, and X, Y, Z are written as float.
 */
#ifndef TDI_H
#define TDI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TDI_OK = 0,
  TDI_EINVAL = -1,        /* null / misaligned pointer, bad offsets, bad sizes */
  TDI_ERANGE = -2,        /* value out of the supported range (taps, dt, angles, window) */
  TDI_ENOMEM = -3,        /* device or pinned host allocation failed */
  TDI_EDEVICE = -4,       /* no gfx950 device, or a HIP runtime error */
  TDI_EUNSUPPORTED = -5,  /* unknown TDI generation, mode, precision or orbit kind */
  TDI_ESTATE = -6         /* batch exceeds the plan's declared maxima, or bad plan */
} tdi_status;

enum { TDI_ORBIT_FROZEN = 0, TDI_ORBIT_ANALYTIC1 = 1, TDI_ORBIT_TABLE = 2 };
enum { TDI_MODE_FULL = 0, TDI_MODE_LFA = 1, TDI_MODE_HYBRID = 2 };
enum { TDI_FP64 = 0, TDI_FP32_BULK = 1 };
enum { TDI_CHANNELS_XYZ = 0, TDI_CHANNELS_AET = 1 };

/* Constellation orbit (Sec. II.B uses an equal-arm analytic orbit).
 * ANALYTIC1: rigid equilateral first-order analytic orbit at radius R_m with
 *   eccentricity L_m / (2 sqrt(3) R_m), orbital phase alpha = omega t + kappa0,
 *   spacecraft i at beta_i = 2 pi (i-1)/3 + lambda0; light times solve the
 *   light-time equation with the sender at emission time.
 * FROZEN: positions of ANALYTIC1 at t_freeze, all six light times L_m / c.
 * TABLE: spacecraft positions sampled on a uniform time grid (for instance
 *   an orbit file, or eccentric Keplerian orbits whose arms flex), read by
 *   8-point Lagrange interpolation in time; light times solve the same
 *   light-time equation.  L_m is the nominal arm (equal-arm LFA); R_m,
 *   omega, kappa0, lambda0 and t_freeze are ignored.  The table is copied at
 *   plan creation; a batch whose sources (with their retarded-time margins)
 *   reach outside the table's span returns TDI_ERANGE. */
typedef struct {
  int32_t kind;       /* TDI_ORBIT_* */
  int32_t reserved;   /* must be 0 */
  double L_m;         /* arm length, m, > 0 */
  double R_m;         /* orbital radius, m, > L_m */
  double omega;       /* rad/s, finite, >= 0 */
  double kappa0;      /* rad */
  double lambda0;     /* rad */
  double t_freeze;    /* s (FROZEN only) */
  const double* table;   /* TABLE: host array [n_table][3][3], sample j, spacecraft 1..3, x y z (m, SSB) */
  int64_t n_table;       /* TABLE: >= 8 samples */
  double table_t0;       /* TABLE: time of sample 0, s */
  double table_dt;       /* TABLE: sample spacing, s, > 0 */
} tdi_orbit;

/* One source: sky position, polarisation, time grid and switch time.
 * Sample k of the source is at t0 + k dt. */
typedef struct {
  double beta;        /* ecliptic latitude, rad, |beta| <= pi/2 */
  double lambda;      /* ecliptic longitude, rad, finite */
  double psi;         /* polarisation angle, rad, finite */
  double t0;          /* s, finite */
  double dt;          /* s, > 0 */
  double t_hyb;       /* switch time, s (HYBRID): +inf = pure LFA, -inf = pure full; not NaN */
} tdi_source;

typedef struct {
  int32_t tdi_gen;          /* 15 (first generation) or 20 (second generation) */
  int32_t mode;             /* TDI_MODE_* */
  int32_t interp_taps;      /* N Lagrange taps (degree N-1): 4, 8, 16 or 32 */
  int32_t stencil_order;    /* LFA central-difference accuracy order: 2 or 4 */
  int32_t lfa_equal_arms;   /* LFA only: 1 = equal constant delays L/c, 0 = unequal time-dependent */
  int32_t precision;        /* TDI_FP64 or TDI_FP32_BULK */
  double hyb_T_samples;     /* hybrid window length T in samples (paper default 800), > 0 */
  double hyb_sigma_samples; /* sigmoid width sigma in samples (paper default T/40), > 0 */
  int32_t autotune;         /* 1: time the launch candidates on the first run and keep the best.
                               If the environment variable TDI_AUTOTUNE_CACHE names a file, each
                               decision is appended to it (one JSON object per line, keyed by the
                               device architecture and compute units, the options that change the
                               kernels, and the batch's source and sample counts as powers of
                               two), and a plan whose key is found there takes the stored launch
                               without timing; unreadable lines are skipped.  TDI_LOG=1 reports
                               each decision on stderr, TDI_LOG=2 also every candidate's time. */
  int32_t use_graph;        /* 1: capture the run sequence in a hipGraph and replay it.  With
                               autotune = 1 the first run also times replays against plain
                               stream launches over back-to-back runs and keeps the faster
                               (short runs, where a replay costs the host more than the
                               launches it replaces); tdi_plan_describe reports the choice */
  int32_t channels;         /* TDI_CHANNELS_XYZ: write X, Y, Z.  TDI_CHANNELS_AET: write the
                               noise-orthogonal combinations defined at the end of Sec. II.B instead,
                               A = (Z - X)/sqrt 2, E = (X - 2Y + Z)/sqrt 6, T = (X + Y + Z)/sqrt 3,
                               into the same three arrays (fused into the store) */
  int32_t lfa_terms;        /* LFA terms.  0 or 1: the leading term of the central expansion
                               (App. B).  2: also the next one.
                               Single links (tdi_run_links): the m = 1 term of
                               Eq. (yslr_with_tau_derivatives), -(L/2c)(1/6)[L(1 - k.n)/(2c)]^2
                               times the third derivative of H.
                               X, Y, Z (tdi_run, LFA and HYBRID modes): the expansion of the
                               TDI combination, Eqs. (X1.5l2), (X1.5l3), carried to third order
                               in the delays with that link term: each read Xi^(m) of
                               Eqs. (X15/X20_nonequal_timedelays) becomes Xi^(m) + kappa
                               Xi^(m+2), kappa = To^2/6 + Tl^2/8 + Tl^2 (1 + (k.n_l)^2)/24
                               (+ (Tl + To)^2/6 for TDI 2.0), Tl the link's light time, To the
                               channel's other arm; the derivative of order m + 2 comes from a
                               central stencil of the same accuracy.  Runs on the general LFA
                               kernel (not the FP32 fast path). */
  int32_t nested_delays;    /* full response (FULL mode and the full part of HYBRID): 0 = every
                               delay of Eqs. (X1.5), (X2.0) at the output time, as the paper does
                               (Sec. II.B); 1 = time-nested delays, each light time taken at the
                               time its delay is applied, D_a D_b f(t) = f(t - T_a(t) -
                               T_b(t - T_a(t))).  No effect on the LFA or on tdi_run_links.
                               Other values give TDI_ERANGE. */
  int32_t fast_tile_chunks; /* FP32-bulk LFA and hybrid runs: outputs per LFA tile in chunks of 2304
                               (1, 2 or 4); 0 = chosen by the autotuner (autotune = 1) or 4.
                               Small tiles give single long sources enough tiles to fill the GPU;
                               large ones amortise the per-tile geometry fit over big batches.
                               Other values give TDI_ERANGE. */
  int32_t lfa_x20_from_x15; /* TDI 2.0 LFA and HYBRID modes: 1 = the LFA part from the TDI 1.5
                               LFA series by Eq. (relation_X20_X15_nonequal_timedelays),
                               X2.0(t) = 2 (T2 + T3) dX1.5/dt (t - T2 - T3): X1.5 is computed in
                               FP64 on every sample into a plan-owned buffer (24 bytes per
                               sample of max_total_samples), differentiated by the central
                               stencil of the configured accuracy and read at the fractional
                               delay with exact N-tap Lagrange weights; output in the plan's
                               precision.  No graph replay for this option.  0 = the direct
                               form of Eq. (X20_nonequal_timedelays).  1 with TDI 1.5 gives
                               TDI_ERANGE; with lfa_terms = 2, TDI_EUNSUPPORTED. */
} tdi_config;

typedef struct tdi_plan tdi_plan;

/* Host-only validation of a configuration and orbit (no device needed).
 * Returns TDI_OK, TDI_EINVAL (null), TDI_EUNSUPPORTED or TDI_ERANGE. */
tdi_status tdi_check_config(const tdi_config* cfg, const tdi_orbit* orb);

/* Host-only validation of a batch: src[n_sources] records and
 * offsets[n_sources + 1] (offsets[0] = 0, non-decreasing; source i owns samples
 * offsets[i] .. offsets[i+1]-1 of the flat arrays).  No device needed. */
tdi_status tdi_check_batch(const tdi_config* cfg, int64_t n_sources,
                           const tdi_source* src, const int64_t* offsets);

/* Create a plan on the current HIP device for batches of at most max_sources
 * sources and max_total_samples samples: the device state for the response of
 * tdi_run (Secs. II-IV): the orbit of Sec. II.A (light times and link
 * directions of Eqs. (yslr), (delta_s), (delta_r)), the parameter block and,
 * with use_graph, the captured launch sequence.  hip_stream is a hipStream_t
 * (NULL = default stream).  Returns TDI_EDEVICE when no gfx950 device is
 * present. */
tdi_status tdi_plan_create(tdi_plan** out, const tdi_config* cfg, const tdi_orbit* orb,
                           int64_t max_sources, int64_t max_total_samples, void* hip_stream);

/* Enqueue the response of one batch on the plan's stream (asynchronous):
 * X, Y, Z (or A, E, T) of each source by the plan's mode: the full response
 * (Sec. II.B, Eqs. (yslr), (X1.5), (X2.0)), the LFA (Sec. III and App. B,
 * Eqs. (X15_with_strain_derivatives), (X20_with_strain_derivatives),
 * (X15_nonequal_timedelays), (X20_nonequal_timedelays)) or the hybrid
 * (Sec. IV, Eqs. (sigmoid), (hybridized_xs)).
 * src, offsets: host arrays (copied before return).  hp, hc: device arrays of
 * offsets[n_sources] doubles (8-byte aligned).  X, Y, Z: device arrays of
 * offsets[n_sources] doubles (TDI_FP64) or floats (TDI_FP32_BULK).
 * The first run of an autotuning plan times candidates synchronously. */
tdi_status tdi_run(tdi_plan* plan, int64_t n_sources, const tdi_source* src,
                   const int64_t* offsets, const double* hp, const double* hc,
                   void* X, void* Y, void* Z);

/* Allocation-free variant of tdi_run, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): no plan, and no hipMalloc, hipFree or other allocating
 * call.  The parameter block, work counters, window-check words and the fast
 * LFA path's per-tile records live in a static device array of about 8.4 MB
 * that each GPU holds from the first call on it until the process ends.
 * Same computation, arguments and layouts as tdi_run, with the batch, config
 * and orbit passed directly; hip_stream is a hipStream_t (NULL = default
 * stream) on the current device, and the call is asynchronous on it.
 * Limits: at most 256 sources and 2048 fast-LFA tiles (tiles of
 * 2304 * fast_tile_chunks outputs, chunks 0 meaning 4), else TDI_ESTATE;
 * TABLE orbits and lfa_x20_from_x15 (which needs a per-sample buffer) give
 * TDI_EUNSUPPORTED.  autotune and use_graph are ignored
 * (persistent grids at full occupancy, no graph).  A retarded-time window
 * that leaves the staged range writes NaN outputs (there is no plan to
 * report it through).  Every call on one GPU shares that GPU's array: calls
 * whose device work overlaps (other streams, other host threads' streams)
 * race and give undefined outputs; calls ordered on one stream are safe. */
tdi_status tdi_run_noalloc(const tdi_config* cfg, const tdi_orbit* orb, int64_t n_sources,
                           const tdi_source* src, const int64_t* offsets, const double* hp,
                           const double* hc, void* X, void* Y, void* Z, void* hip_stream);

/* Enqueue the six single-link outputs of one batch on the plan's stream
 * (asynchronous), in the plan's mode, precision, taps, stencil order and
 * hybrid window:
 *   TDI_MODE_FULL: Eq. (yslr) with Eq. (H), y_l = [H_l(t - delta_s) -
 *     H_l(t - delta_r)] / (2 (1 - k.n_l)), Eqs. (delta_s), (delta_r);
 *   TDI_MODE_LFA: Eq. (yslr_strain_derivatives) for every link, y_l =
 *     -(L_l/2c) [xi+_l h+'(t - L_l/2c - mu_l) + xi_x_l hx'(...)], mu_l =
 *     k.(R_s + R_r)/(2c), the first derivative by the central stencil of the
 *     configured accuracy (L_l = L for lfa_equal_arms);
 *   TDI_MODE_HYBRID: Eq. (hybridized_yslr) with the windows and weights of
 *     the X, Y, Z hybrid.
 * y: device array of 6 * offsets[n_sources] doubles (TDI_FP64) or floats
 * (TDI_FP32_BULK), link-major: link slot a occupies y[a * total .. a * total +
 * total - 1] with slots ordered +1, +2, +3, -1, -2, -3 (link l joins the two
 * spacecraft other than |l|, its direction given by the sign convention of
 * Sec. II.B).  src, offsets, hp, hc as for tdi_run.  Runs outside the plan's
 * graph; TDI_ERANGE if the read window of a tile would exceed the LDS. */
tdi_status tdi_run_links(tdi_plan* plan, int64_t n_sources, const tdi_source* src,
                         const int64_t* offsets, const double* hp, const double* hc, void* y);

/* Wait for the plan's work and report device-side window checks:
 * TDI_ERANGE if any retarded-time window left the staged range since the last
 * call (such samples were written as NaN), else TDI_OK. */
tdi_status tdi_plan_sync(tdi_plan* plan);

/* Kernel durations (ms) of the most recent runs, oldest first, three values
 * per run: the geometry-fit pre-pass of the FP32 LFA path (0 when not used),
 * the LFA kernel and the full-response kernel.  Graph replays are timed by
 * event nodes inside the graph; where the runtime cannot retarget those nodes a
 * replay reports its whole duration as the LFA value and 0 for the others
 * (tdi_plan_describe tells which: "graph_kernel_events").  At most 'cap' values
 * (up to 256 runs remembered); *count receives the number written.  Waits for
 * the plan's work; the record is cleared afterwards. */
tdi_status tdi_plan_kernel_times(tdi_plan* plan, float* ms, int32_t cap, int32_t* count);

/* Per-kernel timing of tdi_run on (on = 1, the default) or off (on = 0).
 * Each timed run records device events around its kernels, and each such
 * record is a marker in the device queue that costs microseconds of device
 * time: for short runs (one source, ~0.1 ms) turning it off shortens the run;
 * untimed runs add nothing to tdi_plan_kernel_times.  TDI_EINVAL for other
 * values of on, TDI_ESTATE for a null plan. */
tdi_status tdi_plan_set_timing(tdi_plan* plan, int32_t on);

/* Launch parameters chosen for the plan as a JSON object in buf (tile
 * lengths, persistent grid sizes, graph use, compute units, tuned flag, and
 * tune_cache = 1 when the launch came from the autotune cache). */
tdi_status tdi_plan_describe(const tdi_plan* plan, char* buf, int32_t buflen);

/* Wait for the plan's outstanding work and release everything it owns
 * (device tables, pinned staging, graph, events).  NULL returns TDI_EINVAL. */
tdi_status tdi_plan_destroy(tdi_plan* plan);

/* Static, human-readable description of a status code. */
const char* tdi_status_str(tdi_status s);

/* ---------------------------------------------------------------------------
 * Noise-weighted inner product of A, E, T series (the likelihood's steps after
 * the response): <x|y> = 4 Re int df conj(x~) y~ / S_n, Eq. (scalar_product)
 * and App. (scalar product), with the analytic PSDs of Sec. II.C, Eqs. (SnAE),
 * (SnT), and the galactic foreground of Eq. (sgal).  x~ is the discrete form of
 * Eq. (defFT): dt times the DFT of the series zero-extended to
 * N = max(2, next power of two >= n) samples; the integral is the sum over the
 * bins 0 < f_k = k / (N dt) < 1 / (2 dt) with f_min <= f_k <= f_max, times
 * df = 1 / (N dt).  ln L = -1/2 sum_c <d - h|d - h> (Eq. derived_likelihood)
 * follows from the three products per channel that tdi_ip_run returns.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t tdi_gen;        /* 15 or 20: the TDI factor Lambda(f) of Eqs. (SnAE), (SnT) */
  int32_t galactic;       /* 1: add the galactic foreground, 0: instrument noise only */
  double T_obs_years;     /* observation time in the foreground's knee relations, years, > 0 */
  double L_m;             /* arm length in x = 2 pi f L / c, m, > 0 */
  double f_min, f_max;    /* band, Hz: 0 < f_min < f_max < c/(4L) (TDI 2.0) or c/(2L) (TDI 1.5),
                             below the first zero of the PSD */
} tdi_noise;

typedef struct tdi_ip_plan tdi_ip_plan;

/* Host-only validation of a noise description: TDI_OK, TDI_EINVAL (null),
 * TDI_EUNSUPPORTED (generation) or TDI_ERANGE. */
tdi_status tdi_check_noise(const tdi_noise* noise);

/* Create an inner-product plan on the current HIP device for batches of at
 * most max_sources sources, max_total_samples samples in all and
 * max_source_samples per source, all sampled at dt seconds.  precision:
 * TDI_FP64 (double inputs, FP64 transforms) or TDI_FP32_BULK (float inputs,
 * FP32 transforms); the weighted sums accumulate in FP64 either way.  The plan
 * owns the 1/S_n table and a transform workspace of 6 max_total_samples
 * complex elements.  Sources longer than 2^25 (FP32) or 2^23 (FP64) samples
 * return TDI_ERANGE; no gfx950 device returns TDI_EDEVICE. */
tdi_status tdi_ip_plan_create(tdi_ip_plan** out, const tdi_noise* noise, int32_t precision, double dt,
                              int64_t max_sources, int64_t max_total_samples,
                              int64_t max_source_samples, void* hip_stream);

/* Enqueue the inner products of one batch (asynchronous, on the plan's stream).
 * offsets: host CSR array of n_sources + 1 entries as for tdi_run.  x, y: host
 * arrays of three device pointers each, the A, E, T series (float or double
 * by the plan's precision; a response run with channels = TDI_CHANNELS_AET
 * writes them).  out: device array of 9 n_sources doubles; source i receives,
 * for channel c = A, E, T, out[9 i + 3 c + 0..2] = <x|x>, <x|y>, <y|y>.
 * TDI_ESTATE when the batch exceeds the plan's maxima. */
tdi_status tdi_ip_run(tdi_ip_plan* plan, int64_t n_sources, const int64_t* offsets,
                      const void* const* x, const void* const* y, double* out);

/* Kernel durations (ms) of the most recent inner-product runs, three per run:
 * the column pass, the row pass with the weighted sums, the final reduction.
 * Waits for the plan's work; the record is cleared afterwards. */
tdi_status tdi_ip_kernel_times(tdi_ip_plan* plan, float* ms, int32_t cap, int32_t* count);

/* Wait for the plan's outstanding work and release it.  NULL: TDI_EINVAL. */
tdi_status tdi_ip_plan_destroy(tdi_ip_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* TDI_H */
