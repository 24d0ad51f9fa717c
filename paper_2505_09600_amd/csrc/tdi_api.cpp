// Host runtime and C ABI of the hybrid time-domain LISA response (include/tdi.h).
//
// Responsibilities: argument validation (host only, before any device work),
// plan construction (device parameter block, launch shape, optional hipGraph),
// per-run upload of the small source table, kernel launches and timing
// records.  No response arithmetic runs here; it is all in tdi_kernels.hip.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "../../include/tdi.h"
#include "tdi_internal.h"

namespace {

constexpr double kC = 299792458.0;
constexpr int kEventRing = 256;
constexpr int kEvPerRun = 4;
constexpr size_t kCtrBytes = 256;     // counters in front of a parameter block     // before the fit pre-pass, before / after the LFA kernel, after the full kernel

struct Launch {
  int grid_lfa;      // 0 = one workgroup per tile
  int grid_full;
  int chunks;        // fast LFA path: chunks of kFastChunk outputs per tile (1, 2 or 4)
};

struct OrbitBounds {
  double rate, tmax, tmin, rmax;
};

struct Caps {
  int g, hl, hf, y;
  size_t lds_lfa, lds_full;
  int goff;
  int fast;          // FP32 bulk LFA kernel
  int nx;            // LFA with the next term (general LFA kernel)
  int tile_lfa;      // outputs per LFA tile
  int hyb;           // HYBRID mode: term-parallel full-response kernel
  int fit_cu;        // fast path: resident pre-pass workgroups per CU (its grid-stride grid)
};

}  // namespace

struct tdi_plan {
  tdi_config cfg;
  tdi_orbit orb;                 // the table pointer of a TABLE orbit is not kept
  OrbitBounds ob;
  double* d_orbtab;              // TABLE: device copy of the sampled positions
  int64_t max_sources, max_total;
  int device, n_cu;
  char arch[64];                 // device architecture name (autotune cache key)
  size_t max_lds;                // LDS bytes available to one workgroup
  int last_fast, last_tile_lfa;  // LFA kernel choice of the latest run
  int last_tile_full;            // full-response tile of the latest run
  hipStream_t user_stream;
  hipStream_t graph_stream;      // private stream used for capture and replay
  // device memory
  tdi::KParams* d_params;        // KParams followed by SrcDev[max_sources]
  void* d_ftiles;                // fast LFA path: per-tile records of the pre-pass
  int64_t fit_tiles;             // their capacity (tiles)
  size_t params_bytes;
  int32_t* d_err;
  // parameter blocks are allocated with kCtrBytes in front for the work
  // counters of the persistent kernels; the upload of each run copies that
  // prefix as zeros, so no separate reset is launched
  unsigned char* d_block;
  unsigned char* h_block;        // the staging image in use (one of h_blk)
  unsigned char* d_block15;
  unsigned char* h_block15;
  // TDI 2.0 LFA from TDI 1.5: the FP64 TDI 1.5 LFA series and its own parameter block
  double* d_x15;
  tdi::KParams* d_params15;
  tdi::KParams* h_params15;
  tdi_config cfg15;
  // pinned staging image of the parameter block
  tdi::KParams* h_params;        // its parameter block
  // two pinned staging images, used in turn, so that the host stages run i + 1
  // while the device still runs run i; an image is rewritten only after the
  // work that uploaded it has completed (its event)
  unsigned char* h_blk[2];
  tdi::KParams* h_par[2];
  hipEvent_t stage_ev[2];
  bool stage_pending[2];
  int stage_slot;                // slot of the next run
  bool double_buffer;            // false if the graph's upload node cannot be retargeted
  hipGraphNode_t graph_mnode;    // the upload (memcpy) node of the graph
  hipEvent_t staged_free;        // recorded after the work of the latest run
  hipEvent_t handoff;            // orders the private stream after the caller's
  bool staged_pending;           // (x15 pass image; see stage_ev for the main images)
  // launch choice
  Launch launch;
  bool tuned;
  bool tune_cached;              // the launch came from the autotune cache file
  bool stream_pick;              // the autotuner found stream launches faster than graph replay
  bool timing;                   // runs record the per-kernel events (tdi_plan_set_timing)
  // graph
  hipGraph_t graph;
  hipGraphExec_t graph_exec;
  Launch graph_launch;
  size_t graph_lds_lfa, graph_lds_full;
  int graph_fast;
  hipGraphNode_t graph_ev_node[kEvPerRun];   // event records around the kernels inside the graph
  bool graph_timed;                  // those nodes are retargeted to the timing ring per replay
  // kernel nodes of the graph (fit pre-pass, LFA, full; null if absent), their
  // captured parameters and the grid each replay last used: every replay trims
  // the persistent grids to the batch's tile counts
  hipGraphNode_t graph_knode[3];
  hipKernelNodeParams graph_kparams[3];
  unsigned graph_kgrid[3];
  // timing: per recorded run, events before the fit pre-pass, before and after
  // the LFA kernel and after the full kernel
  hipEvent_t ev[kEventRing][kEvPerRun];
  int ev_count, ev_head;
};

extern "C" {

const char* tdi_status_str(tdi_status s) {
  switch (s) {
    case TDI_OK: return "ok";
    case TDI_EINVAL: return "invalid argument";
    case TDI_ERANGE: return "value out of range";
    case TDI_ENOMEM: return "out of memory";
    case TDI_EDEVICE: return "device error or no gfx950 device";
    case TDI_EUNSUPPORTED: return "unsupported option";
    case TDI_ESTATE: return "bad plan state or batch exceeds plan maxima";
  }
  return "unknown status";
}

static bool is_fin(double v) { return isfinite(v) != 0; }

tdi_status tdi_check_config(const tdi_config* c, const tdi_orbit* o) {
  if (!c || !o) return TDI_EINVAL;
  if (c->tdi_gen != 15 && c->tdi_gen != 20) return TDI_EUNSUPPORTED;
  if (c->mode < TDI_MODE_FULL || c->mode > TDI_MODE_HYBRID) return TDI_EUNSUPPORTED;
  if (c->precision != TDI_FP64 && c->precision != TDI_FP32_BULK) return TDI_EUNSUPPORTED;
  if (o->kind != TDI_ORBIT_FROZEN && o->kind != TDI_ORBIT_ANALYTIC1 && o->kind != TDI_ORBIT_TABLE)
    return TDI_EUNSUPPORTED;
  if (o->reserved != 0) return TDI_EINVAL;
  const int N = c->interp_taps;
  if (N != 4 && N != 8 && N != 16 && N != 32) return TDI_ERANGE;
  if (c->stencil_order != 2 && c->stencil_order != 4) return TDI_ERANGE;
  if (c->lfa_equal_arms != 0 && c->lfa_equal_arms != 1) return TDI_ERANGE;
  if (c->autotune != 0 && c->autotune != 1) return TDI_ERANGE;
  if (c->use_graph != 0 && c->use_graph != 1) return TDI_ERANGE;
  if (c->channels != TDI_CHANNELS_XYZ && c->channels != TDI_CHANNELS_AET) return TDI_EUNSUPPORTED;
  if (c->lfa_terms < 0 || c->lfa_terms > 2) return TDI_ERANGE;
  if (c->nested_delays != 0 && c->nested_delays != 1) return TDI_ERANGE;
  if (c->fast_tile_chunks != 0 && c->fast_tile_chunks != 1 && c->fast_tile_chunks != 2 &&
      c->fast_tile_chunks != 4)
    return TDI_ERANGE;
  if (c->lfa_x20_from_x15 != 0 && c->lfa_x20_from_x15 != 1) return TDI_ERANGE;
  if (c->lfa_x20_from_x15 && c->tdi_gen != 20) return TDI_ERANGE;
  if (c->lfa_x20_from_x15 && c->lfa_terms == 2) return TDI_EUNSUPPORTED;
  if (!(c->hyb_T_samples > 0.0) || !is_fin(c->hyb_T_samples)) return TDI_ERANGE;
  if (!(c->hyb_sigma_samples > 0.0) || !is_fin(c->hyb_sigma_samples)) return TDI_ERANGE;
  if (!(o->L_m > 0.0) || !is_fin(o->L_m)) return TDI_ERANGE;
  if (o->kind == TDI_ORBIT_TABLE) {
    if (!o->table) return TDI_EINVAL;
    if (o->n_table < 8) return TDI_ERANGE;
    if (!(o->table_dt > 0.0) || !is_fin(o->table_dt) || !is_fin(o->table_t0)) return TDI_ERANGE;
    for (int64_t i = 0; i < 9 * o->n_table; ++i)
      if (!is_fin(o->table[i])) return TDI_ERANGE;
    return TDI_OK;
  }
  if (!(o->R_m > o->L_m) || !is_fin(o->R_m)) return TDI_ERANGE;
  if (!(o->omega >= 0.0) || !is_fin(o->omega)) return TDI_ERANGE;
  if (!is_fin(o->kappa0) || !is_fin(o->lambda0) || !is_fin(o->t_freeze)) return TDI_ERANGE;
  // the constellation must move slowly compared with light (window bounds)
  if (o->R_m * o->omega / kC > 1e-2) return TDI_ERANGE;
  return TDI_OK;
}

tdi_status tdi_check_batch(const tdi_config* c, int64_t n_sources, const tdi_source* src,
                           const int64_t* offsets) {
  if (!c) return TDI_EINVAL;
  if (n_sources < 0) return TDI_EINVAL;
  if (!offsets) return TDI_EINVAL;
  if (n_sources > 0 && !src) return TDI_EINVAL;
  if (offsets[0] != 0) return TDI_EINVAL;
  for (int64_t i = 0; i < n_sources; ++i) {
    if (offsets[i + 1] < offsets[i]) return TDI_EINVAL;
    const tdi_source& s = src[i];
    if (!is_fin(s.beta) || fabs(s.beta) > 1.5707963267948966 + 1e-12) return TDI_ERANGE;
    if (!is_fin(s.lambda) || !is_fin(s.psi) || !is_fin(s.t0)) return TDI_ERANGE;
    if (!(s.dt > 0.0) || !is_fin(s.dt)) return TDI_ERANGE;
    if (isnan(s.t_hyb)) return TDI_ERANGE;
  }
  return TDI_OK;
}

}  // extern "C"

namespace {

// Bounds of an orbit used to size windows: rate = bound of |V| / c (delay
// drift per unit time), light times within [tmin, tmax], |R_i| <= rmax.
OrbitBounds orbit_bounds(const tdi_orbit& o) {
  OrbitBounds b;
  if (o.kind != TDI_ORBIT_TABLE) {
    const double e = o.L_m / (2.0 * sqrt(3.0) * o.R_m);
    b.rate = o.R_m * o.omega * (1.0 + 2.0 * e) / kC + 1e-12;
    b.tmax = o.L_m / kC * (1.0 + 4.0 * b.rate) + 1e-9;
    b.tmin = o.L_m / kC * (1.0 - 4.0 * b.rate) - 1e-9;
    b.rmax = o.R_m + 2.0 * o.L_m;
    return b;
  }
  // sampled orbit: speeds from successive samples (10 % allowance for the
  // curvature between them), arm lengths and distances from the samples
  double vmax = 0.0, dmax = 0.0, dmin = 1e300, rmax = 0.0;
  const double* T = o.table;
  for (int64_t j = 0; j < o.n_table; ++j) {
    for (int i = 0; i < 3; ++i) {
      const double* p = T + 9 * j + 3 * i;
      rmax = std::max(rmax, sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]));
      if (j + 1 < o.n_table) {
        const double* q = p + 9;
        const double d0 = q[0] - p[0], d1 = q[1] - p[1], d2 = q[2] - p[2];
        vmax = std::max(vmax, sqrt(d0 * d0 + d1 * d1 + d2 * d2) / o.table_dt);
      }
      const double* r = T + 9 * j + 3 * ((i + 1) % 3);
      const double e0 = r[0] - p[0], e1 = r[1] - p[1], e2 = r[2] - p[2];
      const double d = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
      dmax = std::max(dmax, d);
      dmin = std::min(dmin, d);
    }
  }
  b.rate = 1.1 * vmax / kC + 1e-12;
  b.tmax = dmax / kC * (1.0 + 4.0 * b.rate) + 1e-9;
  b.tmin = dmin / kC * (1.0 - 4.0 * b.rate) - 1e-9;
  b.rmax = rmax;
  return b;
}

double stage2_bound(const tdi_config& c, const OrbitBounds& b) {
  return (c.tdi_gen == 20 ? 7.0 : 3.0) * b.tmax;
}

// TDI 2.0 LFA from the TDI 1.5 LFA series (lfa_x20_from_x15).
bool x20_shortcut(const tdi_config& c) { return c.lfa_x20_from_x15 == 1 && c.mode != TDI_MODE_FULL; }

// The FP32 bulk LFA kernel applies to steps up to kFastDtMax and to orbits whose
// delays drift by at most kFastRateMax per unit time.
bool fast_lfa(const tdi_config& c, const OrbitBounds& b, double dt_max) {
  return c.precision == TDI_FP32_BULK && c.mode != TDI_MODE_FULL && c.lfa_terms != 2 &&
         !x20_shortcut(c) && dt_max <= tdi::kFastDtMax && b.rate <= tdi::kFastRateMax;
}

// Worst-case staged window lengths (samples) at sampling step dt; the kernels
// recompute the actual windows per tile and check them against these.
Caps window_caps(const tdi_config& c, const OrbitBounds& ob, double dt, bool fast) {
  Caps k;
  k.fast = fast ? 1 : 0;
  k.fit_cu = fast ? tdi::occupancy_lfa_fit(c.interp_taps) : 0;
  k.nx = c.lfa_terms == 2 && c.mode != TDI_MODE_FULL ? 1 : 0;
  k.tile_lfa = fast ? tdi::kTileLfaFast : tdi::kTileLfa;
  const int lfa_span = fast ? tdi::kFastChunk : tdi::kTileLfa;   // outputs sharing one window
  const int N = c.interp_taps;
  const double rate = ob.rate;
  const double Tmax = ob.tmax;
  const double Tmin = ob.tmin;
  const double Lc = Tmax;
  // stencil half width (the next term's stencil, of derivative order m + 2, is wider)
  const int hw = k.nx ? ((c.tdi_gen == 20) ? (c.stencil_order == 4 ? 4 : 3) : (c.stencil_order == 4 ? 3 : 2))
                      : ((c.tdi_gen == 20) ? (c.stencil_order == 4 ? 3 : 2) : (c.stencil_order == 4 ? 2 : 1));
  auto margin = [](double cnt) { return 2 + (int)ceil(4e-4 * cnt); };
  // LFA: the six delays D_c + mu_l spread over half an arm plus arm differences
  const double mult = c.tdi_gen == 20 ? 2.0 : 1.0;
  const double spread_l = 0.5 * Lc * 1.02 + 2.0 * mult * (Tmax - Tmin) + 2.0 * rate * lfa_span * dt;
  k.g = lfa_span + (int)ceil(spread_l / dt) + N + 2 * margin(lfa_span) + 4;
  k.hl = k.g + 2 * hw;
  // full: stage-2 delays reach back (7 or 3) light times
  k.y = tdi::kTileFull + (int)ceil(stage2_bound(c, ob) / dt) + N + 2 * margin(tdi::kTileFull) + 4;
  // stage-1 delays: light time plus spacecraft separations along k, plus drift
  const double spread_f = Tmax + Lc * 1.02 + 2.0 * rate * k.y * dt;
  k.hf = k.y + (int)ceil(spread_f / dt) + N + 2 * margin(k.y) + 4;
  const int fp32 = c.precision == TDI_FP32_BULK;
  k.lds_lfa = tdi::lfa_lds_bytes(N, k.g, k.hl, fp32, k.fast, k.nx, &k.goff);
  if (x20_shortcut(c)) {
    // the shortcut's window: the tile, the spread of T2 + T3 (delays at most two
    // light times), the taps and the first-derivative stencil
    k.g = tdi::kTileLfa + (int)ceil(2.04 * Tmax / dt) + N + 2 * margin(tdi::kTileLfa) + 4 + 2 * 2;
    k.hl = k.g;
    k.goff = 0;
    k.lds_lfa = tdi::x20_lds_bytes(k.g);
  }
  k.hyb = c.mode == TDI_MODE_HYBRID ? 1 : 0;
  k.lds_full = tdi::full_lds_bytes(k.hf, k.y, fp32, k.hyb);
  return k;
}

// A sampled orbit must cover every time the kernels evaluate the geometry at:
// each source's span, the stage-2 and light-time reach before it and the
// tap and tile margins, with the 8-point interpolation stencil inside the table.
bool table_covers(const tdi_plan* p, int64_t n_sources, const tdi_source* src, const int64_t* offsets) {
  if (p->orb.kind != TDI_ORBIT_TABLE) return true;
  const double lo = p->orb.table_t0 + 3.0 * p->orb.table_dt;
  const double hi = p->orb.table_t0 + (double)(p->orb.n_table - 5) * p->orb.table_dt;
  const double pad = p->cfg.interp_taps / 2 + 32;
  for (int64_t i = 0; i < n_sources; ++i) {
    const int64_t n = offsets[i + 1] - offsets[i];
    if (n == 0) continue;
    const double a = src[i].t0 - stage2_bound(p->cfg, p->ob) - 2.0 * p->ob.tmax - pad * src[i].dt;
    const double b = src[i].t0 + (double)(n - 1) * src[i].dt + pad * src[i].dt;
    if (!(a >= lo && b <= hi)) return false;
  }
  return true;
}

// Outputs per full-response tile: the hybrid's full regions are short (about a
// thousand samples per source), so small tiles spread them over more workgroups.
int full_tile(const tdi_config& c) { return c.mode == TDI_MODE_HYBRID ? tdi::kTileFullHybrid : tdi::kTileFull; }

// Full-response tile for a batch: the FULL mode's kTileFull, or kTileFullHybrid
// when kTileFull would not give every compute unit a tile; in the hybrid, whose
// full regions are short, kTileFullHybrid, or kTileFullSmall when the batch's
// full samples would not give every compute unit a tile (one source: the
// region's latency then sets the run time, and small tiles spread it).
int full_tile_for(const tdi_config& c, int64_t full_samples, int n_cu) {
  if (c.mode != TDI_MODE_HYBRID) {
    const int64_t tiles = (full_samples + tdi::kTileFull - 1) / tdi::kTileFull;
    return tiles < n_cu ? tdi::kTileFullHybrid : tdi::kTileFull;
  }
  const int64_t tiles = (full_samples + tdi::kTileFullHybrid - 1) / tdi::kTileFullHybrid;
  return tiles < n_cu ? tdi::kTileFullSmall : tdi::kTileFullHybrid;
}

// Outputs per LFA tile: the fast path takes the launch's chunk count.
int lfa_tile(const Caps& caps, const Launch& ln) {
  return caps.fast ? std::min(std::max(ln.chunks, 1), 4) * tdi::kFastChunk : caps.tile_lfa;
}

// Wait until staging image `slot` may be rewritten and make it current.
bool acquire_stage(tdi_plan* p, int slot) {
  if (p->stage_pending[slot]) {
    if (hipEventSynchronize(p->stage_ev[slot]) != hipSuccess) return false;
    p->stage_pending[slot] = false;
  }
  p->h_block = p->h_blk[slot];
  p->h_params = p->h_par[slot];
  return true;
}

// Mark image `slot` as read by the work enqueued so far on `st` and move on.
bool release_stage(tdi_plan* p, int slot, hipStream_t st) {
  if (hipEventRecord(p->stage_ev[slot], st) != hipSuccess) return false;
  p->stage_pending[slot] = true;
  p->stage_slot = p->double_buffer ? slot ^ 1 : slot;
  return true;
}

// Constant part of the parameter block: orbit, TDI generation, mode, stencil,
// hybrid window (dtab: device copy of a TABLE orbit's samples, else null).
void fill_constants(tdi::KParams& kp, const tdi_config& c, const tdi_orbit& o, const OrbitBounds& ob,
                    const double* dtab) {
  tdi::OrbitDev& od = kp.orb;
  od.kind = o.kind;
  od.L = o.L_m;
  od.R = o.R_m;
  od.omega = o.omega;
  od.kappa0 = o.kappa0;
  od.t_freeze = o.t_freeze;
  od.e = o.L_m / (2.0 * sqrt(3.0) * o.R_m);
  for (int i = 0; i < 3; ++i) {
    const double b = 2.0 * M_PI * (double)i / 3.0 + o.lambda0;
    od.cb[i] = cos(b);
    od.sb[i] = sin(b);
  }
  od.L_over_c = o.L_m / kC;
  if (o.kind == TDI_ORBIT_TABLE) {
    od.tab = dtab;
    od.ntab = o.n_table;
    od.tab_t0 = o.table_t0;
    od.tab_idt = 1.0 / o.table_dt;
    od.R = ob.rmax;
    od.e = 0.0;
  }
  kp.gen = c.tdi_gen;
  kp.mode = c.mode;
  kp.aet = c.channels == TDI_CHANNELS_AET ? 1 : 0;
  kp.lfa_terms = c.lfa_terms == 2 ? 2 : 1;
  kp.nested = c.nested_delays;
  kp.equal_arms = c.lfa_equal_arms;
  kp.stencil_m = c.tdi_gen == 20 ? 3 : 2;
  kp.stencil_p = c.stencil_order;
  kp.T_s = c.hyb_T_samples;
  kp.sigma_s = c.hyb_sigma_samples;
  kp.D2_bound = stage2_bound(c, ob);
}

// Sample ranges of the two kernels for one source ([lb, le) LFA, [fb, fe)
// full); the kernels apply the exact window predicates per sample, these
// ranges only need to contain them.
void kernel_ranges(const tdi_config& c, const tdi_source& s, int64_t n, int64_t& lb, int64_t& le, int64_t& fb,
                   int64_t& fe) {
  lb = le = fb = fe = 0;
  if (c.mode == TDI_MODE_FULL) {
    fe = n;
  } else if (c.mode == TDI_MODE_LFA) {
    le = n;
  } else {
    const double kH = (s.t_hyb - s.t0) / s.dt;
    const double lhi = kH + 0.5 * c.hyb_T_samples;     // LFA where k - kH <= T/2
    const double flo = kH - 0.5 * c.hyb_T_samples;     // full where k - kH >= -T/2
    le = !(lhi < (double)n) ? n : (lhi < 0.0 ? 0 : std::min<int64_t>(n, (int64_t)floor(lhi) + 2));
    fb = !(flo > 0.0) ? 0 : (flo >= (double)n ? n : std::max<int64_t>(0, (int64_t)ceil(flo) - 2));
    fe = n;
  }
}

// Fill the pinned parameter image for one batch (work lists of both kernels).
void stage_batch(const tdi_config& c, tdi::KParams* kp, int64_t n_sources, const tdi_source* src,
                 const int64_t* offsets, const double* hp, const double* hc, void* X, void* Y, void* Z,
                 const Caps& caps, const Launch& ln, int n_cu) {
  tdi::SrcDev* sd = reinterpret_cast<tdi::SrcDev*>(kp + 1);
  const int tile_lfa = lfa_tile(caps, ln);
  int64_t full_samples = 0;
  for (int64_t i = 0; i < n_sources; ++i) {
    int64_t lb, le, fb, fe;
    kernel_ranges(c, src[i], offsets[i + 1] - offsets[i], lb, le, fb, fe);
    full_samples += fe - fb;
  }
  const int tile_full = full_tile_for(c, full_samples, n_cu);
  int64_t tl = 0, tf = 0;
  for (int64_t i = 0; i < n_sources; ++i) {
    const tdi_source& s = src[i];
    tdi::SrcDev& d = sd[i];
    d.beta = s.beta; d.lam = s.lambda; d.psi = s.psi; d.t0 = s.t0; d.dt = s.dt; d.t_hyb = s.t_hyb;
    d.c2psi = cos(2.0 * s.psi);
    d.s2psi = sin(2.0 * s.psi);
    d.off = offsets[i];
    d.n = offsets[i + 1] - offsets[i];
    int64_t lb, le, fb, fe;
    kernel_ranges(c, s, d.n, lb, le, fb, fe);
    d.lfa_kb = lb; d.lfa_ke = le; d.lfa_t0 = tl;
    d.full_kb = fb; d.full_ke = fe; d.full_t0 = tf;
    if (le > lb) tl += (le - lb + tile_lfa - 1) / tile_lfa;
    if (fe > fb) tf += (fe - fb + tile_full - 1) / tile_full;
  }
  kp->n_src = n_sources;
  kp->tile_fast = caps.fast ? tile_lfa : 0;
  kp->tile_full = tile_full;
  // pre-pass: the fewest tiles per workgroup pass that cover the batch in one
  // pass of the resident workgroups (a short batch gets short passes), at most
  // kPrepTiles with several passes beyond that
  {
    const int64_t resident = std::max<int64_t>(1, (int64_t)std::max(caps.fit_cu, 1) * n_cu);
    kp->prep_tiles = (int32_t)std::min<int64_t>(tdi::kPrepTiles, std::max<int64_t>(1, (tl + resident - 1) / resident));
  }
  kp->n_tiles_lfa = tl;
  kp->n_tiles_full = tf;
  kp->hp = hp; kp->hc = hc; kp->X = X; kp->Y = Y; kp->Z = Z;
  kp->cap_g = caps.g; kp->cap_hl = caps.hl; kp->cap_hf = caps.hf; kp->cap_y = caps.y;
  kp->lfa_goff = caps.goff;
  kp->persistent = (ln.grid_lfa > 0 ? 1 : 0) | (ln.grid_full > 0 ? 2 : 0);
}

// Upload (counters and parameter block), the fit pre-pass (fast LFA path) and
// both kernels; evs (optional, kEvPerRun) are recorded between the steps.
hipError_t enqueue(tdi_plan* p, hipStream_t st, size_t copy_bytes, const Caps& caps, const Launch& ln,
                   int64_t tiles_lfa, int64_t tiles_full, const hipEvent_t* evs) {
  // counters (zero) and parameter block in one copy
  hipError_t e = hipMemcpyAsync(p->d_block, p->h_block, kCtrBytes + copy_bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  const int taps = p->cfg.interp_taps, fp32 = p->cfg.precision;
  if (evs && (e = hipEventRecord(evs[0], st)) != hipSuccess) return e;
  const int gl = ln.grid_lfa > 0 ? ln.grid_lfa : (int)std::max<int64_t>(0, tiles_lfa);
  if (gl > 0 && caps.fast && tdi::launch_lfa_fit(p->d_params, taps, caps.fit_cu * p->n_cu, st) != 0)
    return hipErrorLaunchFailure;
  if (evs && (e = hipEventRecord(evs[1], st)) != hipSuccess) return e;
  if (gl > 0 && tdi::launch_lfa(p->d_params, taps, fp32, caps.fast, caps.nx, gl, caps.lds_lfa, st) != 0)
    return hipErrorLaunchFailure;
  if (evs && (e = hipEventRecord(evs[2], st)) != hipSuccess) return e;
  const int gf = ln.grid_full > 0 ? ln.grid_full : (int)std::max<int64_t>(0, tiles_full);
  if (gf > 0 && tdi::launch_full(p->d_params, taps, fp32, caps.hyb, gf, caps.lds_full, st) != 0)
    return hipErrorLaunchFailure;
  if (evs && (e = hipEventRecord(evs[3], st)) != hipSuccess) return e;
  return hipSuccess;
}

void destroy_graph(tdi_plan* p) {
  if (p->graph_exec) hipGraphExecDestroy(p->graph_exec);
  if (p->graph) hipGraphDestroy(p->graph);
  p->graph_exec = nullptr;
  p->graph = nullptr;
}

// The nodes of a captured single chain, from its root to its end.
bool graph_chain(hipGraph_t g, std::vector<hipGraphNode_t>& chain) {
  size_t n = 0, ne = 0;
  if (hipGraphGetNodes(g, nullptr, &n) != hipSuccess || hipGraphGetEdges(g, nullptr, nullptr, &ne) != hipSuccess)
    return false;
  if (n == 0 || ne != n - 1) return false;
  std::vector<hipGraphNode_t> nodes(n), from(ne), to(ne);
  if (hipGraphGetNodes(g, nodes.data(), &n) != hipSuccess) return false;
  if (ne > 0 && hipGraphGetEdges(g, from.data(), to.data(), &ne) != hipSuccess) return false;
  chain.clear();
  for (size_t i = 0; i < n; ++i)
    if (std::find(to.begin(), to.end(), nodes[i]) == to.end()) chain.push_back(nodes[i]);
  if (chain.size() != 1) return false;
  while (chain.size() < n) {
    const auto it = std::find(from.begin(), from.end(), chain.back());
    if (it == from.end()) return false;
    chain.push_back(to[it - from.begin()]);
  }
  return true;
}

// Event-record nodes spliced into the captured chain (stream capture does not
// record events): before the fit pre-pass, before and after the LFA kernel and
// after the full kernel.  The chain is upload -> [fit] -> LFA -> full.
bool add_graph_events(tdi_plan* p, hipGraph_t g, bool fast) {
  size_t n = 0, ne = 0;
  if (hipGraphGetNodes(g, nullptr, &n) != hipSuccess || hipGraphGetEdges(g, nullptr, nullptr, &ne) != hipSuccess)
    return false;
  const size_t want = fast ? 4 : 3;
  if (n != want || ne != want - 1) return false;
  std::vector<hipGraphNode_t> nodes(n), from(ne), to(ne);
  if (hipGraphGetNodes(g, nodes.data(), &n) != hipSuccess) return false;
  if (hipGraphGetEdges(g, from.data(), to.data(), &ne) != hipSuccess) return false;
  // order the chain from its root
  std::vector<hipGraphNode_t> chain;
  for (size_t i = 0; i < n; ++i)
    if (std::find(to.begin(), to.end(), nodes[i]) == to.end()) chain.push_back(nodes[i]);
  if (chain.size() != 1) return false;
  while (chain.size() < n) {
    const auto it = std::find(from.begin(), from.end(), chain.back());
    if (it == from.end()) return false;
    chain.push_back(to[it - from.begin()]);
  }
  // the event before step `at` of the chain (at == n: after the last node)
  auto splice = [&](size_t at, hipEvent_t ev, hipGraphNode_t* out) -> bool {
    hipGraphNode_t a = chain[at - 1];
    if (at < chain.size()) {
      hipGraphNode_t b = chain[at];
      if (hipGraphRemoveDependencies(g, &a, &b, 1) != hipSuccess) return false;
      if (hipGraphAddEventRecordNode(out, g, &a, 1, ev) != hipSuccess) return false;
      if (hipGraphAddDependencies(g, out, &b, 1) != hipSuccess) return false;
    } else if (hipGraphAddEventRecordNode(out, g, &a, 1, ev) != hipSuccess) {
      return false;
    }
    chain.insert(chain.begin() + at, *out);
    return true;
  };
  // chain indices: 0 upload, then [fit], LFA, full
  size_t at = 1;
  if (!splice(at, p->ev[0][0], &p->graph_ev_node[0])) return false;
  at += 1 + (fast ? 1 : 0);
  if (!splice(at, p->ev[0][1], &p->graph_ev_node[1])) return false;
  at += 2;
  if (!splice(at, p->ev[0][2], &p->graph_ev_node[2])) return false;
  at += 2;
  return splice(at, p->ev[0][3], &p->graph_ev_node[3]);
}

// Capture (upload of the counters and the whole parameter block, the fit
// pre-pass and both persistent kernels) once; replays pick up new batches from
// the block.  With timed = true, event-record nodes are added around the
// kernels (using the events of ring slot 0 as placeholders) so that each
// replay can point them at its own ring slot.
bool capture_graph_once(tdi_plan* p, const Caps& caps, const Launch& ln, bool timed) {
  destroy_graph(p);
  p->graph_timed = false;
  if (hipStreamBeginCapture(p->graph_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  hipError_t e = enqueue(p, p->graph_stream, p->params_bytes, caps, ln, 0, 0, nullptr);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(p->graph_stream, &g);
  if (e != hipSuccess || e2 != hipSuccess || !g) {
    if (g) hipGraphDestroy(g);
    (void)hipGetLastError();
    return false;
  }
  p->graph = g;
  // the kernel nodes in chain order: [fit pre-pass], LFA, full
  {
    for (int j = 0; j < 3; ++j) p->graph_knode[j] = nullptr;
    p->graph_mnode = nullptr;
    std::vector<hipGraphNode_t> chain, kn;
    if (!graph_chain(g, chain)) chain.clear();
    if (!chain.empty()) {
      hipGraphNodeType t;
      if (hipGraphNodeGetType(chain[0], &t) == hipSuccess && t == hipGraphNodeTypeMemcpy) p->graph_mnode = chain[0];
    }
    for (hipGraphNode_t nd : chain) {
      hipGraphNodeType t;
      if (hipGraphNodeGetType(nd, &t) == hipSuccess && t == hipGraphNodeTypeKernel) kn.push_back(nd);
    }
    const size_t want = caps.fast ? 3 : 2;
    if (kn.size() == want) {
      for (size_t j = 0; j < kn.size(); ++j) {
        const int slot = caps.fast ? (int)j : (int)j + 1;   // 0 fit, 1 LFA, 2 full
        if (hipGraphKernelNodeGetParams(kn[j], &p->graph_kparams[slot]) == hipSuccess) {
          p->graph_knode[slot] = kn[j];
          p->graph_kgrid[slot] = p->graph_kparams[slot].gridDim.x;
        }
      }
    }
    (void)hipGetLastError();
  }
  if (timed) {
    const bool added = add_graph_events(p, g, caps.fast != 0);
    (void)hipGetLastError();
    if (getenv("TDI_DEBUG")) fprintf(stderr, "tdi: graph event nodes %s\n", added ? "added" : "not added");
    if (!added) {
      destroy_graph(p);
      return false;
    }
  }
  if (hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
    destroy_graph(p);
    (void)hipGetLastError();
    return false;
  }
  p->graph_timed = timed;
  p->graph_launch = ln;
  p->graph_lds_lfa = caps.lds_lfa;
  p->graph_lds_full = caps.lds_full;
  p->graph_fast = caps.fast;
  return true;
}

bool capture_graph(tdi_plan* p, const Caps& caps, const Launch& ln) {
  return capture_graph_once(p, caps, ln, true) || capture_graph_once(p, caps, ln, false);
}

void advance_ring(tdi_plan* p) {
  p->ev_head = (p->ev_head + 1) % kEventRing;
  if (p->ev_count < kEventRing) p->ev_count++;
}

// Window capacities for a batch (smallest step) and the LFA kernel choice
// (largest step); false for a batch without samples.
bool batch_caps(const tdi_config& cfg, const OrbitBounds& ob, int64_t n_sources, const tdi_source* src,
                const int64_t* offsets, Caps* caps) {
  double dt_min = INFINITY, dt_max = 0.0;
  for (int64_t i = 0; i < n_sources; ++i)
    if (offsets[i + 1] > offsets[i]) {
      dt_min = std::min(dt_min, src[i].dt);
      dt_max = std::max(dt_max, src[i].dt);
    }
  if (!isfinite(dt_min)) return false;
  *caps = window_caps(cfg, ob, dt_min, fast_lfa(cfg, ob, dt_max));
  return true;
}

// TDI 2.0 LFA from TDI 1.5: pass 1 runs the FP64 TDI 1.5 LFA over every sample
// of each source into d_x15 (its own parameter block and counters), pass 2
// (k_x20) forms the TDI 2.0 LFA part from it, then the full-response kernel
// adds the hybrid's full part.  Plain stream launches, persistent grids.
tdi_status run_x20(tdi_plan* p, int64_t n_sources, const tdi_source* src, const int64_t* offsets,
                   const double* hp, const double* hc, void* X, void* Y, void* Z, bool record) {
  Caps caps, caps15;
  if (!batch_caps(p->cfg, p->ob, n_sources, src, offsets, &caps)) return TDI_OK;
  if (!batch_caps(p->cfg15, p->ob, n_sources, src, offsets, &caps15)) return TDI_OK;
  if (caps.lds_lfa > p->max_lds || caps.lds_full > p->max_lds || caps15.lds_lfa > p->max_lds) return TDI_ERANGE;
  const int taps = p->cfg.interp_taps, fp32 = p->cfg.precision;
  const int64_t total = offsets[n_sources];
  Launch ln15 = {tdi::occupancy_lfa(taps, 0, 0, 0, caps15.lds_lfa) * p->n_cu, 0, 4};
  Launch ln = {tdi::occupancy_x20(taps, fp32, caps.lds_lfa) * p->n_cu,
               tdi::occupancy_full(taps, fp32, caps.hyb, caps.lds_full) * p->n_cu, 4};
  p->last_fast = 0;
  p->last_tile_lfa = tdi::kTileLfa;
  if (p->staged_pending) {
    if (hipEventSynchronize(p->staged_free) != hipSuccess) return TDI_EDEVICE;
    p->staged_pending = false;
  }
  const int slot = p->stage_slot;
  if (!acquire_stage(p, slot)) return TDI_EDEVICE;
  stage_batch(p->cfg15, p->h_params15, n_sources, src, offsets, hp, hc, p->d_x15, p->d_x15 + total,
              p->d_x15 + 2 * total, caps15, ln15, p->n_cu);
  stage_batch(p->cfg, p->h_params, n_sources, src, offsets, hp, hc, X, Y, Z, caps, ln, p->n_cu);
  p->h_params->x15 = p->d_x15;
  p->h_params->x15_stride = total;
  const size_t copy_bytes = sizeof(tdi::KParams) + sizeof(tdi::SrcDev) * (size_t)n_sources;
  hipStream_t st = p->user_stream;
  const hipEvent_t* evs = record ? p->ev[p->ev_head] : nullptr;
  if (hipMemcpyAsync(p->d_block15, p->h_block15, kCtrBytes + copy_bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(p->d_block, p->h_block, kCtrBytes + copy_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
    return TDI_EDEVICE;
  if (evs && hipEventRecord(evs[0], st) != hipSuccess) return TDI_EDEVICE;
  if (p->h_params15->n_tiles_lfa > 0 &&
      tdi::launch_lfa(p->d_params15, taps, 0, 0, 0, ln15.grid_lfa, caps15.lds_lfa, st) != 0)
    return TDI_EDEVICE;
  if (evs && hipEventRecord(evs[1], st) != hipSuccess) return TDI_EDEVICE;
  if (p->h_params->n_tiles_lfa > 0 && tdi::launch_x20(p->d_params, taps, fp32, ln.grid_lfa, caps.lds_lfa, st) != 0)
    return TDI_EDEVICE;
  if (evs && hipEventRecord(evs[2], st) != hipSuccess) return TDI_EDEVICE;
  if (p->h_params->n_tiles_full > 0 &&
      tdi::launch_full(p->d_params, taps, fp32, caps.hyb, ln.grid_full, caps.lds_full, st) != 0)
    return TDI_EDEVICE;
  if (evs && hipEventRecord(evs[3], st) != hipSuccess) return TDI_EDEVICE;
  hipEventRecord(p->staged_free, st);
  p->staged_pending = true;
  if (!release_stage(p, slot, st)) return TDI_EDEVICE;
  if (record) advance_ring(p);
  return TDI_OK;
}

tdi_status run_with(tdi_plan* p, const Launch& ln, int64_t n_sources, const tdi_source* src,
                    const int64_t* offsets, const double* hp, const double* hc, void* X, void* Y,
                    void* Z, bool record, bool allow_graph) {
  if (x20_shortcut(p->cfg)) return run_x20(p, n_sources, src, offsets, hp, hc, X, Y, Z, record);
  Caps caps;
  if (!batch_caps(p->cfg, p->ob, n_sources, src, offsets, &caps)) return TDI_OK;
  if (caps.lds_lfa > p->max_lds || caps.lds_full > p->max_lds) return TDI_ERANGE;
  p->last_fast = caps.fast;
  p->last_tile_lfa = lfa_tile(caps, ln);

  // the image of this staging slot must have been uploaded by its earlier run
  const int sslot = p->stage_slot;
  if (!acquire_stage(p, sslot)) return TDI_EDEVICE;
  stage_batch(p->cfg, p->h_params, n_sources, src, offsets, hp, hc, X, Y, Z, caps, ln, p->n_cu);
  p->last_tile_full = p->h_params->tile_full;
  const int64_t tl = p->h_params->n_tiles_lfa, tf = p->h_params->n_tiles_full;
  // per-tile records of the fast path: tiles hold at least kFastChunk outputs,
  // so a batch within the plan's maxima always fits; checked all the same
  if (caps.fast && tl > p->fit_tiles) return TDI_ESTATE;
  const size_t copy_bytes = sizeof(tdi::KParams) + sizeof(tdi::SrcDev) * (size_t)n_sources;
  const int slot = p->ev_head;

  const bool graph = allow_graph && p->cfg.use_graph && ln.grid_lfa > 0 && ln.grid_full > 0;
  if (graph) {
    if (!p->graph_exec || p->graph_launch.grid_lfa != ln.grid_lfa ||
        p->graph_launch.grid_full != ln.grid_full || p->graph_lds_lfa != caps.lds_lfa ||
        p->graph_lds_full != caps.lds_full || p->graph_fast != caps.fast) {
      if (!capture_graph(p, caps, ln)) return TDI_EDEVICE;
    }
    // replay on the private stream, ordered after the caller's stream and back
    if (hipEventRecord(p->handoff, p->user_stream) != hipSuccess) return TDI_EDEVICE;
    if (hipStreamWaitEvent(p->graph_stream, p->handoff, 0) != hipSuccess) return TDI_EDEVICE;
    // per-kernel times from the captured event nodes, else the whole replay
    bool inner = false;
    if (p->graph_timed) {
      inner = true;
      for (int j = 0; j < kEvPerRun && inner; ++j) {
        const hipError_t es = hipGraphExecEventRecordNodeSetEvent(p->graph_exec, p->graph_ev_node[j],
                                                                  p->ev[record ? slot : 0][j]);
        inner = es == hipSuccess;
        if (!inner && getenv("TDI_DEBUG"))
          fprintf(stderr, "tdi: retargeting graph event node %d failed: %d\n", j, (int)es);
      }
      if (!inner) {
        (void)hipGetLastError();
        p->graph_timed = false;
      }
    }
    // without inner events the whole replay is reported as the LFA time
    if (record && !inner) {
      hipEventRecord(p->ev[slot][0], p->graph_stream);
      hipEventRecord(p->ev[slot][1], p->graph_stream);
    }
    // persistent grids no larger than the batch's tiles (a short batch is not
    // charged for launching and retiring a full chip's worth of idle workgroups)
    {
      const int64_t ptl = p->h_params->prep_tiles;
      const int64_t tiles[3] = {(tl + ptl - 1) / ptl, tl, tf};   // pre-pass: workgroup passes
      for (int j = 0; j < 3; ++j) {
        if (!p->graph_knode[j]) continue;
        const unsigned full_grid = j == 0 ? (unsigned)(caps.fit_cu * p->n_cu)
                                          : (unsigned)(j == 1 ? ln.grid_lfa : ln.grid_full);
        const unsigned want = (unsigned)std::max<int64_t>(1, std::min<int64_t>(full_grid, tiles[j]));
        if (want == p->graph_kgrid[j]) continue;
        hipKernelNodeParams kp = p->graph_kparams[j];
        kp.gridDim.x = want;
        if (hipGraphExecKernelNodeSetParams(p->graph_exec, p->graph_knode[j], &kp) == hipSuccess) {
          p->graph_kgrid[j] = want;
        } else {
          (void)hipGetLastError();
          p->graph_knode[j] = nullptr;      // keep the captured grid from now on
        }
      }
    }
    // the upload node reads this run's image
    if (p->double_buffer &&
        (!p->graph_mnode ||
         hipGraphExecMemcpyNodeSetParams1D(p->graph_exec, p->graph_mnode, p->d_block, p->h_block,
                                           kCtrBytes + p->params_bytes, hipMemcpyHostToDevice) != hipSuccess)) {
      (void)hipGetLastError();
      // the upload cannot be retargeted: capture again from this image and keep
      // to it from now on (one image, each run waiting for the previous one)
      p->double_buffer = false;
      if (!capture_graph(p, caps, ln)) return TDI_EDEVICE;
    }
    if (hipGraphLaunch(p->graph_exec, p->graph_stream) != hipSuccess) return TDI_EDEVICE;
    if (record) {
      if (!inner) {
        hipEventRecord(p->ev[slot][2], p->graph_stream);
        hipEventRecord(p->ev[slot][3], p->graph_stream);
      }
      advance_ring(p);
    }
    hipEventRecord(p->staged_free, p->graph_stream);
    if (!release_stage(p, sslot, p->graph_stream)) return TDI_EDEVICE;
    if (hipStreamWaitEvent(p->user_stream, p->staged_free, 0) != hipSuccess) return TDI_EDEVICE;
    return TDI_OK;
  }
  hipError_t e = enqueue(p, p->user_stream, copy_bytes, caps, ln, tl, tf, record ? p->ev[slot] : nullptr);
  if (e != hipSuccess) return TDI_EDEVICE;
  if (!release_stage(p, sslot, p->user_stream)) return TDI_EDEVICE;
  if (record) advance_ring(p);
  return TDI_OK;
}

// Diagnostics on stderr, by the TDI_LOG environment variable: 1 reports each
// autotune decision, 2 also every candidate's time.
int log_level() {
  const char* s = getenv("TDI_LOG");
  return s ? atoi(s) : 0;
}

// Autotune cache.  With TDI_AUTOTUNE_CACHE naming a file, each decision of the
// autotuner is appended to it as one JSON object per line, and a later plan
// whose key matches takes the stored launch without timing.  The key holds the
// device architecture and compute-unit count, every option that changes the
// kernels or their windows (including the LDS sizes the batch needs), and the
// batch shape as powers of two of the source and sample counts.  Lines that do
// not parse are skipped; the last matching line wins.
void tune_key(const tdi_plan* p, const Caps& caps, int64_t n_sources, int64_t total, char* key, size_t n) {
  auto lg2 = [](int64_t v) {
    int b = 0;
    while (b < 62 && ((int64_t)1 << b) < v) ++b;
    return b;
  };
  const tdi_config& c = p->cfg;
  snprintf(key, n,
           "%s,cu=%d,gen=%d,mode=%d,prec=%d,taps=%d,p=%d,equal=%d,terms=%d,x20_from_x15=%d,channels=%d,"
           "nested=%d,chunks=%d,graph=%d,orbit=%d,lds=%zu+%zu,sources=2^%d,samples=2^%d",
           p->arch, p->n_cu, c.tdi_gen, c.mode, c.precision, c.interp_taps, c.stencil_order, c.lfa_equal_arms,
           c.lfa_terms, c.lfa_x20_from_x15, c.channels, c.nested_delays, c.fast_tile_chunks, c.use_graph,
           p->orb.kind, caps.lds_lfa, caps.lds_full, lg2(n_sources), lg2(total));
}

bool tune_cache_get(const tdi_plan* p, const char* path, const char* key, Launch* ln, bool* stream) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char head[320];
  snprintf(head, sizeof(head), "{\"key\": \"%s\", ", key);
  const size_t hn = strlen(head);
  char line[512];
  bool hit = false;
  while (fgets(line, sizeof(line), f)) {
    if (strncmp(line, head, hn) != 0) continue;
    int gl = -1, gf = -1, ch = 0, sp = -1;
    if (sscanf(line + hn, "\"grid_lfa\": %d, \"grid_full\": %d, \"chunks\": %d, \"stream\": %d}", &gl, &gf,
               &ch, &sp) != 4)
      continue;
    const int gmax = 64 * p->n_cu;
    if (gl < 0 || gf < 0 || gl > gmax || gf > gmax || (ch != 1 && ch != 2 && ch != 4) || (sp != 0 && sp != 1))
      continue;
    *ln = {gl, gf, ch};
    *stream = sp == 1;
    hit = true;
  }
  fclose(f);
  return hit;
}

void tune_cache_put(const char* path, const char* key, const Launch& ln, bool stream) {
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "{\"key\": \"%s\", \"grid_lfa\": %d, \"grid_full\": %d, \"chunks\": %d, \"stream\": %d}\n", key,
          ln.grid_lfa, ln.grid_full, ln.chunks, stream ? 1 : 0);
  fclose(f);
}

void autotune(tdi_plan* p, int64_t n_sources, const tdi_source* src, const int64_t* offsets,
              const double* hp, const double* hc, void* X, void* Y, void* Z) {
  Caps caps;
  if (!batch_caps(p->cfg, p->ob, n_sources, src, offsets, &caps)) return;
  const int verbose = log_level();
  const char* cache = getenv("TDI_AUTOTUNE_CACHE");
  char key[256];
  tune_key(p, caps, n_sources, offsets[n_sources], key, sizeof(key));
  if (cache && *cache) {
    Launch ln;
    bool sp = false;
    if (tune_cache_get(p, cache, key, &ln, &sp)) {
      p->launch = ln;
      p->stream_pick = p->cfg.use_graph && sp;
      p->tuned = true;
      p->tune_cached = true;
      if (verbose >= 1)
        fprintf(stderr, "[tdi] autotune %s: from cache, grid_lfa %d grid_full %d chunks %d stream %d\n", key,
                ln.grid_lfa, ln.grid_full, ln.chunks, sp ? 1 : 0);
      return;
    }
  }
  const int ol = tdi::occupancy_lfa(p->cfg.interp_taps, p->cfg.precision, caps.fast, caps.nx, caps.lds_lfa);
  const int of = tdi::occupancy_full(p->cfg.interp_taps, p->cfg.precision, caps.hyb, caps.lds_full);
  // grid candidates (persistent at the resident count, half and twice that, or
  // one workgroup per tile), each with every tile shape of the fast LFA path:
  // small tiles give single long sources enough tiles to fill the chip, large
  // ones amortise the per-tile geometry fit over big batches
  std::vector<Launch> grids;
  grids.push_back({ol * p->n_cu, of * p->n_cu, 4});
  grids.push_back({0, 0, 4});
  if (ol > 1) grids.push_back({(ol / 2) * p->n_cu, of * p->n_cu, 4});
  grids.push_back({2 * ol * p->n_cu, 2 * of * p->n_cu, 4});
  std::vector<Launch> cands;
  for (const int ch : {4, 2, 1}) {
    // the chunk count only matters on the fast path; a forced one is kept
    const bool keep = caps.fast ? (p->cfg.fast_tile_chunks == 0 || ch == p->cfg.fast_tile_chunks) : ch == 4;
    if (!keep) continue;
    for (Launch g : grids) {
      // graph replay needs persistent launches: with graphs only those are timed
      if (p->cfg.use_graph && (g.grid_lfa == 0 || g.grid_full == 0)) continue;
      g.chunks = ch;
      cands.push_back(g);
    }
  }
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  float best = INFINITY;
  Launch best_l = cands[0];
  for (const Launch& ln : cands) {
    float ms_sum = 0.0f;
    bool ok = true;
    for (int rep = 0; rep < 3 && ok; ++rep) {
      hipEventRecord(a, p->user_stream);
      if (run_with(p, ln, n_sources, src, offsets, hp, hc, X, Y, Z, false, false) != TDI_OK) ok = false;
      hipEventRecord(b, p->user_stream);
      if (hipEventSynchronize(b) != hipSuccess) ok = false;
      float ms = 0.0f;
      hipEventElapsedTime(&ms, a, b);
      if (rep > 0) ms_sum += ms;
    }
    if (verbose >= 2)
      fprintf(stderr, "[tdi] autotune candidate grid_lfa %d grid_full %d chunks %d: %.4f ms%s\n", ln.grid_lfa,
              ln.grid_full, ln.chunks, 0.5f * ms_sum, ok ? "" : " (failed)");
    if (ok && ms_sum < best) {
      best = ms_sum;
      best_l = ln;
    }
  }
  p->launch = best_l;
  p->stream_pick = false;
  if (p->cfg.use_graph) {
    // With graphs the candidates are persistent launches, which replay.  A
    // replay saves host work per run, but on short runs it can cost the host
    // more than the stream launches it replaces: time both over back-to-back
    // runs and keep the faster.
    auto batch_ms = [&](const Launch& ln, bool graph) -> float {
      hipEventRecord(a, p->user_stream);
      for (int rep = 0; rep < 8; ++rep)
        if (run_with(p, ln, n_sources, src, offsets, hp, hc, X, Y, Z, false, graph) != TDI_OK) return INFINITY;
      hipEventRecord(b, p->user_stream);
      if (hipEventSynchronize(b) != hipSuccess) return INFINITY;
      float ms = 0.0f;
      hipEventElapsedTime(&ms, a, b);
      return ms;
    };
    (void)batch_ms(best_l, true);                        // capture and warm the graph
    const float tg = batch_ms(best_l, true);
    const float ts = batch_ms(best_l, false);
    (void)hipGetLastError();
    p->stream_pick = ts < 0.97f * tg;
    if (verbose >= 2)
      fprintf(stderr, "[tdi] autotune 8 runs: graph %.4f ms, stream %.4f ms\n", tg, ts);
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  p->tuned = true;
  if (verbose >= 1)
    fprintf(stderr, "[tdi] autotune %s: grid_lfa %d grid_full %d chunks %d stream %d\n", key, best_l.grid_lfa,
            best_l.grid_full, best_l.chunks, p->stream_pick ? 1 : 0);
  if (cache && *cache && std::isfinite(best)) tune_cache_put(cache, key, best_l, p->stream_pick);
}

}  // namespace

extern "C" {

tdi_status tdi_plan_create(tdi_plan** out, const tdi_config* cfg, const tdi_orbit* orb,
                           int64_t max_sources, int64_t max_total_samples, void* hip_stream) {
  if (!out) return TDI_EINVAL;
  *out = nullptr;
  tdi_status st = tdi_check_config(cfg, orb);
  if (st != TDI_OK) return st;
  if (max_sources < 1 || max_total_samples < 0) return TDI_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return TDI_EDEVICE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TDI_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return TDI_EDEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TDI_EDEVICE;
  if (tdi::set_constants() != 0) return TDI_EDEVICE;

  tdi_plan* p = (tdi_plan*)calloc(1, sizeof(tdi_plan));
  if (!p) return TDI_ENOMEM;
  p->cfg = *cfg;
  p->orb = *orb;
  p->orb.table = nullptr;
  p->ob = orbit_bounds(*orb);
  p->max_sources = max_sources;
  p->max_total = max_total_samples;
  p->device = dev;
  p->n_cu = prop.multiProcessorCount;
  snprintf(p->arch, sizeof(p->arch), "%s", prop.gcnArchName);
  p->max_lds = prop.sharedMemPerBlock;
  p->last_fast = 0;
  p->last_tile_lfa = tdi::kTileLfa;
  p->user_stream = (hipStream_t)hip_stream;
  p->params_bytes = sizeof(tdi::KParams) + sizeof(tdi::SrcDev) * (size_t)max_sources;
  bool ok = hipMalloc((void**)&p->d_block, kCtrBytes + p->params_bytes) == hipSuccess;
  ok = ok && hipMalloc((void**)&p->d_err, 64) == hipSuccess;
  if (ok && cfg->precision == TDI_FP32_BULK && cfg->mode != TDI_MODE_FULL) {
    // records of the fast LFA path: at most one partial tile per source beyond the full ones
    p->fit_tiles = max_total_samples / tdi::kFastChunk + max_sources + 1;
    ok = hipMalloc(&p->d_ftiles, (size_t)p->fit_tiles * tdi::fast_tile_bytes()) == hipSuccess;
  }
  for (int j = 0; j < 2 && ok; ++j) {
    ok = hipHostMalloc((void**)&p->h_blk[j], kCtrBytes + p->params_bytes, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&p->stage_ev[j], hipEventDisableTiming) == hipSuccess;
    if (ok) p->h_par[j] = reinterpret_cast<tdi::KParams*>(p->h_blk[j] + kCtrBytes);
  }
  if (ok) {
    p->d_params = reinterpret_cast<tdi::KParams*>(p->d_block + kCtrBytes);
    p->h_block = p->h_blk[0];
    p->h_params = p->h_par[0];
    p->stage_slot = 0;
    p->double_buffer = true;
  }
  if (ok && x20_shortcut(*cfg)) {
    ok = hipMalloc((void**)&p->d_x15, sizeof(double) * 3 * (size_t)std::max<int64_t>(1, max_total_samples)) ==
         hipSuccess;
    ok = ok && hipMalloc((void**)&p->d_block15, kCtrBytes + p->params_bytes) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&p->h_block15, kCtrBytes + p->params_bytes, hipHostMallocDefault) == hipSuccess;
    if (ok) {
      p->d_params15 = reinterpret_cast<tdi::KParams*>(p->d_block15 + kCtrBytes);
      p->h_params15 = reinterpret_cast<tdi::KParams*>(p->h_block15 + kCtrBytes);
    }
  }
  ok = ok && hipEventCreateWithFlags(&p->staged_free, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&p->handoff, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&p->graph_stream, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; ok && i < kEventRing; ++i)
    for (int j = 0; ok && j < kEvPerRun; ++j) ok = hipEventCreate(&p->ev[i][j]) == hipSuccess;
  if (!ok) {
    tdi_plan_destroy(p);
    return TDI_ENOMEM;
  }
  if (hipMemset(p->d_err, 0, 64) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    tdi_plan_destroy(p);
    return TDI_EDEVICE;
  }
  for (int j = 0; j < 2; ++j) memset(p->h_blk[j], 0, kCtrBytes + p->params_bytes);

  if (orb->kind == TDI_ORBIT_TABLE) {
    const size_t tb = sizeof(double) * 9 * (size_t)orb->n_table;
    if (hipMalloc((void**)&p->d_orbtab, tb) != hipSuccess) {
      tdi_plan_destroy(p);
      return TDI_ENOMEM;
    }
    if (hipMemcpy(p->d_orbtab, orb->table, tb, hipMemcpyHostToDevice) != hipSuccess) {
      tdi_plan_destroy(p);
      return TDI_EDEVICE;
    }
  }
  for (int j = 0; j < 2; ++j) {
    fill_constants(*p->h_par[j], *cfg, *orb, p->ob, p->d_orbtab);
    p->h_par[j]->err = p->d_err;
    p->h_par[j]->lfa_tiles = p->d_ftiles;
    p->h_par[j]->counters = reinterpret_cast<uint32_t*>(p->d_block);
  }
  if (x20_shortcut(*cfg)) {
    // pass 1: the same source set at TDI 1.5, LFA mode, FP64, over every sample
    p->cfg15 = *cfg;
    p->cfg15.tdi_gen = 15;
    p->cfg15.mode = TDI_MODE_LFA;
    p->cfg15.precision = TDI_FP64;
    p->cfg15.lfa_terms = 0;
    p->cfg15.lfa_x20_from_x15 = 0;
    p->cfg15.channels = TDI_CHANNELS_XYZ;
    memset(p->h_block15, 0, kCtrBytes + p->params_bytes);
    fill_constants(*p->h_params15, p->cfg15, *orb, p->ob, p->d_orbtab);
    p->h_params15->err = p->d_err;
    p->h_params15->lfa_tiles = nullptr;
    p->h_params15->counters = reinterpret_cast<uint32_t*>(p->d_block15);
  }

  p->timing = true;
  p->launch = {0, 0, cfg->fast_tile_chunks != 0 ? cfg->fast_tile_chunks : 4};
  p->tuned = cfg->autotune && !x20_shortcut(*cfg) ? false : true;
  if (!cfg->autotune && cfg->use_graph) {
    // graph replay needs persistent launches: one full occupancy of the chip
    const Caps caps = window_caps(*cfg, p->ob, 1.0, fast_lfa(*cfg, p->ob, 1.0));
    p->launch.grid_lfa = tdi::occupancy_lfa(cfg->interp_taps, cfg->precision, caps.fast, caps.nx, caps.lds_lfa) * p->n_cu;
    p->launch.grid_full = tdi::occupancy_full(cfg->interp_taps, cfg->precision, caps.hyb, caps.lds_full) * p->n_cu;
  }
  *out = p;
  return TDI_OK;
}

tdi_status tdi_plan_destroy(tdi_plan* p) {
  if (!p) return TDI_EINVAL;
  if (p->graph_stream) hipStreamSynchronize(p->graph_stream);
  hipStreamSynchronize(p->user_stream);
  destroy_graph(p);
  for (int i = 0; i < kEventRing; ++i)
    for (int j = 0; j < kEvPerRun; ++j)
      if (p->ev[i][j]) hipEventDestroy(p->ev[i][j]);
  if (p->staged_free) hipEventDestroy(p->staged_free);
  if (p->handoff) hipEventDestroy(p->handoff);
  if (p->graph_stream) hipStreamDestroy(p->graph_stream);
  if (p->d_block) hipFree(p->d_block);
  if (p->d_err) hipFree(p->d_err);
  if (p->d_ftiles) hipFree(p->d_ftiles);
  if (p->d_orbtab) hipFree(p->d_orbtab);
  if (p->d_x15) hipFree(p->d_x15);
  if (p->d_block15) hipFree(p->d_block15);
  if (p->h_block15) hipHostFree(p->h_block15);
  for (int j = 0; j < 2; ++j) {
    if (p->h_blk[j]) hipHostFree(p->h_blk[j]);
    if (p->stage_ev[j]) hipEventDestroy(p->stage_ev[j]);
  }
  free(p);
  return TDI_OK;
}

tdi_status tdi_run(tdi_plan* p, int64_t n_sources, const tdi_source* src, const int64_t* offsets,
                   const double* hp, const double* hc, void* X, void* Y, void* Z) {
  if (!p) return TDI_ESTATE;
  tdi_status st = tdi_check_batch(&p->cfg, n_sources, src, offsets);
  if (st != TDI_OK) return st;
  if (n_sources > p->max_sources || offsets[n_sources] > p->max_total) return TDI_ESTATE;
  const int64_t total = offsets[n_sources];
  if (total == 0) return TDI_OK;
  if (!hp || !hc || !X || !Y || !Z) return TDI_EINVAL;
  const uintptr_t al = p->cfg.precision == TDI_FP64 ? 8 : 4;
  if (((uintptr_t)hp | (uintptr_t)hc) & 7) return TDI_EINVAL;
  if ((((uintptr_t)X) | ((uintptr_t)Y) | ((uintptr_t)Z)) & (al - 1)) return TDI_EINVAL;
  if (!table_covers(p, n_sources, src, offsets)) return TDI_ERANGE;
  if (!p->tuned) autotune(p, n_sources, src, offsets, hp, hc, X, Y, Z);
  return run_with(p, p->launch, n_sources, src, offsets, hp, hc, X, Y, Z, p->timing, !p->stream_pick);
}

tdi_status tdi_plan_set_timing(tdi_plan* p, int32_t on) {
  if (!p) return TDI_ESTATE;
  if (on != 0 && on != 1) return TDI_EINVAL;
  p->timing = on != 0;
  return TDI_OK;
}

tdi_status tdi_run_links(tdi_plan* p, int64_t n_sources, const tdi_source* src, const int64_t* offsets,
                         const double* hp, const double* hc, void* y) {
  if (!p) return TDI_ESTATE;
  tdi_status st = tdi_check_batch(&p->cfg, n_sources, src, offsets);
  if (st != TDI_OK) return st;
  if (n_sources > p->max_sources || offsets[n_sources] > p->max_total) return TDI_ESTATE;
  const int64_t total = offsets[n_sources];
  if (total == 0) return TDI_OK;
  if (!hp || !hc || !y) return TDI_EINVAL;
  const int fp32 = p->cfg.precision == TDI_FP32_BULK ? 1 : 0;
  if (((uintptr_t)hp | (uintptr_t)hc) & 7) return TDI_EINVAL;
  if (((uintptr_t)y) & (fp32 ? 3 : 7)) return TDI_EINVAL;
  // read window of a tile: the tile, the spread of every delay the links use
  // (|k.R|/c <= (R (1 + e) + L)/c, light times <= 1.01 L/c), the taps, margins
  if (!table_covers(p, n_sources, src, offsets)) return TDI_ERANGE;
  const double spread = 2.0 * p->ob.rmax / kC + p->ob.tmax;
  const int N = p->cfg.interp_taps;
  const int margin = 2 + (int)ceil(4e-4 * (double)tdi::kTileLinks);
  int cap = 0;
  for (int64_t i = 0; i < n_sources; ++i)
    cap = std::max(cap, tdi::kTileLinks + (int)ceil(spread / src[i].dt) + N + 2 * margin + 8);
  const size_t lds = tdi::links_lds_bytes(cap, fp32, p->cfg.lfa_terms == 2 ? 3 : 2);
  if (lds > p->max_lds) return TDI_ERANGE;
  const int slot = p->stage_slot;
  if (!acquire_stage(p, slot)) return TDI_EDEVICE;
  tdi::KParams* kp = p->h_params;
  tdi::SrcDev* sd = reinterpret_cast<tdi::SrcDev*>(kp + 1);
  int64_t tiles = 0;
  for (int64_t i = 0; i < n_sources; ++i) {
    const tdi_source& s = src[i];
    tdi::SrcDev& d = sd[i];
    d.beta = s.beta; d.lam = s.lambda; d.psi = s.psi; d.t0 = s.t0; d.dt = s.dt; d.t_hyb = s.t_hyb;
    d.c2psi = cos(2.0 * s.psi);
    d.s2psi = sin(2.0 * s.psi);
    d.off = offsets[i];
    d.n = offsets[i + 1] - offsets[i];
    d.lfa_kb = 0; d.lfa_ke = d.n; d.lfa_t0 = tiles;
    d.full_kb = 0; d.full_ke = 0; d.full_t0 = 0;
    tiles += (d.n + tdi::kTileLinks - 1) / tdi::kTileLinks;
  }
  kp->n_src = n_sources;
  kp->n_tiles_lfa = tiles;
  kp->n_tiles_full = 0;
  kp->hp = hp; kp->hc = hc; kp->X = y; kp->Y = nullptr; kp->Z = nullptr;
  kp->cap_lk = cap;
  kp->link_stride = total;
  kp->persistent = 0;
  const size_t copy_bytes = sizeof(tdi::KParams) + sizeof(tdi::SrcDev) * (size_t)n_sources;
  hipStream_t s = p->user_stream;
  if (hipMemcpyAsync(p->d_block, p->h_block, kCtrBytes + copy_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
    return TDI_EDEVICE;
  if (!release_stage(p, slot, s)) return TDI_EDEVICE;
  const int arm = fp32 && p->cfg.mode != TDI_MODE_FULL && p->cfg.lfa_terms != 2 ? 1 : 0;
  if (tdi::launch_links(p->d_params, N, fp32, arm, tiles, lds, s) != 0) return TDI_EDEVICE;
  return TDI_OK;
}

tdi_status tdi_plan_sync(tdi_plan* p) {
  if (!p) return TDI_ESTATE;
  if (hipStreamSynchronize(p->user_stream) != hipSuccess) return TDI_EDEVICE;
  if (hipStreamSynchronize(p->graph_stream) != hipSuccess) return TDI_EDEVICE;
  int32_t info[8] = {0};
  if (hipMemcpy(info, p->d_err, sizeof(info), hipMemcpyDeviceToHost) != hipSuccess) return TDI_EDEVICE;
  if (info[0]) {
    if (getenv("TDI_DEBUG"))
      fprintf(stderr, "tdi: window check failed: codes 0x%x, first: code %d sample %d offset %d len %d\n",
              info[0], info[2], info[3], info[4], info[5]);
    int32_t zero[8] = {0};
    hipMemcpy(p->d_err, zero, sizeof(zero), hipMemcpyHostToDevice);
    return TDI_ERANGE;
  }
  return TDI_OK;
}

tdi_status tdi_plan_kernel_times(tdi_plan* p, float* ms, int32_t cap, int32_t* count) {
  if (!p || !count || (cap > 0 && !ms)) return TDI_EINVAL;
  *count = 0;
  if (hipStreamSynchronize(p->user_stream) != hipSuccess) return TDI_EDEVICE;
  if (hipStreamSynchronize(p->graph_stream) != hipSuccess) return TDI_EDEVICE;
  // three values per run: fit pre-pass, LFA kernel, full kernel
  const int runs = std::min<int>(p->ev_count, cap / 3);
  int first = (p->ev_head - p->ev_count + kEventRing) % kEventRing;
  first = (first + (p->ev_count - runs)) % kEventRing;
  for (int i = 0; i < runs; ++i) {
    const int slot = (first + i) % kEventRing;
    for (int j = 0; j < 3; ++j) {
      float v = 0.0f;
      if (hipEventElapsedTime(&v, p->ev[slot][j], p->ev[slot][j + 1]) != hipSuccess) return TDI_EDEVICE;
      ms[3 * i + j] = v;
    }
  }
  *count = 3 * runs;
  p->ev_count = 0;
  return TDI_OK;
}

tdi_status tdi_plan_describe(const tdi_plan* p, char* buf, int32_t buflen) {
  if (!p || !buf || buflen < 1) return TDI_EINVAL;
  snprintf(buf, (size_t)buflen,
           "{\"tile_lfa\": %d, \"tile_full\": %d, \"grid_lfa\": %d, \"grid_full\": %d, "
           "\"graph\": %d, \"graph_kernel_events\": %d, \"cu\": %d, \"tuned\": %d, \"lfa_fast\": %d, "
           "\"x20_from_x15\": %d, \"tune_cache\": %d}",
           p->last_tile_lfa, p->last_tile_full > 0 ? p->last_tile_full : full_tile(p->cfg), p->launch.grid_lfa,
           p->launch.grid_full,
           (p->cfg.use_graph && !p->stream_pick && !x20_shortcut(p->cfg) && p->launch.grid_lfa > 0 &&
            p->launch.grid_full > 0) ? 1 : 0,
           p->graph_timed ? 1 : 0, p->n_cu,
           p->tuned ? 1 : 0, p->last_fast, x20_shortcut(p->cfg) ? 1 : 0, p->tune_cached ? 1 : 0);
  return TDI_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free entry point.  The memory that a plan allocates for a run
// (parameter block, window-check words, work counters, per-tile records of the
// fast LFA path) lives instead in one file-scope device array, `scratch`, of
// which every GPU holds its own copy.  Host code never passes the array's
// name to a kernel: it takes each device's address once with
// hipGetSymbolAddress and uses that.  The parameter block travels as kernel
// arguments of a small copy kernel (no host staging buffer that must outlive
// the call), and the counters and check words are cleared the same way.
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kNaMaxSources = 256;
constexpr int64_t kNaMaxTiles = 2048;
constexpr int kNaMaxDevices = 64;
constexpr size_t kNaErrOff = 0;            // 8 window-check words (int32)
constexpr size_t kNaCntOff = 256;          // work counters of the persistent kernels
constexpr size_t kNaParOff = 512;          // KParams followed by SrcDev[kNaMaxSources]
constexpr size_t kNaParBytes = sizeof(tdi::KParams) + sizeof(tdi::SrcDev) * (size_t)kNaMaxSources;
constexpr size_t kNaTileOff = (kNaParOff + kNaParBytes + 255) / 256 * 256;
constexpr size_t kNaBytes = kNaTileOff + (size_t)kNaMaxTiles * tdi::kFastTileBytesMax;
constexpr int kPutWords = 512;             // 2 KB of payload per copy-kernel launch

static __device__ __align__(256) unsigned char scratch[kNaBytes];

struct PutArgs {
  uint32_t w[kPutWords];
  uint32_t n;                              // words to write
};

__global__ void k_put(uint32_t* __restrict__ dst, PutArgs a) {
  for (uint32_t i = threadIdx.x; i < a.n; i += blockDim.x) dst[i] = a.w[i];
}

struct NaDevice {
  bool ready;
  unsigned char* ptr;                      // this device's address of scratch
  int n_cu;
  size_t max_lds;
};

NaDevice g_na[kNaMaxDevices];
std::mutex g_na_mu;
// host image of the cleared words and the parameter block, written under g_na_mu
alignas(16) unsigned char g_na_image[kNaParOff + kNaParBytes];

// Once per device, with that device current: gfx950 check, constant tables and
// the device address of scratch.
tdi_status na_setup(int dev) {
  NaDevice& d = g_na[dev];
  if (d.ready) return TDI_OK;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return TDI_EDEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TDI_EDEVICE;
  if (tdi::set_constants() != 0) return TDI_EDEVICE;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TDI_EDEVICE;
  d.ptr = static_cast<unsigned char*>(ptr);
  d.n_cu = prop.multiProcessorCount;
  d.max_lds = prop.sharedMemPerBlock;
  d.ready = true;
  return TDI_OK;
}

// Copy `bytes` (a multiple of 4) of the host image to dst by kernel arguments.
bool na_put(uint32_t* dst, const unsigned char* src, size_t bytes, hipStream_t st) {
  PutArgs a;
  const size_t words = bytes / 4;
  for (size_t w0 = 0; w0 < words; w0 += kPutWords) {
    a.n = (uint32_t)std::min<size_t>(kPutWords, words - w0);
    memcpy(a.w, src + 4 * w0, 4 * (size_t)a.n);
    hipLaunchKernelGGL(k_put, dim3(1), dim3(256), 0, st, dst + w0, a);
    if (hipGetLastError() != hipSuccess) return false;
  }
  return true;
}

}  // namespace

extern "C" {

tdi_status tdi_run_noalloc(const tdi_config* cfg, const tdi_orbit* orb, int64_t n_sources,
                           const tdi_source* src, const int64_t* offsets, const double* hp,
                           const double* hc, void* X, void* Y, void* Z, void* hip_stream) {
  tdi_status st = tdi_check_config(cfg, orb);
  if (st != TDI_OK) return st;
  if (orb->kind == TDI_ORBIT_TABLE) return TDI_EUNSUPPORTED;
  if (x20_shortcut(*cfg)) return TDI_EUNSUPPORTED;
  st = tdi_check_batch(cfg, n_sources, src, offsets);
  if (st != TDI_OK) return st;
  if (n_sources > kNaMaxSources) return TDI_ESTATE;
  const int64_t total = offsets[n_sources];
  if (total == 0) return TDI_OK;
  if (!hp || !hc || !X || !Y || !Z) return TDI_EINVAL;
  const uintptr_t al = cfg->precision == TDI_FP64 ? 8 : 4;
  if (((uintptr_t)hp | (uintptr_t)hc) & 7) return TDI_EINVAL;
  if ((((uintptr_t)X) | ((uintptr_t)Y) | ((uintptr_t)Z)) & (al - 1)) return TDI_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return TDI_EDEVICE;
  if (dev >= kNaMaxDevices) return TDI_EUNSUPPORTED;

  std::lock_guard<std::mutex> lock(g_na_mu);
  st = na_setup(dev);
  if (st != TDI_OK) return st;
  const NaDevice& d = g_na[dev];
  const OrbitBounds ob = orbit_bounds(*orb);
  Caps caps;
  if (!batch_caps(*cfg, ob, n_sources, src, offsets, &caps)) return TDI_OK;
  if (caps.lds_lfa > d.max_lds || caps.lds_full > d.max_lds) return TDI_ERANGE;
  const int taps = cfg->interp_taps, fp32 = cfg->precision;
  Launch ln;
  ln.grid_lfa = tdi::occupancy_lfa(taps, fp32, caps.fast, caps.nx, caps.lds_lfa) * d.n_cu;
  ln.grid_full = tdi::occupancy_full(taps, fp32, caps.hyb, caps.lds_full) * d.n_cu;
  ln.chunks = cfg->fast_tile_chunks != 0 ? cfg->fast_tile_chunks : 4;

  memset(g_na_image, 0, sizeof(g_na_image));
  tdi::KParams* kp = reinterpret_cast<tdi::KParams*>(g_na_image + kNaParOff);
  fill_constants(*kp, *cfg, *orb, ob, nullptr);
  stage_batch(*cfg, kp, n_sources, src, offsets, hp, hc, X, Y, Z, caps, ln, d.n_cu);
  if (caps.fast && kp->n_tiles_lfa > kNaMaxTiles) return TDI_ESTATE;
  kp->err = reinterpret_cast<int32_t*>(d.ptr + kNaErrOff);
  kp->counters = reinterpret_cast<uint32_t*>(d.ptr + kNaCntOff);
  kp->lfa_tiles = d.ptr + kNaTileOff;
  const tdi::KParams* dp = reinterpret_cast<const tdi::KParams*>(d.ptr + kNaParOff);

  // cleared check words and counters, then the parameter block, in one image
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t bytes = kNaParOff + sizeof(tdi::KParams) + sizeof(tdi::SrcDev) * (size_t)n_sources;
  if (!na_put(reinterpret_cast<uint32_t*>(d.ptr), g_na_image, (bytes + 3) / 4 * 4, s)) return TDI_EDEVICE;
  if (kp->n_tiles_lfa > 0) {
    if (caps.fast && tdi::launch_lfa_fit(dp, taps, caps.fit_cu * d.n_cu, s) != 0) return TDI_EDEVICE;
    if (tdi::launch_lfa(dp, taps, fp32, caps.fast, caps.nx, ln.grid_lfa, caps.lds_lfa, s) != 0) return TDI_EDEVICE;
  }
  if (kp->n_tiles_full > 0 && tdi::launch_full(dp, taps, fp32, caps.hyb, ln.grid_full, caps.lds_full, s) != 0)
    return TDI_EDEVICE;
  return TDI_OK;
}

}  // extern "C"
