// Host runtime and C ABI of the hybrid time-domain LISA response (include/tdi.h).
//
// Responsibilities: argument validation (host only, before any device work),
// plan construction (device tables, launch shape, optional hipGraph), per-run
// upload of the small source table, kernel launches and timing records.  No
// response arithmetic runs here; it is all in tdi_kernels.hip.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/tdi.h"
#include "tdi_internal.h"

namespace {

constexpr double kC = 299792458.0;
constexpr int kEventRing = 256;

struct Candidate {
  int tile;
  int grid;          // 0 = one workgroup per tile (non-persistent)
};

}  // namespace

struct tdi_plan {
  tdi_config cfg;
  tdi_orbit orb;
  int64_t max_sources, max_total;
  int device;
  int n_cu;
  hipStream_t user_stream;
  hipStream_t graph_stream;      // private stream used for capture and replay
  // device memory
  void* d_run;                   // RunDesc + SrcDev[max_sources]
  size_t run_bytes;
  int32_t* d_err;
  uint32_t* d_counter;
  // pinned staging for the per-run table
  void* h_run;
  hipEvent_t staged_free;        // recorded after the upload of the previous run
  bool staged_pending;
  // launch choice
  Candidate cand;
  bool tuned;
  // graph
  hipGraph_t graph;
  hipGraphExec_t graph_exec;
  size_t graph_lds;
  int graph_grid, graph_tile;
  // timing
  hipEvent_t ev_start[kEventRing], ev_stop[kEventRing];
  int ev_count;                  // runs recorded since last read (capped)
  int ev_head;
  tdi::KParams kp;               // constant part of the kernel parameters
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
  if (o->kind != TDI_ORBIT_FROZEN && o->kind != TDI_ORBIT_ANALYTIC1) return TDI_EUNSUPPORTED;
  if (o->reserved != 0) return TDI_EINVAL;
  const int N = c->interp_taps;
  if (N != 4 && N != 8 && N != 16 && N != 32) return TDI_ERANGE;
  if (c->stencil_order != 2 && c->stencil_order != 4) return TDI_ERANGE;
  if (c->lfa_equal_arms != 0 && c->lfa_equal_arms != 1) return TDI_ERANGE;
  if (!(c->hyb_T_samples > 0.0) || !is_fin(c->hyb_T_samples)) return TDI_ERANGE;
  if (!(c->hyb_sigma_samples > 0.0) || !is_fin(c->hyb_sigma_samples)) return TDI_ERANGE;
  if (!(o->L_m > 0.0) || !is_fin(o->L_m)) return TDI_ERANGE;
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

// Worst-case staged window lengths (samples) for a tile of 'tile' outputs at
// sampling step dt; the kernel re-checks the actual windows per tile.
void window_caps(const tdi_config& c, const tdi_orbit& o, int tile, double dt,
                 int& cap_g, int& cap_h, int& cap_y) {
  const int N = c.interp_taps;
  const double Lc = o.L_m / kC;
  const double e = o.L_m / (2.0 * sqrt(3.0) * o.R_m);
  const double rate = o.R_m * o.omega * (1.0 + 2.0 * e) / kC + 1e-12;  // |k.V| / c bound
  const double Tmax = Lc * (1.0 + 4.0 * rate) + 1e-9;
  const double Tmin = Lc * (1.0 - 4.0 * rate) - 1e-9;
  const int hw = c.stencil_order == 4 ? 3 : 2;
  auto margin = [](double cnt) { return 2 + (int)ceil(4e-4 * cnt); };
  // LFA: the six delays D_c + mu_l spread over half an arm plus arm differences
  const double mult = c.tdi_gen == 20 ? 2.0 : 1.0;
  const double spread_l = 0.5 * Lc * 1.02 + 2.0 * mult * (Tmax - Tmin) + 2.0 * rate * tile * dt;
  cap_g = tile + (int)ceil(spread_l / dt) + N + 2 * margin(tile) + 4;
  const int h_lfa = cap_g + 2 * hw;
  // full: stage-2 delays reach back (7 or 3) light times
  const double D2 = (c.tdi_gen == 20 ? 7.0 : 3.0) * Tmax;
  cap_y = tile + (int)ceil(D2 / dt) + N + 2 * margin(tile) + 4;
  // stage-1 delays: light time plus spacecraft separations along k
  const double spread_f = Tmax + Lc * 1.02 + 2.0 * rate * cap_y * dt;
  const int h_full = cap_y + (int)ceil(spread_f / dt) + N + 2 * margin(cap_y) + 4;
  cap_h = std::max(h_lfa, h_full);
}

hipError_t upload_and_launch(tdi_plan* p, hipStream_t st, size_t copy_bytes, size_t lds,
                             const Candidate& cd, bool record_events) {
  hipError_t e = hipMemcpyAsync(p->d_run, p->h_run, copy_bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  if (tdi::launch_reset(p->d_counter, p->d_err, 0, st) != 0) return hipErrorLaunchFailure;
  tdi::KParams kp = p->kp;
  kp.tile = cd.tile;
  kp.persistent = cd.grid > 0 ? 1 : 0;
  const tdi::RunDesc* rd = reinterpret_cast<const tdi::RunDesc*>(p->h_run);
  int grid = cd.grid > 0 ? cd.grid : (int)std::max<int64_t>(1, rd->n_tiles);
  if (record_events) hipEventRecord(p->ev_start[p->ev_head], st);
  if (tdi::launch_main(kp, p->cfg.interp_taps, p->cfg.precision, grid, lds, st) != 0)
    return hipErrorLaunchFailure;
  if (record_events) {
    hipEventRecord(p->ev_stop[p->ev_head], st);
    p->ev_head = (p->ev_head + 1) % kEventRing;
    if (p->ev_count < kEventRing) p->ev_count++;
  }
  return hipSuccess;
}

// Fill the pinned run table for one batch; returns the number of tiles.
int64_t stage_batch(tdi_plan* p, int tile, int64_t n_sources, const tdi_source* src,
                    const int64_t* offsets, const double* hp, const double* hc, void* X, void* Y,
                    void* Z, int caps[3]) {
  tdi::RunDesc* rd = reinterpret_cast<tdi::RunDesc*>(p->h_run);
  tdi::SrcDev* sd = reinterpret_cast<tdi::SrcDev*>(rd + 1);
  int64_t tiles = 0;
  for (int64_t i = 0; i < n_sources; ++i) {
    const tdi_source& s = src[i];
    tdi::SrcDev& d = sd[i];
    d.beta = s.beta; d.lam = s.lambda; d.psi = s.psi; d.t0 = s.t0; d.dt = s.dt; d.t_hyb = s.t_hyb;
    d.off = offsets[i];
    d.n = offsets[i + 1] - offsets[i];
    d.tile0 = tiles;
    d.pad = 0;
    tiles += (d.n + tile - 1) / tile;
  }
  rd->n_src = n_sources;
  rd->n_tiles = tiles;
  rd->hp = hp; rd->hc = hc; rd->X = X; rd->Y = Y; rd->Z = Z;
  rd->cap_g = caps[0]; rd->cap_h = caps[1]; rd->cap_y = caps[2];
  rd->pad = 0;
  return tiles;
}

void destroy_graph(tdi_plan* p) {
  if (p->graph_exec) hipGraphExecDestroy(p->graph_exec);
  if (p->graph) hipGraphDestroy(p->graph);
  p->graph_exec = nullptr;
  p->graph = nullptr;
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

  tdi_plan* p = (tdi_plan*)calloc(1, sizeof(tdi_plan));
  if (!p) return TDI_ENOMEM;
  p->cfg = *cfg;
  p->orb = *orb;
  p->max_sources = max_sources;
  p->max_total = max_total_samples;
  p->device = dev;
  p->n_cu = prop.multiProcessorCount;
  p->user_stream = (hipStream_t)hip_stream;
  p->run_bytes = sizeof(tdi::RunDesc) + sizeof(tdi::SrcDev) * (size_t)max_sources;
  bool ok = hipMalloc(&p->d_run, p->run_bytes) == hipSuccess;
  ok = ok && hipMalloc((void**)&p->d_err, 64) == hipSuccess;
  ok = ok && hipMalloc((void**)&p->d_counter, 64) == hipSuccess;
  ok = ok && hipHostMalloc(&p->h_run, p->run_bytes, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&p->staged_free, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&p->graph_stream, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; ok && i < kEventRing; ++i) {
    ok = hipEventCreate(&p->ev_start[i]) == hipSuccess && hipEventCreate(&p->ev_stop[i]) == hipSuccess;
  }
  if (!ok) {
    tdi_plan_destroy(p);
    return TDI_ENOMEM;
  }
  hipMemset(p->d_err, 0, 64);
  hipMemset(p->d_counter, 0, 64);
  hipDeviceSynchronize();

  // constant kernel parameters
  tdi::KParams& kp = p->kp;
  memset(&kp, 0, sizeof(kp));
  kp.rd = reinterpret_cast<const tdi::RunDesc*>(p->d_run);
  kp.src = reinterpret_cast<const tdi::SrcDev*>(reinterpret_cast<const tdi::RunDesc*>(p->d_run) + 1);
  kp.err_flag = p->d_err;
  kp.counter = p->d_counter;
  tdi::OrbitDev& od = kp.orb;
  od.kind = orb->kind;
  od.L = orb->L_m;
  od.R = orb->R_m;
  od.omega = orb->omega;
  od.kappa0 = orb->kappa0;
  od.t_freeze = orb->t_freeze;
  od.e = orb->L_m / (2.0 * sqrt(3.0) * orb->R_m);
  for (int i = 0; i < 3; ++i) {
    double b = 2.0 * M_PI * (double)i / 3.0 + orb->lambda0;
    od.cb[i] = cos(b);
    od.sb[i] = sin(b);
  }
  od.L_over_c = orb->L_m / kC;
  kp.gen = cfg->tdi_gen;
  kp.mode = cfg->mode;
  kp.equal_arms = cfg->lfa_equal_arms;
  kp.stencil_m = cfg->tdi_gen == 20 ? 3 : 2;
  kp.T_s = cfg->hyb_T_samples;
  kp.sigma_s = cfg->hyb_sigma_samples;
  const int N = cfg->interp_taps;
  for (int a = 0; a < N; ++a) {          // 1 / prod_{m != j} (j - m), nodes j = a - N/2 + 1
    int j = a - N / 2 + 1;
    double prod = 1.0;
    for (int b = 0; b < N; ++b) {
      int m = b - N / 2 + 1;
      if (m != j) prod *= (double)(j - m);
    }
    kp.lag_c[a] = 1.0 / prod;
  }
  // central stencils of derivative order m (2 for TDI 1.5, 3 for TDI 2.0) and accuracy p
  static const double s22[] = {1, -2, 1}, s24[] = {-1, 16, -30, 16, -1};
  static const double s32[] = {-1, 2, 0, -2, 1}, s34[] = {1, -8, 13, 0, -13, 8, -1};
  const double* num;
  if (kp.stencil_m == 2) {
    if (cfg->stencil_order == 2) { num = s22; kp.st_hw = 1; kp.st_den = 1.0; }
    else { num = s24; kp.st_hw = 2; kp.st_den = 12.0; }
  } else {
    if (cfg->stencil_order == 2) { num = s32; kp.st_hw = 2; kp.st_den = 2.0; }
    else { num = s34; kp.st_hw = 3; kp.st_den = 8.0; }
  }
  for (int s = 0; s < 2 * kp.st_hw + 1; ++s) kp.st_num[s] = num[s];
  p->cand.tile = 256;
  p->cand.grid = 0;
  p->tuned = cfg->autotune ? false : true;
  *out = p;
  return TDI_OK;
}

tdi_status tdi_plan_destroy(tdi_plan* p) {
  if (!p) return TDI_EINVAL;
  if (p->graph_stream) hipStreamSynchronize(p->graph_stream);
  if (p->user_stream || true) hipStreamSynchronize(p->user_stream);
  destroy_graph(p);
  for (int i = 0; i < kEventRing; ++i) {
    if (p->ev_start[i]) hipEventDestroy(p->ev_start[i]);
    if (p->ev_stop[i]) hipEventDestroy(p->ev_stop[i]);
  }
  if (p->staged_free) hipEventDestroy(p->staged_free);
  if (p->graph_stream) hipStreamDestroy(p->graph_stream);
  if (p->d_run) hipFree(p->d_run);
  if (p->d_err) hipFree(p->d_err);
  if (p->d_counter) hipFree(p->d_counter);
  if (p->h_run) hipHostFree(p->h_run);
  free(p);
  return TDI_OK;
}

static tdi_status run_with(tdi_plan* p, const Candidate& cd, int64_t n_sources,
                           const tdi_source* src, const int64_t* offsets, const double* hp,
                           const double* hc, void* X, void* Y, void* Z, bool record) {
  double dt_min = INFINITY;
  for (int64_t i = 0; i < n_sources; ++i)
    if (offsets[i + 1] > offsets[i]) dt_min = std::min(dt_min, src[i].dt);
  int caps[3] = {0, 0, 0};
  if (isfinite(dt_min)) window_caps(p->cfg, p->orb, cd.tile, dt_min, caps[0], caps[1], caps[2]);
  size_t lds = tdi::lds_bytes_for(cd.tile, caps[0], caps[1], caps[2], p->cfg.precision);
  if (lds > (size_t)tdi::max_lds_bytes()) return TDI_ERANGE;

  // the previous upload must have left the pinned buffer before it is rewritten
  if (p->staged_pending) {
    if (hipEventSynchronize(p->staged_free) != hipSuccess) return TDI_EDEVICE;
    p->staged_pending = false;
  }
  int64_t tiles = stage_batch(p, cd.tile, n_sources, src, offsets, hp, hc, X, Y, Z, caps);
  if (tiles == 0) return TDI_OK;
  const size_t copy_bytes = sizeof(tdi::RunDesc) + sizeof(tdi::SrcDev) * (size_t)n_sources;

  if (p->cfg.use_graph && cd.grid > 0) {
    // replay a graph of (upload max table, reset, persistent kernel) on the
    // private stream, ordered after the caller's stream and back
    if (!p->graph_exec || p->graph_lds != lds || p->graph_grid != cd.grid || p->graph_tile != cd.tile) {
      destroy_graph(p);
      if (hipStreamBeginCapture(p->graph_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return TDI_EDEVICE;
      hipError_t e = upload_and_launch(p, p->graph_stream, p->run_bytes, lds, cd, false);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(p->graph_stream, &g);
      if (e != hipSuccess || e2 != hipSuccess || !g) {
        if (g) hipGraphDestroy(g);
        return TDI_EDEVICE;
      }
      p->graph = g;
      if (hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
        destroy_graph(p);
        return TDI_EDEVICE;
      }
      p->graph_lds = lds;
      p->graph_grid = cd.grid;
      p->graph_tile = cd.tile;
    }
    hipEvent_t ev = p->ev_start[p->ev_head];
    if (hipEventRecord(ev, p->user_stream) != hipSuccess) return TDI_EDEVICE;
    if (hipStreamWaitEvent(p->graph_stream, ev, 0) != hipSuccess) return TDI_EDEVICE;
    if (record) hipEventRecord(p->ev_start[p->ev_head], p->graph_stream);
    if (hipGraphLaunch(p->graph_exec, p->graph_stream) != hipSuccess) return TDI_EDEVICE;
    hipEventRecord(p->ev_stop[p->ev_head], p->graph_stream);
    hipEventRecord(p->staged_free, p->graph_stream);
    p->staged_pending = true;
    if (hipStreamWaitEvent(p->user_stream, p->ev_stop[p->ev_head], 0) != hipSuccess) return TDI_EDEVICE;
    if (record) {
      p->ev_head = (p->ev_head + 1) % kEventRing;
      if (p->ev_count < kEventRing) p->ev_count++;
    }
    return TDI_OK;
  }
  hipError_t e = upload_and_launch(p, p->user_stream, copy_bytes, lds, cd, record);
  if (e != hipSuccess) return TDI_EDEVICE;
  hipEventRecord(p->staged_free, p->user_stream);
  p->staged_pending = true;
  return TDI_OK;
}

static void autotune(tdi_plan* p, int64_t n_sources, const tdi_source* src, const int64_t* offsets,
                     const double* hp, const double* hc, void* X, void* Y, void* Z) {
  std::vector<Candidate> cands;
  for (int tile : {256, 512}) {
    cands.push_back({tile, 0});
    for (int per_cu : {1, 2, 3, 4}) cands.push_back({tile, per_cu * p->n_cu});
  }
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  float best = INFINITY;
  Candidate best_c = p->cand;
  for (const Candidate& cd : cands) {
    float tsum = 0.0f;
    bool ok = true;
    for (int rep = 0; rep < 2 && ok; ++rep) {
      hipEventRecord(a, p->user_stream);
      Candidate c0 = cd;
      bool ug = p->cfg.use_graph;
      p->cfg.use_graph = 0;
      tdi_status s = run_with(p, c0, n_sources, src, offsets, hp, hc, X, Y, Z, false);
      p->cfg.use_graph = ug;
      hipEventRecord(b, p->user_stream);
      if (s != TDI_OK || hipEventSynchronize(b) != hipSuccess) { ok = false; break; }
      float ms = 0.0f;
      hipEventElapsedTime(&ms, a, b);
      if (rep == 1) tsum += ms;
    }
    if (ok && tsum < best) { best = tsum; best_c = cd; }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  p->cand = best_c;
  p->tuned = true;
}

tdi_status tdi_run(tdi_plan* p, int64_t n_sources, const tdi_source* src, const int64_t* offsets,
                   const double* hp, const double* hc, void* X, void* Y, void* Z) {
  if (!p) return TDI_ESTATE;
  tdi_status st = tdi_check_batch(&p->cfg, n_sources, src, offsets);
  if (st != TDI_OK) return st;
  if (n_sources > p->max_sources || offsets[n_sources] > p->max_total) return TDI_ESTATE;
  const int64_t total = offsets[n_sources];
  if (total > 0) {
    if (!hp || !hc || !X || !Y || !Z) return TDI_EINVAL;
    const uintptr_t al = p->cfg.precision == TDI_FP64 ? 8 : 4;
    if (((uintptr_t)hp | (uintptr_t)hc) & 7) return TDI_EINVAL;
    if ((((uintptr_t)X) | ((uintptr_t)Y) | ((uintptr_t)Z)) & (al - 1)) return TDI_EINVAL;
  } else {
    return TDI_OK;
  }
  if (!p->tuned) autotune(p, n_sources, src, offsets, hp, hc, X, Y, Z);
  return run_with(p, p->cand, n_sources, src, offsets, hp, hc, X, Y, Z, true);
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
  int n = std::min<int>(p->ev_count, cap);
  int first = (p->ev_head - p->ev_count + kEventRing) % kEventRing;
  first = (first + (p->ev_count - n)) % kEventRing;
  for (int i = 0; i < n; ++i) {
    int slot = (first + i) % kEventRing;
    float v = 0.0f;
    if (hipEventElapsedTime(&v, p->ev_start[slot], p->ev_stop[slot]) != hipSuccess) return TDI_EDEVICE;
    ms[i] = v;
  }
  *count = n;
  p->ev_count = 0;
  return TDI_OK;
}

tdi_status tdi_plan_describe(const tdi_plan* p, char* buf, int32_t buflen) {
  if (!p || !buf || buflen < 1) return TDI_EINVAL;
  snprintf(buf, (size_t)buflen,
           "{\"tile\": %d, \"grid\": %d, \"persistent\": %d, \"graph\": %d, \"cu\": %d, \"tuned\": %d}",
           p->cand.tile, p->cand.grid, p->cand.grid > 0 ? 1 : 0,
           (p->cfg.use_graph && p->cand.grid > 0) ? 1 : 0, p->n_cu, p->tuned ? 1 : 0);
  return TDI_OK;
}

}  // extern "C"
