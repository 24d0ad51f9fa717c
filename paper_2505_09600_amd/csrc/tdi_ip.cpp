// Host runtime of the noise-weighted inner product (include/tdi.h, tdi_ip_*).
//
// Validates the noise description and batches on the host, builds the table
// of 1 / S_n (Sec. II.C, Eqs. SnAE and SnT, with the galactic foreground of
// Eq. sgal) once per plan, splits each source's zero-extended transform into
// the two passes of tdi_ip_kernels.hip, uploads the per-source records and
// launches the kernels.  No transform or sum runs here.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/tdi.h"
#include "tdi_ip_internal.h"

namespace {

constexpr double kC = 299792458.0;
constexpr int kRing = 64;        // remembered runs for tdi_ip_kernel_times

// Sec. II.C noise model (fractional-frequency PSDs)
constexpr double kSqrtSacc = 2.4e-15;     // m s^-2 Hz^-1/2
constexpr double kSqrtSoms = 7.9e-12;     // m Hz^-1/2
constexpr double kGalA = 1.28265531e-44, kGalAlpha = 1.62966700, kGalF2 = 4.81078093e-4;
constexpr double kGalA1 = -0.223499956, kGalB1 = -2.70408439;
constexpr double kGalAk = -0.360976122, kGalBk = -2.37822436;

struct Psd {
  double L, f1, fknee;
  int gen, gal;
  explicit Psd(const tdi_noise& n)
      : L(n.L_m),
        f1(pow(10.0, kGalA1 * log10(n.T_obs_years) + kGalB1)),
        fknee(pow(10.0, kGalAk * log10(n.T_obs_years) + kGalBk)),
        gen(n.tdi_gen),
        gal(n.galactic) {}
  // returns S_AE and S_T at f > 0
  void eval(double f, double* sae, double* st) const {
    const double pi = M_PI;
    const double x = 2.0 * pi * f * L / kC;
    const double spm = kSqrtSacc * kSqrtSacc / ((2.0 * pi * f * kC) * (2.0 * pi * f * kC)) *
                       (1.0 + (4.0e-4 / f) * (4.0e-4 / f)) * (1.0 + pow(f / 8.0e-3, 4.0));
    const double sop = kSqrtSoms * kSqrtSoms * (2.0 * pi * f / kC) * (2.0 * pi * f / kC) *
                       (1.0 + pow(2.0e-3 / f, 4.0));
    const double lam = gen == 20 ? 4.0 * sin(2.0 * x) * sin(2.0 * x) : 1.0;
    const double sx2 = sin(x) * sin(x);
    double g = 0.0;
    if (gal) {
      g = 2.0 * x * x * sx2 * kGalA * pow(f, -7.0 / 3.0) * exp(-pow(f / f1, kGalAlpha)) *
          (1.0 + tanh((fknee - f) / kGalF2));
    }
    const double sh = sin(0.5 * x);
    *sae = 8.0 * lam * sx2 * (2.0 * (3.0 + 2.0 * cos(x) + cos(2.0 * x)) * spm + (2.0 + cos(x)) * sop) +
           1.5 * lam * g;
    *st = 16.0 * lam * sx2 * ((1.0 - cos(x)) * sop + 8.0 * sh * sh * sh * sh * spm) + lam * g;
  }
};

// e^{-2 pi i m / 2^logM} for m in [0, count), stored as (re, im) pairs of T
template <typename T>
std::vector<T> roots(int64_t count, int logM, int64_t stride) {
  std::vector<T> v(2 * (size_t)count);
  const double M = ldexp(1.0, logM);
  for (int64_t m = 0; m < count; ++m) {
    const double a = 2.0 * M_PI * ((double)(m * stride) / M);
    v[2 * (size_t)m] = (T)cos(a);
    v[2 * (size_t)m + 1] = (T)(-sin(a));
  }
  return v;
}

template <typename T>
bool upload_roots(void** dst, int64_t count, int logM, int64_t stride) {
  const std::vector<T> v = roots<T>(count, logM, stride);
  if (hipMalloc(dst, sizeof(T) * v.size()) != hipSuccess) return false;
  return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) == hipSuccess;
}

int log2_fft_length(int64_t n) {
  int lg = 1;
  while (((int64_t)1 << lg) < n) ++lg;
  return lg;
}

// the two-pass split of one source (N1 = 1: one pass)
struct Split {
  int logN, logN1, logN2, cols, n1, n2;
};

// pass-1 and pass-2 tile elements (log2) of the transform precision
int log_tile(int fp64, int pass) {
  return fp64 ? (pass == 1 ? tdi_ip::Tile<double, 1>::kLogE : tdi_ip::Tile<double, 2>::kLogE)
              : (pass == 1 ? tdi_ip::Tile<float, 1>::kLogE : tdi_ip::Tile<float, 2>::kLogE);
}

bool split_of(int64_t n, int fp64, Split* s) {
  const int E1 = 1 << log_tile(fp64, 1), logE2 = log_tile(fp64, 2);
  s->logN = log2_fft_length(n);
  if (s->logN <= logE2) {
    *s = {s->logN, 0, s->logN, 0, 0, n > 0 ? 1 : 0};
    return true;
  }
  s->logN2 = logE2 - 1;                    // two rows of the second pass share its tile
  s->logN1 = s->logN - s->logN2;
  const int N1 = 1 << s->logN1, N2 = 1 << s->logN2;
  if (N1 > E1 / 2) return false;           // at least two columns per first-pass task
  s->cols = std::min(E1 / N1, N2);
  s->n1 = N2 / s->cols;
  s->n2 = N1 / 2 + 1;
  return true;
}

}  // namespace

struct tdi_ip_plan {
  tdi_noise noise;
  int32_t precision;
  double dt;
  int64_t max_sources, max_total, max_source;
  int logNmax;
  int grid1, grid2;               // persistent workgroups of the passes (resident count, multiple of 8)
  hipStream_t stream;
  void* d_wt;                     // weight tables, one per length, transform precision (see IpParams)
  int32_t wexp;                   // power-of-two scale of the FP32 weight table
  int64_t wofs[32];               // offset of the table of length 2^logN
  void* d_tw;                     // twiddle tables (see IpParams)
  void* d_th;
  void* d_tl;
  int tbits;
  void* d_ws;
  int64_t ws_cap;                 // complex elements
  double* d_part;
  int64_t part_cap;               // pass-2 tasks
  tdi_ip::IpParams* d_params;
  tdi_ip::IpParams* h_params;     // pinned staging image
  size_t params_bytes;
  hipEvent_t staged_free;
  bool staged_pending;
  hipEvent_t ev[kRing][4];
  int ev_count, ev_head;
};

extern "C" {

tdi_status tdi_check_noise(const tdi_noise* n) {
  if (!n) return TDI_EINVAL;
  if (n->tdi_gen != 15 && n->tdi_gen != 20) return TDI_EUNSUPPORTED;
  if (n->galactic != 0 && n->galactic != 1) return TDI_ERANGE;
  if (!(n->T_obs_years > 0.0) || !isfinite(n->T_obs_years)) return TDI_ERANGE;
  if (!(n->L_m > 0.0) || !isfinite(n->L_m)) return TDI_ERANGE;
  if (!(n->f_min > 0.0) || !(n->f_max > n->f_min) || !isfinite(n->f_max)) return TDI_ERANGE;
  // the first zero of the PSD: sin 2x (TDI 2.0) or sin x (TDI 1.5)
  const double f_zero = kC / ((n->tdi_gen == 20 ? 4.0 : 2.0) * n->L_m);
  if (!(n->f_max < f_zero)) return TDI_ERANGE;
  return TDI_OK;
}

tdi_status tdi_ip_plan_destroy(tdi_ip_plan* p) {
  if (!p) return TDI_EINVAL;
  (void)hipStreamSynchronize(p->stream);
  if (p->d_wt) hipFree(p->d_wt);
  if (p->d_tw) hipFree(p->d_tw);
  if (p->d_th) hipFree(p->d_th);
  if (p->d_tl) hipFree(p->d_tl);
  if (p->d_ws) hipFree(p->d_ws);
  if (p->d_part) hipFree(p->d_part);
  if (p->d_params) hipFree(p->d_params);
  if (p->h_params) hipHostFree(p->h_params);
  if (p->staged_free) hipEventDestroy(p->staged_free);
  for (int i = 0; i < kRing; ++i)
    for (int j = 0; j < 4; ++j)
      if (p->ev[i][j]) hipEventDestroy(p->ev[i][j]);
  free(p);
  return TDI_OK;
}

tdi_status tdi_ip_plan_create(tdi_ip_plan** out, const tdi_noise* noise, int32_t precision, double dt,
                              int64_t max_sources, int64_t max_total_samples, int64_t max_source_samples,
                              void* hip_stream) {
  if (!out) return TDI_EINVAL;
  *out = nullptr;
  tdi_status st = tdi_check_noise(noise);
  if (st != TDI_OK) return st;
  if (precision != TDI_FP64 && precision != TDI_FP32_BULK) return TDI_EUNSUPPORTED;
  if (!(dt > 0.0) || !isfinite(dt)) return TDI_ERANGE;
  if (max_sources < 1 || max_total_samples < 0 || max_source_samples < 1) return TDI_EINVAL;
  const int fp64 = precision == TDI_FP64;
  Split sp;
  if (!split_of(max_source_samples, fp64, &sp)) return TDI_ERANGE;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return TDI_EDEVICE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TDI_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return TDI_EDEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TDI_EDEVICE;

  tdi_ip_plan* p = (tdi_ip_plan*)calloc(1, sizeof(tdi_ip_plan));
  if (!p) return TDI_ENOMEM;
  p->noise = *noise;
  p->precision = precision;
  p->dt = dt;
  p->max_sources = max_sources;
  p->max_total = max_total_samples;
  p->max_source = max_source_samples;
  p->logNmax = sp.logN;
  const int per1 = fp64 ? tdi_ip::Tile<double, 1>::kPerCu : tdi_ip::Tile<float, 1>::kPerCu;
  const int per2 = fp64 ? tdi_ip::Tile<double, 2>::kPerCu : tdi_ip::Tile<float, 2>::kPerCu;
  p->grid1 = std::max(8, (per1 * prop.multiProcessorCount + 7) & ~7);
  p->grid2 = std::max(8, (per2 * prop.multiProcessorCount + 7) & ~7);
  p->stream = (hipStream_t)hip_stream;
  const int64_t row = (int64_t)1 << (log_tile(fp64, 2) - 1);
  const size_t vbytes = fp64 ? 16 : 8;
  // every zero-extended length is below twice the source length; three channels
  p->ws_cap = 6 * std::max<int64_t>(max_total_samples, 1);
  p->part_cap = 3 * (max_total_samples / row + max_sources) + 3;
  p->params_bytes = sizeof(tdi_ip::IpParams) + sizeof(tdi_ip::IpSrc) * (size_t)max_sources;
  // weight tables for every length 2^1 .. N_max: N entries each (two classes of N/2)
  int64_t wt_total = 0;
  for (int lg = 1; lg <= sp.logN; ++lg) {
    p->wofs[lg] = wt_total;
    wt_total += (int64_t)1 << lg;
  }
  const size_t wbytes = fp64 ? sizeof(double) : sizeof(float);
  bool ok = hipMalloc(&p->d_wt, wbytes * (size_t)wt_total) == hipSuccess;
  ok = ok && hipMalloc(&p->d_ws, vbytes * (size_t)p->ws_cap) == hipSuccess;
  ok = ok && hipMalloc((void**)&p->d_part, sizeof(double) * 3 * (size_t)p->part_cap) == hipSuccess;
  ok = ok && hipMalloc((void**)&p->d_params, p->params_bytes) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&p->h_params, p->params_bytes, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&p->staged_free, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < kRing; ++i)
    for (int j = 0; ok && j < 4; ++j) ok = hipEventCreate(&p->ev[i][j]) == hipSuccess;
  if (!ok) {
    tdi_ip_plan_destroy(p);
    return TDI_ENOMEM;
  }
  // 1 / S_n on the finest grid f = k / (N_max dt), k < N_max / 2; a length
  // N = N_max / 2^s reads entry k 2^s.  Each length's table is reordered to
  // the second pass's bin order and zeroed outside the band [f_min, f_max].
  const int64_t half_max = ((int64_t)1 << sp.logN) / 2;
  std::vector<double> base(2 * (size_t)half_max, 0.0);
  const Psd psd(*noise);
  const double Ndt_max = (double)((int64_t)1 << sp.logN) * dt;
  for (int64_t k = 1; k < half_max; ++k) {
    double sae, stt;
    psd.eval((double)k / Ndt_max, &sae, &stt);
    base[2 * (size_t)k] = sae > 0.0 ? 1.0 / sae : 0.0;
    base[2 * (size_t)k + 1] = stt > 0.0 ? 1.0 / stt : 0.0;
  }
  std::vector<double> wt((size_t)wt_total, 0.0);
  for (int lg = 1; lg <= sp.logN; ++lg) {
    Split s;
    split_of((int64_t)1 << lg, fp64, &s);
    const int64_t N = (int64_t)1 << lg, N1 = (int64_t)1 << s.logN1, hw = ((int64_t)1 << s.logN2) / 2;
    const double Ndt = (double)N * dt;
    double* t = wt.data() + p->wofs[lg];
    for (int64_t k1 = 0; k1 < N1; ++k1) {
      for (int64_t k2 = 0; k2 < hw; ++k2) {
        const int64_t k = k1 + N1 * k2;
        const double f = (double)k / Ndt;
        if (k < 1 || f < noise->f_min || f > noise->f_max) continue;
        const size_t kb = (size_t)(k << (sp.logN - lg));
        t[k1 * hw + k2] = base[2 * kb];
        t[N / 2 + k1 * hw + k2] = base[2 * kb + 1];
      }
    }
  }
  // FP32 transforms read the weights scaled by 2^-wexp (largest weight in
  // [0.5, 1)) and rounded once to FP32; the reduction multiplies by 2^wexp
  p->wexp = 0;
  std::vector<float> wt32(fp64 ? 0 : wt.size());
  if (!fp64) {
    double wmax = 0.0;
    for (double v : wt) wmax = std::max(wmax, v);
    if (wmax > 0.0) frexp(wmax, &p->wexp);
    for (size_t i = 0; i < wt32.size(); ++i) wt32[i] = (float)ldexp(wt[i], -p->wexp);
  }
  const void* wsrc = fp64 ? (const void*)wt.data() : (const void*)wt32.data();
  if (hipMemcpy(p->d_wt, wsrc, wbytes * wt.size(), hipMemcpyHostToDevice) != hipSuccess) {
    tdi_ip_plan_destroy(p);
    return TDI_EDEVICE;
  }
  // twiddles: LDS stages (2^log_tw roots of unity) and the four-step factor
  // e^{-2 pi i m / N_max} split as th[m >> tbits] tl[m mod 2^tbits]
  const int logE = fp64 ? tdi_ip::log_tw<double>() : tdi_ip::log_tw<float>();
  p->tbits = (sp.logN + 1) / 2;
  const int64_t nh = (int64_t)1 << (sp.logN - p->tbits), nl = (int64_t)1 << p->tbits;
  ok = fp64 ? upload_roots<double>(&p->d_tw, (int64_t)1 << logE, logE, 1) &&
                  upload_roots<double>(&p->d_th, nh, sp.logN, nl) &&
                  upload_roots<double>(&p->d_tl, nl, sp.logN, 1)
            : upload_roots<float>(&p->d_tw, (int64_t)1 << logE, logE, 1) &&
                  upload_roots<float>(&p->d_th, nh, sp.logN, nl) &&
                  upload_roots<float>(&p->d_tl, nl, sp.logN, 1);
  if (!ok) {
    tdi_ip_plan_destroy(p);
    return TDI_ENOMEM;
  }
  *out = p;
  return TDI_OK;
}

tdi_status tdi_ip_run(tdi_ip_plan* p, int64_t n_sources, const int64_t* offsets,
                      const void* const* x, const void* const* y, double* out) {
  if (!p || !offsets || !x || !y) return TDI_EINVAL;
  if (n_sources < 0 || offsets[0] != 0) return TDI_EINVAL;
  if (n_sources > p->max_sources) return TDI_ESTATE;
  const int fp64 = p->precision == TDI_FP64;
  const size_t tb = fp64 ? 8 : 4;
  for (int64_t i = 0; i < n_sources; ++i) {
    if (offsets[i + 1] < offsets[i]) return TDI_EINVAL;
    if (offsets[i + 1] - offsets[i] > p->max_source) return TDI_ESTATE;
  }
  const int64_t total = offsets[n_sources];
  if (total > p->max_total) return TDI_ESTATE;
  if (n_sources > 0 && !out) return TDI_EINVAL;
  if (((uintptr_t)out & 7) != 0) return TDI_EINVAL;
  for (int c = 0; c < 3; ++c) {
    if (total > 0 && (!x[c] || !y[c])) return TDI_EINVAL;
    if (((uintptr_t)x[c] % tb) != 0 || ((uintptr_t)y[c] % tb) != 0) return TDI_EINVAL;
  }
  if (n_sources == 0) return TDI_OK;

  // wait until the previous run's upload has left the pinned image
  if (p->staged_pending) {
    if (hipEventSynchronize(p->staged_free) != hipSuccess) return TDI_EDEVICE;
    p->staged_pending = false;
  }
  tdi_ip::IpParams& P = *p->h_params;
  tdi_ip::IpSrc* S = reinterpret_cast<tdi_ip::IpSrc*>(p->h_params + 1);
  int64_t t1 = 0, t2 = 0, part = 0, ws = 0;
  for (int64_t i = 0; i < n_sources; ++i) {
    const int64_t n = offsets[i + 1] - offsets[i];
    Split sp;
    if (!split_of(n, fp64, &sp)) return TDI_ESTATE;
    tdi_ip::IpSrc& r = S[i];
    r.off = offsets[i];
    r.n = n;
    r.logN = sp.logN;
    r.logN1 = sp.logN1;
    r.logN2 = sp.logN2;
    r.cols = sp.cols;
    r.n1 = sp.n1;
    r.n2 = sp.n2;
    r.t1 = t1;
    r.t2 = t2;
    r.part = part;
    r.ws = ws;
    r.wofs = p->wofs[sp.logN];
    t1 += 3 * (int64_t)sp.n1;
    t2 += 3 * (int64_t)sp.n2;
    part += 3 * (int64_t)sp.n2;
    if (sp.logN1 > 0) ws += 3 * ((int64_t)1 << sp.logN);
  }
  if (ws > p->ws_cap || part > p->part_cap) return TDI_ESTATE;
  P.n_src = n_sources;
  P.n_t1 = t1;
  P.n_t2 = t2;
  for (int c = 0; c < 3; ++c) {
    P.x[c] = x[c];
    P.y[c] = y[c];
  }
  P.ws = p->d_ws;
  P.part = p->d_part;
  P.out = out;
  P.wt = p->d_wt;
  P.wexp = p->wexp;
  P.tw = p->d_tw;
  P.th = p->d_th;
  P.tl = p->d_tl;
  P.tbits = p->tbits;
  P.logNmax = p->logNmax;
  P.dt = p->dt;
  P.f_min = p->noise.f_min;
  P.f_max = p->noise.f_max;
  const size_t bytes = sizeof(tdi_ip::IpParams) + sizeof(tdi_ip::IpSrc) * (size_t)n_sources;
  hipStream_t s = p->stream;
  if (hipMemcpyAsync(p->d_params, p->h_params, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
    return TDI_EDEVICE;
  if (hipEventRecord(p->staged_free, s) != hipSuccess) return TDI_EDEVICE;
  p->staged_pending = true;
  const int slot = p->ev_head;
  bool ok = hipEventRecord(p->ev[slot][0], s) == hipSuccess;
  ok = ok && tdi_ip::launch_pass1(p->d_params, fp64, t1, p->grid1, s) == 0;
  ok = ok && hipEventRecord(p->ev[slot][1], s) == hipSuccess;
  ok = ok && tdi_ip::launch_pass2(p->d_params, fp64, t2, p->grid2, s) == 0;
  ok = ok && hipEventRecord(p->ev[slot][2], s) == hipSuccess;
  ok = ok && tdi_ip::launch_reduce(p->d_params, n_sources, s) == 0;
  ok = ok && hipEventRecord(p->ev[slot][3], s) == hipSuccess;
  if (!ok) return TDI_EDEVICE;
  p->ev_head = (p->ev_head + 1) % kRing;
  p->ev_count = std::min(p->ev_count + 1, kRing);
  return TDI_OK;
}

tdi_status tdi_ip_kernel_times(tdi_ip_plan* p, float* ms, int32_t cap, int32_t* count) {
  if (!p || !count || (cap > 0 && !ms)) return TDI_EINVAL;
  *count = 0;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return TDI_EDEVICE;
  const int runs = std::min<int>(p->ev_count, cap / 3);
  int first = (p->ev_head - p->ev_count + kRing) % kRing;
  first = (first + (p->ev_count - runs)) % kRing;
  for (int i = 0; i < runs; ++i) {
    const int slot = (first + i) % kRing;
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

}  // extern "C"
