// Device kernels of the hybrid time-domain LISA response for gfx950.
//
// One launch processes a batch of sources split into tiles of output samples.
// A tile is handled by one 256-thread workgroup and, depending on the mode and
// on where the tile sits relative to the hybrid window, runs
//   * the LFA phase  : FP64 central stencil of the strain staged in LDS, then
//                      six two-component fractional-delay reads per output
//                      (App. B, Eqs. X15_nonequal_timedelays / X20_nonequal_timedelays
//                      with the single-link LFA of Eq. yslr_strain_derivatives);
//   * the full phase : stage 1 builds the six link series y_l on an LDS window
//                      (Eq. yslr with Eq. H), stage 2 forms X, Y, Z from the
//                      TDI term lists with arm delays evaluated at the output
//                      time (Eqs. X1.5, X2.0);
//   * the blend      : sigmoid weights of Eqs. (sigmoid, hybridized_xs).
// Orbit geometry, retarded-time arguments and stencils are FP64; the compute
// type TC of the interpolation and TDI arithmetic is double or float.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tdi_internal.h"

namespace tdi {
namespace {

constexpr double kC = 299792458.0;

// Link slots +1,+2,+3,-1,-2,-3 -> sender / receiver spacecraft (0-based).
// Link l joins the two spacecraft other than |l| with sgn(l) = eps_{s|l|r}.
__constant__ int c_snd[6] = {2, 0, 1, 1, 2, 0};
__constant__ int c_rcv[6] = {1, 2, 0, 2, 0, 1};

// TDI Michelson X terms: sign, link slot of y, number of delays, delay slots
// (in the order written in Eqs. X1.5 and X2.0).  Y and Z: cyclic relabelling.
struct Term { int sign, link, nd, d[7]; };
__constant__ Term c_terms[16] = {
    {+1, 5, 3, {4, 1, 2}},                  // y_{1-32}(t - L-2 - L2 - L3)
    {-1, 5, 1, {2}},                        // y_{1-32}(t - L3)
    {+1, 2, 2, {1, 4}},                     // y_{231}(t - L2 - L-2)
    {-1, 2, 0, {0}},                        // y_{231}(t)
    {+1, 1, 1, {4}},                        // y_{123}(t - L-2)
    {-1, 1, 3, {4, 5, 2}},                  // y_{123}(t - L-2 - L-3 - L3)
    {+1, 4, 0, {0}},                        // y_{3-21}(t)
    {-1, 4, 2, {5, 2}},                     // y_{3-21}(t - L-3 - L3)
    {+1, 5, 5, {4, 1, 2, 2, 5}},            // y_{1-32}(t - L-2 - L2 - 2L3 - L-3)
    {-1, 5, 7, {2, 2, 5, 4, 4, 1, 1}},      // y_{1-32}(t - 2L3 - L-3 - 2L-2 - 2L2)
    {+1, 2, 4, {4, 1, 2, 5}},               // y_{231}(t - L-2 - L2 - L3 - L-3)
    {-1, 2, 6, {2, 5, 4, 4, 1, 1}},         // y_{231}(t - L3 - L-3 - 2L-2 - 2L2)
    {+1, 1, 7, {4, 4, 1, 2, 2, 5, 5}},      // y_{123}(t - 2L-2 - L2 - 2L3 - 2L-3)
    {-1, 1, 5, {2, 5, 4, 4, 1}},            // y_{123}(t - L3 - L-3 - 2L-2 - L2)
    {+1, 4, 6, {4, 1, 2, 2, 5, 5}},         // y_{3-21}(t - L-2 - L2 - 2L3 - 2L-3)
    {-1, 4, 4, {2, 5, 4, 1}},               // y_{3-21}(t - L3 - L-3 - L-2 - L2)
};

__device__ __forceinline__ int rot_slot(int slot, int c) {
  return (slot % 3 + c) % 3 + (slot >= 3 ? 3 : 0);
}

struct Triad { double k[3], u[3], v[3]; };

__device__ __forceinline__ void triad_of(double beta, double lam, Triad& T) {
  double sb, cb, sl, cl;
  sincos(beta, &sb, &cb);
  sincos(lam, &sl, &cl);
  T.k[0] = -cb * cl; T.k[1] = -cb * sl; T.k[2] = -sb;
  T.u[0] = sl;       T.u[1] = -cl;      T.u[2] = 0.0;
  T.v[0] = -sb * cl; T.v[1] = -sb * sl; T.v[2] = cb;
}

__device__ __forceinline__ double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Spacecraft i position given cos / sin of the orbital phase alpha.
__device__ __forceinline__ void sc_pos(const OrbitDev& o, double ca, double sa, int i, double P[3]) {
  double c2a = ca * ca - sa * sa, s2a = 2.0 * sa * ca;
  double cb = o.cb[i], sb = o.sb[i];
  double c2ab = c2a * cb + s2a * sb;      // cos(2 alpha - beta_i)
  double s2ab = s2a * cb - c2a * sb;      // sin(2 alpha - beta_i)
  double cab = ca * cb + sa * sb;         // cos(alpha - beta_i)
  double eR = o.e * o.R;
  P[0] = o.R * ca + 0.5 * eR * (c2ab - 3.0 * cb);
  P[1] = o.R * sa + 0.5 * eR * (s2ab - 3.0 * sb);
  P[2] = -1.7320508075688772 * eR * cab;
}

// Geometry of one link at a time whose orbital phase has cos/sin (ca, sa) and
// spacecraft positions R: light time (sender at emission), photon direction,
// antenna patterns, k.n and k.R of both ends.
struct LinkGeo { double T, xp, xc, kn, kRs, kRr; };

__device__ void link_geo(const OrbitDev& o, const Triad& tr, double ca, double sa,
                         const double R[3][3], int slot, LinkGeo& g) {
  const int s = c_snd[slot], r = c_rcv[slot];
  double T = o.L_over_c;
  double E[3] = {R[s][0], R[s][1], R[s][2]};
  if (o.kind != 0) {
    for (int it = 0; it < 12; ++it) {
      double w = o.omega * T, w2 = w * w;
      double sw = w * (1.0 - w2 * (1.0 / 6.0));
      double cw = 1.0 - 0.5 * w2 + w2 * w2 * (1.0 / 24.0);
      sc_pos(o, ca * cw + sa * sw, sa * cw - ca * sw, s, E);   // alpha - omega T
      double d0 = R[r][0] - E[0], d1 = R[r][1] - E[1], d2 = R[r][2] - E[2];
      double Tn = sqrt(d0 * d0 + d1 * d1 + d2 * d2) / kC;
      double dT = Tn - T;
      T = Tn;
      if (fabs(dT) <= 4e-15) break;
    }
    double w = o.omega * T, w2 = w * w;
    double sw = w * (1.0 - w2 * (1.0 / 6.0));
    double cw = 1.0 - 0.5 * w2 + w2 * w2 * (1.0 / 24.0);
    sc_pos(o, ca * cw + sa * sw, sa * cw - ca * sw, s, E);
  }
  double n[3];
  double inv = 1.0 / (kC * T);
  n[0] = (R[r][0] - E[0]) * inv;
  n[1] = (R[r][1] - E[1]) * inv;
  n[2] = (R[r][2] - E[2]) * inv;
  double un = dot3(tr.u, n), vn = dot3(tr.v, n);
  g.T = T;
  g.xp = un * un - vn * vn;
  g.xc = 2.0 * un * vn;
  g.kn = dot3(tr.k, n);
  g.kRs = dot3(tr.k, R[s]) / kC;
  g.kRr = dot3(tr.k, R[r]) / kC;
}

__device__ __forceinline__ void orbit_phase(const OrbitDev& o, double t, double& ca, double& sa,
                                            double R[3][3]) {
  double a = o.omega * (o.kind == 0 ? o.t_freeze : t) + o.kappa0;
  sincos(a, &sa, &ca);
  for (int i = 0; i < 3; ++i) sc_pos(o, ca, sa, i, R[i]);
}

// Split of delay d (s) at sample k: read position k - d/dt = i0 + x, x in [0,1).
__device__ __forceinline__ void split(int64_t k, double d, double dt, int64_t& i0, double& x) {
  double q = d / dt;
  double m = ceil(q);
  i0 = k - (int64_t)m;
  x = m - q;
}

// Lagrange weights on nodes j = -N/2+1 .. N/2 via prefix / suffix products.
template <int N>
__device__ __forceinline__ void lag_weights(double x, const double* __restrict__ cj, double w[N]) {
  double pre[N];
  pre[0] = 1.0;
#pragma unroll
  for (int j = 1; j < N; ++j) pre[j] = pre[j - 1] * (x - (double)(j - N / 2));
  double suf = 1.0;
#pragma unroll
  for (int j = N - 1; j >= 0; --j) {
    w[j] = cj[j] * pre[j] * suf;
    suf *= (x - (double)(j + 1 - N / 2));
  }
}

template <int N, typename TC>
__device__ __forceinline__ TC dotw(const double w[N], const TC* __restrict__ b) {
  TC acc = (TC)0;
#pragma unroll
  for (int j = 0; j < N; ++j) acc += (TC)w[j] * b[j];
  return acc;
}

// ---------------------------------------------------------------------------
// LDS layout
// ---------------------------------------------------------------------------
struct TileHdr {
  int64_t w0;        // first sample index of the staged h window
  int64_t g0;        // first index of the g (LFA) or y (full) window
  int32_t nh, ng;    // window lengths
  int32_t bad;       // window does not fit
  int32_t pad;
  int64_t src;       // source index of the tile
};

__host__ __device__ __forceinline__ size_t align_up(size_t v) { return (v + 15) & ~size_t(15); }

// Record a failed window check: err[0] |= code; the first failure also stores
// (code, sample index, offset, window length) in err[2..5].
__device__ __forceinline__ void report(int32_t* err, int code, int64_t k, int64_t b, int64_t len) {
  atomicOr(err, code);
  if (atomicCAS(err + 1, 0, 1) == 0) {
    err[2] = code;
    err[3] = (int32_t)k;
    err[4] = (int32_t)b;
    err[5] = (int32_t)len;
  }
}

// ---------------------------------------------------------------------------
// LFA phase: outputs k0 .. k0+cnt-1.  acc == nullptr: write results; else add
// w+ X^LFA into acc (double[3][tile]) for samples inside the LFA window.
// ---------------------------------------------------------------------------
template <int N, typename TC>
__device__ void lfa_phase(const KParams& P, const RunDesc& RD, const SrcDev& S, const Triad& tr, int64_t k0, int cnt,
                          char* region, TileHdr* hdr, double* acc, double kH) {
  const int tid = threadIdx.x;
  const double dt = S.dt;
  const double Lc = P.orb.L_over_c;
  const int hw = P.st_hw;
  double* hwin_p = reinterpret_cast<double*>(region);
  double* hwin_c = hwin_p + RD.cap_h;
  TC* gwin_p = reinterpret_cast<TC*>(region + align_up(2 * sizeof(double) * (size_t)RD.cap_h));
  TC* gwin_c = gwin_p + RD.cap_g;

  // Window of the derivative series from the delays at both ends of the tile.
  __shared__ double s_qext[2][2];
  if (tid < 2) {
    int64_t k = tid == 0 ? k0 : k0 + cnt - 1;
    double ca, sa, R[3][3];
    orbit_phase(P.orb, S.t0 + (double)k * dt, ca, sa, R);
    LinkGeo g[3];
    for (int a = 0; a < 3; ++a) link_geo(P.orb, tr, ca, sa, R, a, g[a]);
    double qmin = 1e300, qmax = -1e300;
    for (int c = 0; c < 3; ++c) {
      int la = (c + 1) % 3, lb = (c + 2) % 3;
      double Ta = P.equal_arms ? Lc : g[la].T, Tb = P.equal_arms ? Lc : g[lb].T;
      double D = (P.gen == 20) ? 2.0 * (Ta + Tb) : (Ta + Tb);
      double da = D + 0.5 * (g[la].kRs + g[la].kRr), db = D + 0.5 * (g[lb].kRs + g[lb].kRr);
      qmin = fmin(qmin, fmin(da, db) / dt);
      qmax = fmax(qmax, fmax(da, db) / dt);
    }
    s_qext[tid][0] = qmin;
    s_qext[tid][1] = qmax;
  }
  __syncthreads();
  if (tid == 0) {
    double qmin = fmin(s_qext[0][0], s_qext[1][0]), qmax = fmax(s_qext[0][1], s_qext[1][1]);
    int margin = 2 + (int)ceil(4e-4 * (double)cnt);
    int64_t g0 = k0 - (int64_t)ceil(qmax) - N / 2 + 1 - margin;
    int64_t g1 = k0 + cnt - 1 - (int64_t)floor(qmin) + N / 2 + margin;
    int64_t ng = g1 - g0 + 1, nh = ng + 2 * hw;
    hdr->g0 = g0;
    hdr->w0 = g0 - hw;
    hdr->ng = (int32_t)ng;
    hdr->nh = (int32_t)nh;
    hdr->bad = (ng > RD.cap_g || nh > RD.cap_h) ? 1 : 0;
  }
  __syncthreads();
  const int64_t w0 = hdr->w0, g0 = hdr->g0;
  const int nh = hdr->nh, ng = hdr->ng;
  const bool bad = hdr->bad != 0;
  if (!bad) {
    // stage raw h (zero outside the series)
    for (int i = tid; i < nh; i += kBlock) {
      int64_t j = w0 + i;
      bool in = (j >= 0 && j < S.n);
      hwin_p[i] = in ? RD.hp[S.off + j] : 0.0;
      hwin_c[i] = in ? RD.hc[S.off + j] : 0.0;
    }
    __syncthreads();
    // FP64 central stencil, divided by den * dt^m; zero outside the series
    double scale = P.st_den;
    for (int q = 0; q < P.stencil_m; ++q) scale *= dt;
    for (int i = tid; i < ng; i += kBlock) {
      int64_t j = g0 + i;
      double ap = 0.0, ac = 0.0;
      if (j >= 0 && j < S.n) {
        for (int s = 0; s < 2 * hw + 1; ++s) {
          ap += P.st_num[s] * hwin_p[i + s];
          ac += P.st_num[s] * hwin_c[i + s];
        }
        ap /= scale;
        ac /= scale;
      }
      gwin_p[i] = (TC)ap;
      gwin_c[i] = (TC)ac;
    }
  }
  __syncthreads();

  double c2, s2;
  sincos(2.0 * S.psi, &s2, &c2);
  const TC tc2 = (TC)c2, ts2 = (TC)s2;
  for (int i = tid; i < cnt; i += kBlock) {
    const int64_t k = k0 + i;
    double outv[3];
    const double rel = (double)k - kH;
    const bool in_lfa = acc == nullptr || rel <= 0.5 * P.T_s;
    if (!in_lfa) continue;
    if (bad) {
      outv[0] = outv[1] = outv[2] = __builtin_nan("");
    } else {
      double ca, sa, R[3][3];
      orbit_phase(P.orb, S.t0 + (double)k * dt, ca, sa, R);
      LinkGeo g[3];
      for (int a = 0; a < 3; ++a) link_geo(P.orb, tr, ca, sa, R, a, g[a]);
      for (int c = 0; c < 3; ++c) {
        int lab[2] = {(c + 1) % 3, (c + 2) % 3};
        double Ta = P.equal_arms ? Lc : g[lab[0]].T, Tb = P.equal_arms ? Lc : g[lab[1]].T;
        double pref, D;
        if (P.gen == 20) { pref = -4.0 * Ta * Tb * (Ta + Tb); D = 2.0 * (Ta + Tb); }
        else { pref = -2.0 * Ta * Tb; D = Ta + Tb; }
        TC xi[2];
        bool ok = true;
        for (int q = 0; q < 2; ++q) {
          const LinkGeo& L = g[lab[q]];
          int64_t i0; double x;
          split(k, D + 0.5 * (L.kRs + L.kRr), dt, i0, x);
          int64_t b = i0 - N / 2 + 1 - g0;
          if (b < 0 || b + N > ng) { ok = false; report(P.err_flag, 2, k, b, ng); break; }
          TC vp, vc;
          if (x == 0.0) {
            vp = gwin_p[b + N / 2 - 1];
            vc = gwin_c[b + N / 2 - 1];
          } else {
            double w[N];
            lag_weights<N>(x, P.lag_c, w);
            vp = dotw<N, TC>(w, gwin_p + b);
            vc = dotw<N, TC>(w, gwin_c + b);
          }
          TC sp = tc2 * vp - ts2 * vc;     // rotation by the polarisation angle
          TC sc = ts2 * vp + tc2 * vc;
          xi[q] = (TC)L.xp * sp + (TC)L.xc * sc;
        }
        outv[c] = ok ? (double)((TC)pref * (xi[0] - xi[1])) : __builtin_nan("");
      }
    }
    if (acc == nullptr) {
      const int64_t o = S.off + k;
      if constexpr (sizeof(TC) == 8) {
        ((double*)RD.X)[o] = outv[0]; ((double*)RD.Y)[o] = outv[1]; ((double*)RD.Z)[o] = outv[2];
      } else {
        ((float*)RD.X)[o] = (float)outv[0]; ((float*)RD.Y)[o] = (float)outv[1]; ((float*)RD.Z)[o] = (float)outv[2];
      }
    } else {
      const double z = rel / P.sigma_s;
      if constexpr (sizeof(TC) == 8) {
        const double wp = 1.0 / (1.0 + exp(z));
        for (int c = 0; c < 3; ++c) acc[c * P.tile + i] += wp * outv[c];
      } else {
        const float wp = 1.0f / (1.0f + expf((float)z));
        for (int c = 0; c < 3; ++c) acc[c * P.tile + i] += (double)(wp * (float)outv[c]);
      }
    }
  }
  if (bad && tid == 0) report(P.err_flag, 1, k0, ng, nh);
}

// ---------------------------------------------------------------------------
// Full phase: stage 1 (link series on an LDS window) then stage 2 (TDI).
// ---------------------------------------------------------------------------
template <int N, typename TC>
__device__ void full_phase(const KParams& P, const RunDesc& RD, const SrcDev& S, const Triad& tr, int64_t k0, int cnt,
                           char* region, TileHdr* hdr, double* acc, double kH) {
  const int tid = threadIdx.x;
  const double dt = S.dt;
  const int ny6 = RD.cap_y;
  TC* hwin_p = reinterpret_cast<TC*>(region);
  TC* hwin_c = hwin_p + RD.cap_h;
  TC* ywin = reinterpret_cast<TC*>(region + align_up(2 * sizeof(TC) * (size_t)RD.cap_h));
  double* Tcache = reinterpret_cast<double*>(
      region + align_up(2 * sizeof(TC) * (size_t)RD.cap_h) + align_up(6 * sizeof(TC) * (size_t)ny6));

  // y window from the longest stage-2 delay; h window from the stage-1 delays
  // at both ends of the y window.
  __shared__ double s_ext[4];
  __shared__ int64_t s_y[2];
  if (tid < 2) {
    int64_t k = tid == 0 ? k0 : k0 + cnt - 1;
    double ca, sa, R[3][3];
    orbit_phase(P.orb, S.t0 + (double)k * dt, ca, sa, R);
    double Tmax = 0.0;
    for (int a = 0; a < 6; ++a) { LinkGeo g; link_geo(P.orb, tr, ca, sa, R, a, g); Tmax = fmax(Tmax, g.T); }
    s_ext[tid] = Tmax;
  }
  __syncthreads();
  if (tid == 0) {
    double Tmax = fmax(s_ext[0], s_ext[1]);
    int margin = 2 + (int)ceil(4e-4 * (double)cnt);
    double Dmax = (P.gen == 20 ? 7.0 : 3.0) * Tmax;
    s_y[0] = k0 - (int64_t)ceil(Dmax / dt) - N / 2 + 1 - margin;
    s_y[1] = k0 + cnt - 1 + N / 2 + margin;
  }
  __syncthreads();
  if (tid < 2) {
    int64_t i = s_y[tid];
    double ca, sa, R[3][3];
    orbit_phase(P.orb, S.t0 + (double)i * dt, ca, sa, R);
    double dmin = 1e300, dmax = -1e300;
    for (int a = 0; a < 6; ++a) {
      LinkGeo g;
      link_geo(P.orb, tr, ca, sa, R, a, g);
      dmin = fmin(dmin, fmin(g.T + g.kRs, g.kRr));
      dmax = fmax(dmax, fmax(g.T + g.kRs, g.kRr));
    }
    s_ext[2 * tid] = dmin;
    s_ext[2 * tid + 1] = dmax;
  }
  __syncthreads();
  if (tid == 0) {
    double dmin = fmin(s_ext[0], s_ext[2]), dmax = fmax(s_ext[1], s_ext[3]);
    int64_t y0 = s_y[0], y1 = s_y[1];
    int margin = 2 + (int)ceil(4e-4 * (double)(y1 - y0 + 1));
    int64_t w0 = y0 - (int64_t)ceil(dmax / dt) - N / 2 + 1 - margin;
    int64_t w1 = y1 - (int64_t)floor(dmin / dt) + N / 2 + margin;
    hdr->g0 = y0;
    hdr->ng = (int32_t)(y1 - y0 + 1);
    hdr->w0 = w0;
    hdr->nh = (int32_t)(w1 - w0 + 1);
    hdr->bad = (hdr->ng > RD.cap_y || hdr->nh > RD.cap_h) ? 1 : 0;
  }
  __syncthreads();
  const int64_t w0 = hdr->w0, y0 = hdr->g0;
  const int nh = hdr->nh, ny = hdr->ng;
  const bool bad = hdr->bad != 0;

  double c2, s2;
  sincos(2.0 * S.psi, &s2, &c2);
  if (!bad) {
    for (int i = tid; i < nh; i += kBlock) {
      int64_t j = w0 + i;
      bool in = (j >= 0 && j < S.n);
      hwin_p[i] = (TC)(in ? RD.hp[S.off + j] : 0.0);
      hwin_c[i] = (TC)(in ? RD.hc[S.off + j] : 0.0);
    }
    __syncthreads();
    // Stage 1: y_l[i] = [H_l(t_i - ds) - H_l(t_i - dr)] / (2 (1 - k.n)), zero
    // outside the series.
    const TC tc2 = (TC)c2, ts2 = (TC)s2;
    for (int ii = tid; ii < ny; ii += kBlock) {
      const int64_t i = y0 + ii;
      TC yv[6] = {0, 0, 0, 0, 0, 0};
      bool ok = true;
      if (i >= 0 && i < S.n) {
        double ca, sa, R[3][3];
        orbit_phase(P.orb, S.t0 + (double)i * dt, ca, sa, R);
        for (int a = 0; a < 6; ++a) {
          LinkGeo g;
          link_geo(P.orb, tr, ca, sa, R, a, g);
          if (i >= k0 && i < k0 + cnt) Tcache[a * P.tile + (int)(i - k0)] = g.T;
          TC H[2];
          const double dd[2] = {g.T + g.kRs, g.kRr};
          for (int q = 0; q < 2; ++q) {
            int64_t i0; double x;
            split(i, dd[q], dt, i0, x);
            int64_t b = i0 - N / 2 + 1 - w0;
            if (b < 0 || b + N > nh) { ok = false; H[q] = 0; report(P.err_flag, 8, i, b, nh); continue; }
            TC vp, vc;
            if (x == 0.0) {
              vp = hwin_p[b + N / 2 - 1];
              vc = hwin_c[b + N / 2 - 1];
            } else {
              double w[N];
              lag_weights<N>(x, P.lag_c, w);
              vp = dotw<N, TC>(w, hwin_p + b);
              vc = dotw<N, TC>(w, hwin_c + b);
            }
            TC sp = tc2 * vp - ts2 * vc, sc = ts2 * vp + tc2 * vc;
            H[q] = (TC)g.xp * sp + (TC)g.xc * sc;
          }
          yv[a] = (H[0] - H[1]) / (TC)(2.0 * (1.0 - g.kn));
        }
      }
      if (!ok) {
        for (int a = 0; a < 6; ++a) yv[a] = (TC)__builtin_nan("");
      }
      for (int a = 0; a < 6; ++a) ywin[a * ny6 + ii] = yv[a];
    }
    // outputs beyond the series end never enter stage 2; their light times
    // are still needed when a tile extends past n (it does not: cnt <= n - k0)
  }
  __syncthreads();

  // Stage 2: X, Y, Z from the term lists; every delay uses the light times at
  // the output sample, summed in FP64 before the split.
  const int nterms = P.gen == 20 ? 16 : 8;
  for (int i = tid; i < cnt; i += kBlock) {
    const int64_t k = k0 + i;
    const double rel = (double)k - kH;
    if (acc != nullptr && !(rel >= -0.5 * P.T_s)) continue;
    double outv[3];
    if (bad) {
      outv[0] = outv[1] = outv[2] = __builtin_nan("");
    } else {
      double T6[6];
      for (int a = 0; a < 6; ++a) T6[a] = Tcache[a * P.tile + i];
      for (int a = 0; a < 6; ++a)
        if (!(T6[a] > 0.0 && T6[a] < 1e3)) report(P.err_flag, 32, k, (int64_t)(a * 100000 + i), (int64_t)(cnt * 1000 + ny));
      for (int c = 0; c < 3; ++c) {
        TC sum = (TC)0;
        for (int t = 0; t < nterms; ++t) {
          const Term& tm = c_terms[t];
          const int ls = rot_slot(tm.link, c);
          const TC* ys = ywin + ls * ny6;
          TC v;
          if (tm.nd == 0) {
            v = ys[k - y0];
          } else {
            double d = 0.0;
            for (int q = 0; q < tm.nd; ++q) d += T6[rot_slot(tm.d[q], c)];
            int64_t i0; double x;
            split(k, d, dt, i0, x);
            int64_t b = i0 - N / 2 + 1 - y0;
            if (b < 0 || b + N > ny) { v = (TC)__builtin_nan(""); report(P.err_flag, 16, k, b, ny); }
            else if (x == 0.0) v = ys[b + N / 2 - 1];
            else {
              double w[N];
              lag_weights<N>(x, P.lag_c, w);
              v = dotw<N, TC>(w, ys + b);
            }
          }
          sum += tm.sign > 0 ? v : -v;
        }
        outv[c] = (double)sum;
      }
    }
    if (acc == nullptr) {
      const int64_t o = S.off + k;
      if constexpr (sizeof(TC) == 8) {
        ((double*)RD.X)[o] = outv[0]; ((double*)RD.Y)[o] = outv[1]; ((double*)RD.Z)[o] = outv[2];
      } else {
        ((float*)RD.X)[o] = (float)outv[0]; ((float*)RD.Y)[o] = (float)outv[1]; ((float*)RD.Z)[o] = (float)outv[2];
      }
    } else {
      const double z = rel / P.sigma_s;
      if constexpr (sizeof(TC) == 8) {
        const double wm = 1.0 / (1.0 + exp(-z));
        for (int c = 0; c < 3; ++c) acc[c * P.tile + i] += wm * outv[c];
      } else {
        const float wm = 1.0f / (1.0f + expf((float)-z));
        for (int c = 0; c < 3; ++c) acc[c * P.tile + i] += (double)(wm * (float)outv[c]);
      }
    }
  }
  if (bad && tid == 0) report(P.err_flag, 4, k0, ny, nh);
}

// ---------------------------------------------------------------------------
// Tile driver
// ---------------------------------------------------------------------------
template <int N, typename TC>
__device__ void do_tile(const KParams& P, const RunDesc& RD, int64_t tile, char* smem) {
  TileHdr* hdr = reinterpret_cast<TileHdr*>(smem);
  double* acc = reinterpret_cast<double*>(smem + align_up(sizeof(TileHdr)));
  char* region = smem + align_up(sizeof(TileHdr)) + align_up(3 * sizeof(double) * (size_t)P.tile);
  const int tid = threadIdx.x;
  if (tid == 0) {
    // last source whose first tile is <= tile (sources without samples own no tiles)
    int64_t lo = 0, hi = RD.n_src - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) >> 1;
      if (P.src[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
    }
    hdr->src = lo;
  }
  __syncthreads();
  const SrcDev S = P.src[hdr->src];
  const int64_t k0 = (tile - S.tile0) * (int64_t)P.tile;
  const int cnt = (int)min((int64_t)P.tile, S.n - k0);
  Triad tr;
  triad_of(S.beta, S.lam, tr);

  bool needL, needF;
  double kH = 0.0;
  if (P.mode == 0) { needL = false; needF = true; }
  else if (P.mode == 1) { needL = true; needF = false; }
  else {
    kH = (S.t_hyb - S.t0) / S.dt;
    needL = ((double)k0 - kH <= 0.5 * P.T_s);
    needF = ((double)(k0 + cnt - 1) - kH >= -0.5 * P.T_s);
  }
  if (P.mode != 2) {
    if (needL) lfa_phase<N, TC>(P, RD, S, tr, k0, cnt, region, hdr, nullptr, 0.0);
    else full_phase<N, TC>(P, RD, S, tr, k0, cnt, region, hdr, nullptr, 0.0);
  } else {
    for (int i = tid; i < 3 * P.tile; i += kBlock) acc[i] = 0.0;
    __syncthreads();
    if (needL) lfa_phase<N, TC>(P, RD, S, tr, k0, cnt, region, hdr, acc, kH);
    __syncthreads();
    if (needF) full_phase<N, TC>(P, RD, S, tr, k0, cnt, region, hdr, acc, kH);
    __syncthreads();
    for (int i = tid; i < cnt; i += kBlock) {
      const int64_t o = S.off + k0 + i;
      if constexpr (sizeof(TC) == 8) {
        ((double*)RD.X)[o] = acc[i]; ((double*)RD.Y)[o] = acc[P.tile + i]; ((double*)RD.Z)[o] = acc[2 * P.tile + i];
      } else {
        ((float*)RD.X)[o] = (float)acc[i]; ((float*)RD.Y)[o] = (float)acc[P.tile + i];
        ((float*)RD.Z)[o] = (float)acc[2 * P.tile + i];
      }
    }
  }
  __syncthreads();
}

template <int N, typename TC>
__global__ __launch_bounds__(kBlock) void k_response(KParams P) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int64_t s_next;
  const RunDesc RD = *P.rd;
  if (!P.persistent) {
    if ((int64_t)blockIdx.x < RD.n_tiles) do_tile<N, TC>(P, RD, (int64_t)blockIdx.x, smem);
    return;
  }
  for (;;) {
    if (threadIdx.x == 0) s_next = (int64_t)atomicAdd(P.counter, 1u);
    __syncthreads();
    const int64_t t = s_next;
    __syncthreads();
    if (t >= RD.n_tiles) break;
    do_tile<N, TC>(P, RD, t, smem);
  }
}

__global__ void k_reset(uint32_t* counter, int32_t* err, int reset_err) {
  if (threadIdx.x < 8) {
    if (threadIdx.x == 0) *counter = 0u;
    if (reset_err) err[threadIdx.x] = 0;
  }
}

template <int N, typename TC>
int launch_t(const KParams& p, int grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k_response<N, TC>), dim3(grid), dim3(kBlock), lds, st, p);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

size_t lds_bytes_for(int tile, int cap_g, int cap_h, int cap_y, int fp32) {
  size_t tcs = fp32 ? sizeof(float) : sizeof(double);
  size_t lfa = align_up(2 * sizeof(double) * (size_t)cap_h) + align_up(2 * tcs * (size_t)cap_g);
  size_t full = align_up(2 * tcs * (size_t)cap_h) + align_up(6 * tcs * (size_t)cap_y) +
                align_up(6 * sizeof(double) * (size_t)tile);
  size_t region = lfa > full ? lfa : full;
  return align_up(sizeof(TileHdr)) + align_up(3 * sizeof(double) * (size_t)tile) + region;
}

int max_lds_bytes() { return 64 * 1024; }

int launch_reset(uint32_t* counter, int32_t* err_flag, int reset_err, void* stream) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, (hipStream_t)stream, counter, err_flag, reset_err);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_main(const KParams& p, int taps, int fp32, int grid, size_t lds, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (fp32) {
    switch (taps) {
      case 4: return launch_t<4, float>(p, grid, lds, st);
      case 8: return launch_t<8, float>(p, grid, lds, st);
      case 16: return launch_t<16, float>(p, grid, lds, st);
      case 32: return launch_t<32, float>(p, grid, lds, st);
    }
  } else {
    switch (taps) {
      case 4: return launch_t<4, double>(p, grid, lds, st);
      case 8: return launch_t<8, double>(p, grid, lds, st);
      case 16: return launch_t<16, double>(p, grid, lds, st);
      case 32: return launch_t<32, double>(p, grid, lds, st);
    }
  }
  return -2;
}

}  // namespace tdi
