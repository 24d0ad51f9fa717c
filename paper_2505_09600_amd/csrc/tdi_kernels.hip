// Device kernels of the hybrid time-domain LISA response for gfx950.
//
// A batch of sources is cut into tiles of output samples; two persistent
// kernels walk their tile lists with an atomic work counter:
//
//   k_lfa  : low-frequency approximation (Sec. III and App. B).  The strain is
//            staged in LDS, an FP64 central stencil gives its 2nd (TDI 1.5) or
//            3rd (TDI 2.0) derivative, and each output reads that series at six
//            retarded times (two links per Michelson channel), Eqs.
//            (X15_nonequal_timedelays, X20_nonequal_timedelays) with the
//            single-link LFA of Eq. (yslr_strain_derivatives).
//   k_full : full response.  Stage 1 builds the six link series y_l on an LDS
//            window (Eqs. H, yslr, delta_s, delta_r); stage 2 forms X, Y, Z
//            from the TDI term lists with every arm delay evaluated at the
//            output time (Eqs. X1.5, X2.0).
//
// In the hybrid mode the LFA kernel writes w+ X^LFA inside the LFA window and
// the full kernel, which runs after it, adds w- X^Full inside the full window
// (Eqs. sigmoid, hybridized_xs).
//
// Geometry (orbits, light times, antenna patterns, delays) is evaluated
// exactly in FP64 at seven Chebyshev nodes per tile and fitted by a degree-6
// polynomial; over a tile (at most a few hours of orbit) the fit error is far
// below FP64 rounding of the delays.  Retarded-time splits and stencils are
// FP64.  The compute type TC of interpolation and TDI sums is double or float.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tdi_internal.h"

namespace tdi {
namespace {

constexpr double kC = 299792458.0;

__constant__ double c_vinv[kNodes][kNodes];   // monomial coefficients from node values
__constant__ double c_snode[kNodes];          // Chebyshev nodes on [-1, 1]

// Link slots +1,+2,+3,-1,-2,-3: link l joins the two spacecraft other than |l|,
// with sgn(l) = eps_{s|l|r} (Sec. II.B).  Spacecraft are 0-based here.
__host__ __device__ constexpr int snd_of(int a) {
  return a == 0 ? 2 : a == 1 ? 0 : a == 2 ? 1 : a == 3 ? 1 : a == 4 ? 2 : 0;
}
__host__ __device__ constexpr int rcv_of(int a) {
  return a == 0 ? 1 : a == 1 ? 2 : a == 2 ? 0 : a == 3 ? 2 : a == 4 ? 0 : 1;
}

// Fitted quantity index: T_a (a = 0..5), xi+_a, xi_x_a, D_a = 2(1 - k.n_a), k.R_i/c.
__host__ __device__ constexpr int qT(int a) { return a; }
__host__ __device__ constexpr int qXp(int a) { return 6 + a; }
__host__ __device__ constexpr int qXc(int a) { return 12 + a; }
__host__ __device__ constexpr int qD(int a) { return 18 + a; }
__host__ __device__ constexpr int qKR(int i) { return 24 + i; }

// TDI Michelson X terms of Eqs. (X1.5) and (X2.0): sign, link slot of y and
// the multiplicity of each light time (slot order) in the delay.  Y and Z
// follow by cyclic relabelling of the spacecraft.
__constant__ int c_tsign[16] = {+1, -1, +1, -1, +1, -1, +1, -1, +1, -1, +1, -1, +1, -1, +1, -1};
__constant__ int c_tlink[16] = {5, 5, 2, 2, 1, 1, 4, 4, 5, 5, 2, 2, 1, 1, 4, 4};
__constant__ int c_tcoef[16][6] = {
    {0, 1, 1, 0, 1, 0},   // y_{1-32}(t - L-2 - L2 - L3)
    {0, 0, 1, 0, 0, 0},   // y_{1-32}(t - L3)
    {0, 1, 0, 0, 1, 0},   // y_{231}(t - L2 - L-2)
    {0, 0, 0, 0, 0, 0},   // y_{231}(t)
    {0, 0, 0, 0, 1, 0},   // y_{123}(t - L-2)
    {0, 0, 1, 0, 1, 1},   // y_{123}(t - L-2 - L-3 - L3)
    {0, 0, 0, 0, 0, 0},   // y_{3-21}(t)
    {0, 0, 1, 0, 0, 1},   // y_{3-21}(t - L-3 - L3)
    {0, 1, 2, 0, 1, 1},   // y_{1-32}(t - L-2 - L2 - 2L3 - L-3)
    {0, 2, 2, 0, 2, 1},   // y_{1-32}(t - 2L3 - L-3 - 2L-2 - 2L2)
    {0, 1, 1, 0, 1, 1},   // y_{231}(t - L-2 - L2 - L3 - L-3)
    {0, 2, 1, 0, 2, 1},   // y_{231}(t - L3 - L-3 - 2L-2 - 2L2)
    {0, 1, 2, 0, 2, 2},   // y_{123}(t - 2L-2 - L2 - 2L3 - 2L-3)
    {0, 1, 1, 0, 2, 1},   // y_{123}(t - L3 - L-3 - 2L-2 - L2)
    {0, 1, 2, 0, 1, 2},   // y_{3-21}(t - L-2 - L2 - 2L3 - 2L-3)
    {0, 1, 1, 0, 1, 1},   // y_{3-21}(t - L3 - L-3 - L-2 - L2)
};

// The same terms with time-nested delays (optional): a delay operator shifts
// by the light time of its link at the time it is applied, so a product's
// leftmost factor is taken at the output time and each later one at the
// output time less the delays before it.  With the round trips from
// spacecraft 1, A = D+3 D-3 and B = D-2 D+2, and the one-arm signals
// eta2 = y+3 + D+3 y-3 and eta3 = y-2 + D-2 y+2, Eq. (X1.5) is
// B eta2 - eta2 + eta3 - A eta3 and Eq. (X2.0) adds
// B A eta2 - A B B eta2 + B A A eta3 - A B eta3.  Slots in application order
// (A = {2, 5}, B = {4, 1}); the far link of a one-arm signal takes one more leg.
__constant__ int c_nsign[16] = {+1, +1, -1, -1, +1, +1, -1, -1, +1, +1, -1, -1, +1, +1, -1, -1};
__constant__ int c_nlink[16] = {2, 5, 2, 5, 4, 1, 4, 1, 2, 5, 2, 5, 4, 1, 4, 1};
__constant__ int c_nlen[16] = {2, 3, 0, 1, 0, 1, 2, 3, 4, 5, 6, 7, 6, 7, 4, 5};
__constant__ int c_nseq[16][7] = {
    {4, 1},                  // B eta2: y+3
    {4, 1, 2},               //         y-3
    {},                      // -eta2
    {2},
    {},                      // eta3: y-2
    {4},                     //       y+2
    {2, 5},                  // -A eta3
    {2, 5, 4},
    {4, 1, 2, 5},            // B A eta2
    {4, 1, 2, 5, 2},
    {2, 5, 4, 1, 4, 1},      // -A B B eta2
    {2, 5, 4, 1, 4, 1, 2},
    {4, 1, 2, 5, 2, 5},      // B A A eta3
    {4, 1, 2, 5, 2, 5, 4},
    {2, 5, 4, 1},            // -A B eta3
    {2, 5, 4, 1, 4},
};

// slot of link l relabelled c times (1->2->3->1), and its inverse
__host__ __device__ constexpr int rot_slot(int slot, int c) { return (slot % 3 + c) % 3 + (slot >= 3 ? 3 : 0); }
__host__ __device__ constexpr int unrot_slot(int slot, int c) { return (slot % 3 + 3 - c) % 3 + (slot >= 3 ? 3 : 0); }

__host__ __device__ constexpr size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void report(int32_t* err, int code, int64_t k, int64_t b, int64_t len) {
  atomicOr(err, code);
  if (atomicCAS(err + 1, 0, 1) == 0) {
    err[2] = code;
    err[3] = (int32_t)k;
    err[4] = (int32_t)b;
    err[5] = (int32_t)len;
  }
}

// Make LDS writes of the wave visible to all its lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lagrange normalisation 1 / prod_{m != j} (j - m) for nodes j = a - N/2 + 1.
template <int N>
__host__ __device__ constexpr double lag_norm(int a) {
  double p = 1.0;
  for (int b = 0; b < N; ++b)
    if (b != a) p *= (double)(a - b);
  return 1.0 / p;
}

// Lagrange weights on nodes j = -N/2+1 .. N/2 via prefix / suffix products.
template <int N>
__device__ __forceinline__ void lag_weights(double x, double w[N]) {
  double pre[N];
  pre[0] = 1.0;
#pragma unroll
  for (int j = 1; j < N; ++j) pre[j] = pre[j - 1] * (x - (double)(j - N / 2));
  double suf = 1.0;
#pragma unroll
  for (int j = N - 1; j >= 0; --j) {
    w[j] = lag_norm<N>(j) * pre[j] * suf;
    suf *= (x - (double)(j + 1 - N / 2));
  }
}

// Lagrange interpolation of NC interleaved series (element j*NC + c) at offset
// x from the node block starting at b: prefix products forward, suffix products
// and accumulation backward, so only the N prefix values are live.
// Weights and sums in TA (the stored type by default; FP64 for exact reads of
// FP32 series).
template <int N, int NC, typename TC, typename TA = TC>
__device__ __forceinline__ void lag_interp(double x, const TC* __restrict__ b, TA out[NC]) {
  double pre[N];
  pre[0] = 1.0;
#pragma unroll
  for (int j = 1; j < N; ++j) pre[j] = pre[j - 1] * (x - (double)(j - N / 2));
  double suf = 1.0;
  TA acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = (TA)0;
#pragma unroll
  for (int j = N - 1; j >= 0; --j) {
    const TA w = (TA)(lag_norm<N>(j) * pre[j] * suf);
    suf *= (x - (double)(j + 1 - N / 2));
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += w * (TA)b[j * NC + c];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) out[c] = acc[c];
}

__device__ __forceinline__ double sel3(double a0, double a1, double a2, int i) {
  return i == 0 ? a0 : (i == 1 ? a1 : a2);
}

// Split of delay d (s) at sample k: read position k - d/dt = i0 + x, x in [0, 1).
__device__ __forceinline__ void split(int64_t k, double d, double dt, int64_t& i0, double& x) {
  const double q = d / dt;
  const double m = ceil(q);
  i0 = k - (int64_t)m;
  x = m - q;
}

// Central stencil numerators (offsets -hw..hw, zero padded to 7), half widths
// and denominators, indexed by 2 * (m == 3) + (p == 4).
__constant__ double c_stnum[4][7] = {
    {1, -2, 1, 0, 0, 0, 0},           // m = 2, p = 2
    {-1, 16, -30, 16, -1, 0, 0},      // m = 2, p = 4
    {-1, 2, 0, -2, 1, 0, 0},          // m = 3, p = 2
    {1, -8, 13, 0, -13, 8, -1},       // m = 3, p = 4
};
__constant__ int c_sthw[4] = {1, 2, 2, 3};
__constant__ double c_stden[4] = {1.0, 12.0, 2.0, 8.0};

// Stencils of the next LFA term, derivative order m + 2 (4 for TDI 1.5, 5 for
// TDI 2.0), same indexing and layout, zero padded to 9.
__constant__ double c_stnum2[4][9] = {
    {1, -4, 6, -4, 1, 0, 0, 0, 0},                // m + 2 = 4, p = 2
    {-1, 12, -39, 56, -39, 12, -1, 0, 0},         // m + 2 = 4, p = 4
    {-1, 4, -5, 0, 5, -4, 1, 0, 0},               // m + 2 = 5, p = 2
    {1, -9, 26, -29, 0, 29, -26, 9, -1},          // m + 2 = 5, p = 4
};
__constant__ int c_sthw2[4] = {2, 3, 3, 4};
__constant__ double c_stden2[4] = {1.0, 6.0, 2.0, 6.0};

// Central stencil numerators (offsets -hw..hw) and denominators of derivative
// order m (1, 2, 3) and accuracy p (2, 4).
__host__ __device__ __forceinline__ void stencil_coeffs(int m, int p, double c[7], int& hw, double& den) {
  for (int s = 0; s < 7; ++s) c[s] = 0.0;
  if (m == 1 && p == 2) { hw = 1; den = 2.0; c[0] = -1; c[1] = 0; c[2] = 1; }
  else if (m == 1) { hw = 2; den = 12.0; c[0] = 1; c[1] = -8; c[2] = 0; c[3] = 8; c[4] = -1; }
  else if (m == 2 && p == 2) { hw = 1; den = 1.0; c[0] = 1; c[1] = -2; c[2] = 1; }
  else if (m == 2) { hw = 2; den = 12.0; c[0] = -1; c[1] = 16; c[2] = -30; c[3] = 16; c[4] = -1; }
  else if (p == 2) { hw = 2; den = 2.0; c[0] = -1; c[1] = 2; c[2] = 0; c[3] = -2; c[4] = 1; }
  else { hw = 3; den = 8.0; c[0] = 1; c[1] = -8; c[2] = 13; c[3] = 0; c[4] = -13; c[5] = 8; c[6] = -1; }
}

// ---------------------------------------------------------------------------
// Orbit geometry (exact, FP64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sc_pos(const OrbitDev& o, double ca, double sa, int i, double P[3]) {
  const double c2a = ca * ca - sa * sa, s2a = 2.0 * sa * ca;
  const double cb = o.cb[i], sb = o.sb[i];
  const double c2ab = c2a * cb + s2a * sb;   // cos(2 alpha - beta_i)
  const double s2ab = s2a * cb - c2a * sb;   // sin(2 alpha - beta_i)
  const double cab = ca * cb + sa * sb;      // cos(alpha - beta_i)
  const double eR = o.e * o.R;
  P[0] = o.R * ca + 0.5 * eR * (c2ab - 3.0 * cb);
  P[1] = o.R * sa + 0.5 * eR * (s2ab - 3.0 * sb);
  P[2] = -1.7320508075688772 * eR * cab;
}

// Sampled orbit: position of spacecraft i at time t by 8-point Lagrange
// interpolation in time (nodes j0 .. j0 + 7 around t, clamped to the table;
// the host checks that every evaluated time lies inside it).
__device__ void tab_pos(const OrbitDev& o, double t, int i, double P[3]) {
  const double u = (t - o.tab_t0) * o.tab_idt;
  int64_t j0 = (int64_t)floor(u) - 3;
  j0 = j0 < 0 ? 0 : (j0 > o.ntab - 8 ? o.ntab - 8 : j0);
  const double x = u - (double)(j0 + 3);
  // weights of the nodes at offsets m = -3 .. 4 from j0 + 3
  double w[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    double num = 1.0, den = 1.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q == m) continue;
      num *= x - (double)(q - 3);
      den *= (double)(m - q);
    }
    w[m] = num / den;
  }
  P[0] = P[1] = P[2] = 0.0;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const double* r = o.tab + 9 * (j0 + m) + 3 * i;
    P[0] = fma(w[m], r[0], P[0]);
    P[1] = fma(w[m], r[1], P[1]);
    P[2] = fma(w[m], r[2], P[2]);
  }
}

// Geometry of link slot a at time t: T, xi+, xi_x, D = 2(1 - k.n) and k.R/c of
// spacecraft a (meaningful for a < 3).  Light time: receiver at t, sender at
// the emission time t - T (fixed point from L/c); n is the photon direction.
__device__ void node_geometry(const OrbitDev& o, double beta, double lam, double t, int a,
                                          double out[5]) {
  double sb, cb, sl, cl;
  sincos(beta, &sb, &cb);
  sincos(lam, &sl, &cl);
  const double k[3] = {-cb * cl, -cb * sl, -sb};
  const double u[3] = {sl, -cl, 0.0};
  const double v[3] = {-sb * cl, -sb * sl, cb};
  const int s = snd_of(a), r = rcv_of(a);
  double Rr[3], E[3];
  double T = o.L_over_c;
  double sa = 0.0, ca = 1.0;
  if (o.kind == 2) {
    tab_pos(o, t, r, Rr);
    for (int it = 0; it < 12; ++it) {
      tab_pos(o, t - T, s, E);
      const double d0 = Rr[0] - E[0], d1 = Rr[1] - E[1], d2 = Rr[2] - E[2];
      const double Tn = sqrt(d0 * d0 + d1 * d1 + d2 * d2) / kC;
      const double dT = Tn - T;
      T = Tn;
      if (fabs(dT) <= 4e-15) break;
    }
    tab_pos(o, t - T, s, E);
  } else {
    sincos(o.omega * (o.kind == 0 ? o.t_freeze : t) + o.kappa0, &sa, &ca);
    sc_pos(o, ca, sa, r, Rr);
    sc_pos(o, ca, sa, s, E);
  }
  if (o.kind == 1) {
    for (int it = 0; it < 12; ++it) {
      const double w = o.omega * T, w2 = w * w;
      const double sw = w * (1.0 - w2 * (1.0 / 6.0));
      const double cw = 1.0 - 0.5 * w2 + w2 * w2 * (1.0 / 24.0);
      sc_pos(o, ca * cw + sa * sw, sa * cw - ca * sw, s, E);   // phase alpha - omega T
      const double d0 = Rr[0] - E[0], d1 = Rr[1] - E[1], d2 = Rr[2] - E[2];
      const double Tn = sqrt(d0 * d0 + d1 * d1 + d2 * d2) / kC;
      const double dT = Tn - T;
      T = Tn;
      if (fabs(dT) <= 4e-15) break;
    }
    const double w = o.omega * T, w2 = w * w;
    const double sw = w * (1.0 - w2 * (1.0 / 6.0));
    const double cw = 1.0 - 0.5 * w2 + w2 * w2 * (1.0 / 24.0);
    sc_pos(o, ca * cw + sa * sw, sa * cw - ca * sw, s, E);
  }
  const double inv = 1.0 / (kC * T);
  const double n0 = (Rr[0] - E[0]) * inv, n1 = (Rr[1] - E[1]) * inv, n2 = (Rr[2] - E[2]) * inv;
  const double un = u[0] * n0 + u[1] * n1 + u[2] * n2;
  const double vn = v[0] * n0 + v[1] * n1 + v[2] * n2;
  const double kn = k[0] * n0 + k[1] * n1 + k[2] * n2;
  out[0] = T;
  out[1] = un * un - vn * vn;
  out[2] = 2.0 * un * vn;
  out[3] = 2.0 * (1.0 - kn);
  double Ra[3];
  if (o.kind == 2) tab_pos(o, t, a < 3 ? a : 0, Ra);
  else sc_pos(o, ca, sa, a < 3 ? a : 0, Ra);
  out[4] = (k[0] * Ra[0] + k[1] * Ra[1] + k[2] * Ra[2]) / kC;
}

// Per-tile fit of the geometry over samples [ka, kb] of one source.
struct GeoFit {
  double coef[kNQ][kNodes];    // monomial coefficients in s = (k - kc) / kh
  double vals[kNodes][kNQ];    // node values (scratch)
  double kc, ikh;
};

__device__ __forceinline__ double geo_eval(const GeoFit& F, int q, double s) {
  double v = F.coef[q][kNodes - 1];
#pragma unroll
  for (int m = kNodes - 2; m >= 0; --m) v = fma(v, s, F.coef[q][m]);
  return v;
}

// Fit interval [ka, kb] (sample indices) -> centre and half width.
__device__ __forceinline__ void fit_span(double ka, double kb, double& kc, double& kh) {
  kc = 0.5 * (ka + kb);
  kh = fmax(0.5 * (kb - ka), 0.5);
}

// Node values r = j * 6 + a (node j, link slot a) of the fit over [kc - kh, kc + kh].
__device__ __forceinline__ void fit_node(const KParams& P, const SrcDev& S, double kc, double kh, int r,
                                         double vals[kNodes][kNQ]) {
  const int j = r / 6, a = r % 6;
  const double t = S.t0 + (kc + c_snode[j] * kh) * S.dt;
  double g[5];
  node_geometry(P.orb, S.beta, S.lam, t, a, g);
  vals[j][qT(a)] = g[0];
  vals[j][qXp(a)] = g[1];
  vals[j][qXc(a)] = g[2];
  vals[j][qD(a)] = g[3];
  if (a < 3) vals[j][qKR(a)] = g[4];
}

// Monomial coefficient e = q * kNodes + m from the node values.
template <int NQ>
__device__ __forceinline__ double fit_coef(const double vals[kNodes][NQ], int e) {
  const int q = e / kNodes, m = e % kNodes;
  if (m == 0) return vals[kNodes / 2][q];    // the centre node is s = 0
  double c = 0.0;
  for (int j = 0; j < kNodes; ++j) c = fma(c_vinv[m][j], vals[j][q], c);
  return c;
}

// Collective: all threads of the block must call.
__device__ void fit_geometry(const KParams& P, const SrcDev& S, double ka, double kb, GeoFit& F) {
  const int tid = threadIdx.x;
  double kc, kh;
  fit_span(ka, kb, kc, kh);
  if (tid < kNodes * 6) fit_node(P, S, kc, kh, tid, F.vals);
  if (tid == 0) {
    F.kc = kc;
    F.ikh = 1.0 / kh;
  }
  __syncthreads();
  if (tid < kNQ * kNodes) F.coef[tid / kNodes][tid % kNodes] = fit_coef<kNQ>(F.vals, tid);
  __syncthreads();
}

// Source of global tile t: the last source whose first tile is <= t.  Called
// by one whole wave (t uniform, all 64 lanes active): each round tests 64
// evenly spaced candidates at once, so 512 sources take two rounds of
// dependent loads where a binary search takes nine.
__device__ __forceinline__ int64_t find_source_wave(const SrcDev* S, int64_t n_src, int64_t t, bool lfa) {
  const int lane = (int)(threadIdx.x & 63);
  int64_t lo = 0, hi = n_src - 1;
  while (lo < hi) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t c = lo + (int64_t)(lane + 1) * step;
    const bool ok = c <= hi && (lfa ? S[c].lfa_t0 : S[c].full_t0) <= t;
    // first tiles are nondecreasing in the source index: the passing
    // candidates are a prefix of the lanes
    const int64_t nlo = lo + (int64_t)__popcll(__ballot(ok)) * step;
    hi = min(hi, nlo + step - 1);
    lo = nlo;
  }
  return lo;
}

// Next tile of a persistent or one-shot launch (collective).
__device__ __forceinline__ int64_t next_tile(const KParams& P, uint32_t* counter, int64_t n_tiles,
                                             int64_t& iter, int64_t* s_slot) {
  if (!P.persistent) {
    const int64_t t = iter == 0 ? (int64_t)blockIdx.x : n_tiles;
    ++iter;
    return t;
  }
  if (threadIdx.x == 0) *s_slot = (int64_t)atomicAdd(counter, 1u);
  __syncthreads();
  const int64_t t = *s_slot;
  __syncthreads();
  return t;
}

// LFA per-channel structure: channel c uses links a = (c+1)%3 (sign +) and
// b = (c+2)%3 (sign -); link slot l is used by channel (l+2)%3 as side a and by
// channel (l+1)%3 as side b.
__host__ __device__ constexpr int chan_of_use(int l, int side) { return side == 0 ? (l + 2) % 3 : (l + 1) % 3; }

// Delay (s) of use (l, side) and its signed prefactor (Eqs. X15/X20 with
// non-equal time delays): X_c += spref * [ (xi+ c2 + xi_x s2) g+ + (xi_x c2 - xi+ s2) g_x ].
__device__ __forceinline__ void lfa_delay(const KParams& P, const double T3[3], const double mu3[3],
                                          int l, int side, double& d, double& spref) {
  const int c = chan_of_use(l, side);
  const int a = (c + 1) % 3, b = (c + 2) % 3;
  const double Ta = P.equal_arms ? P.orb.L_over_c : T3[a];
  const double Tb = P.equal_arms ? P.orb.L_over_c : T3[b];
  double pref, D;
  if (P.gen == 20) { pref = -4.0 * Ta * Tb * (Ta + Tb); D = 2.0 * (Ta + Tb); }
  else { pref = -2.0 * Ta * Tb; D = Ta + Tb; }
  d = D + mu3[l];
  spref = side == 0 ? pref : -pref;
}

// Delay and coefficients of use (l, side) on the raw (+, x) derivative series.
__device__ __forceinline__ void lfa_use(const KParams& P, const double T3[3], const double xp3[3],
                                        const double xc3[3], const double mu3[3], int l, int side,
                                        double c2, double s2, double& d, double& kp, double& kx) {
  double sg;
  lfa_delay(P, T3, mu3, l, side, d, sg);
  kp = sg * (xp3[l] * c2 + xc3[l] * s2);
  kx = sg * (xc3[l] * c2 - xp3[l] * s2);
}

// Coefficient of the next LFA term of use (l, side) (lfa_terms = 2): the read
// of link l becomes Xi^(m) + kappa Xi^(m+2) with kappa = To^2/6 + Tl^2/8 +
// Tl^2 (1 + (k.n_l)^2)/24, plus (Tl + To)^2/6 for TDI 2.0, To the other arm of
// the use's channel.  This is the central expansion of App. B one order
// further: the m = 1 term of Eq. (yslr_with_tau_derivatives) averaged over
// the two directions of the arm, and the third-order terms of the TDI
// combination of Eqs. (X1.5l2), (X1.5l3) (and of X2.0 = X1.5 - delayed X1.5).
__device__ __forceinline__ double lfa_kappa(const KParams& P, const double T3[3], const double kn3[3],
                                            int l, int side) {
  const int c = chan_of_use(l, side);
  const int o = side == 0 ? (c + 2) % 3 : (c + 1) % 3;   // the channel's other link
  const double Tl = P.equal_arms ? P.orb.L_over_c : T3[l];
  const double To = P.equal_arms ? P.orb.L_over_c : T3[o];
  double kap = To * To / 6.0 + Tl * Tl / 8.0 + Tl * Tl * (1.0 + kn3[l] * kn3[l]) / 24.0;
  if (P.gen == 20) kap += (Tl + To) * (Tl + To) / 6.0;
  return kap;
}

// k.n of the positive links at sample k from the fit (D = 2 (1 - k.n)).
__device__ __forceinline__ void lfa_kn(const GeoFit& F, double s, double kn3[3]) {
#pragma unroll
  for (int l = 0; l < 3; ++l) kn3[l] = 1.0 - 0.5 * geo_eval(F, qD(l), s);
}

// Positive-link geometry at sample k from the fit.
__device__ __forceinline__ void lfa_geo(const GeoFit& F, double s, double T3[3], double xp3[3],
                                        double xc3[3], double mu3[3]) {
  double kR[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) kR[i] = geo_eval(F, qKR(i), s);
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    T3[l] = geo_eval(F, qT(l), s);
    xp3[l] = geo_eval(F, qXp(l), s);
    xc3[l] = geo_eval(F, qXc(l), s);
    mu3[l] = 0.5 * (kR[snd_of(l)] + kR[rcv_of(l)]);
  }
}

// A, E, T from X, Y, Z (end of Sec. II.B): an orthonormal map, applied in the
// output precision just before the store.
template <typename TC>
__device__ __forceinline__ void to_aet(TC& x, TC& y, TC& z) {
  const TC r2 = (TC)0.70710678118654752440, r6 = (TC)0.40824829046386301637,
           r3 = (TC)0.57735026918962576451;
  const TC a = (z - x) * r2;
  const TC e = (x - (TC)2 * y + z) * r6;
  const TC t = (x + y + z) * r3;
  x = a;
  y = e;
  z = t;
}

template <typename TC>
__device__ __forceinline__ void store3(const KParams& P, int64_t o, TC x, TC y, TC z) {
  if (P.aet) to_aet<TC>(x, y, z);
  static_cast<TC*>(P.X)[o] = x;
  static_cast<TC*>(P.Y)[o] = y;
  static_cast<TC*>(P.Z)[o] = z;
}

// ---------------------------------------------------------------------------
// LFA kernel
// ---------------------------------------------------------------------------
struct LfaShared {
  GeoFit F;
  int64_t src, k0, g0;
  int32_t cnt, ng, bad, nh;
  double c2, s2, inv_scale, inv_scale2, kH;
  double qext[2][2];
};

// Per wave, FP32 path: the expansion point of each link and quadratic models
// (in r = k - centre of the wave) of the per-output offset and coefficients.
struct WaveParams {
  int64_t mbar[3];                    // integer part of the link's reference delay (samples)
  float xbar[3];                      // fractional reference offset
  float delta[6], a1[6], a2[6];       // eps_u(r) = delta - r (a1 + a2 r)
  float kp0[6], kp1[6], kp2[6];       // coefficient on g+ : kp0 + r (kp1 + r kp2)
  float kx0[6], kx1[6], kx2[6];
  float kq0[6], kq1[6], kq2[6];       // next term (lfa_terms = 2): coefficient on g+^(m+2)
  float kz0[6], kz1[6], kz2[6];       // and on g_x^(m+2)
  double vals[3][6][5];               // scratch: (point, use, {q, kp, kx, kq, kz})
};

constexpr size_t kWaveParamsBytes = align16(sizeof(WaveParams));

template <int N>
constexpr size_t wave_tables_bytes() {
  return 4 * kWaveParamsBytes + (size_t)4 * 3 * N * 16;
}

// One LFA output with exact FP64 Lagrange weights for each of its six reads
// (the FP64 path, and the FP32 path next to the series ends, where the zero
// extension makes the derivative series jump and an offset expansion fails).
// The derivative window gwin holds NC components per element from g0 on.
template <int N, typename TC, bool NX>
__device__ __forceinline__ void lfa_exact_out(const KParams& P, const LfaShared& sh, const SrcDev& S,
                                              const TC* __restrict__ gwin, int64_t g0, int ng, int64_t k,
                                              double out[3]) {
  constexpr int NC = NX ? 4 : 2;
  const double s = ((double)k - sh.F.kc) * sh.F.ikh;
  double T3[3], xp3[3], xc3[3], mu3[3], kn3[3];
  lfa_geo(sh.F, s, T3, xp3, xc3, mu3);
  if constexpr (NX) lfa_kn(sh.F, s, kn3);
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
#pragma unroll 1
  for (int u = 0; u < 6; ++u) {
    const int l = u >> 1, side = u & 1;
    const int c = side == 0 ? (l + 2) % 3 : (l + 1) % 3;
    const int a = (c + 1) % 3, bb = (c + 2) % 3;
    const double Ta = P.equal_arms ? P.orb.L_over_c : sel3(T3[0], T3[1], T3[2], a);
    const double Tb = P.equal_arms ? P.orb.L_over_c : sel3(T3[0], T3[1], T3[2], bb);
    double pref, D;
    if (P.gen == 20) { pref = -4.0 * Ta * Tb * (Ta + Tb); D = 2.0 * (Ta + Tb); }
    else { pref = -2.0 * Ta * Tb; D = Ta + Tb; }
    int64_t i0;
    double x;
    split(k, D + sel3(mu3[0], mu3[1], mu3[2], l), S.dt, i0, x);
    const int64_t b = i0 - N / 2 + 1 - g0;
    double v[NC];
    if (b < 0 || b + N > ng) {
      report(P.err, 2, k, b, ng);
#pragma unroll
      for (int q = 0; q < NC; ++q) v[q] = __builtin_nan("");
    } else if (x == 0.0) {
#pragma unroll
      for (int q = 0; q < NC; ++q) v[q] = (double)gwin[NC * (b + N / 2 - 1) + q];
    } else {
      lag_interp<N, NC, TC, double>(x, gwin + NC * b, v);
    }
    double gp = (v[0] * sh.c2 - v[1] * sh.s2) * sh.inv_scale;   // rotation to the SSB frame
    double gc = (v[0] * sh.s2 + v[1] * sh.c2) * sh.inv_scale;
    if constexpr (NX) {
      const double kap = lfa_kappa(P, T3, kn3, l, side) * sh.inv_scale2;
      gp = fma(kap, v[NC - 2] * sh.c2 - v[NC - 1] * sh.s2, gp);
      gc = fma(kap, v[NC - 2] * sh.s2 + v[NC - 1] * sh.c2, gc);
    }
    const double xi = sel3(xp3[0], xp3[1], xp3[2], l) * gp + sel3(xc3[0], xc3[1], xc3[2], l) * gc;
    const double term = side == 0 ? pref * xi : -(pref * xi);
    if (c == 0) acc0 += term; else if (c == 1) acc1 += term; else acc2 += term;
  }
  out[0] = acc0;
  out[1] = acc1;
  out[2] = acc2;
}

// NX: with the next term of the LFA (lfa_terms = 2); the derivative window then
// holds four components per element, g+^(m), g_x^(m), g+^(m+2), g_x^(m+2).
template <int N, typename TC, bool NX>
__global__ __launch_bounds__(kBlock, 2) void k_lfa(const KParams* __restrict__ Pp) {
  const KParams& P = *Pp;
  const SrcDev* __restrict__ SS = sources_of(Pp);
  __shared__ LfaShared sh;
  __shared__ int64_t s_next;
  extern __shared__ __align__(16) char dyn[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr bool kF32 = sizeof(TC) == 4;
  constexpr int NC = NX ? 4 : 2;                                 // components per element
  double* hwin = reinterpret_cast<double*>(dyn);                 // [nh][2], FP64
  TC* gwin = reinterpret_cast<TC*>(dyn + P.lfa_goff);           // [ng][NC]
  const int st = 2 * (P.stencil_m == 3 ? 1 : 0) + (P.stencil_p == 4 ? 1 : 0);
  const int hw1 = c_sthw[st];
  const int hw = NX ? c_sthw2[st] : hw1;                         // half width of the h window margin

  int64_t iter = 0;
  for (;;) {
    const int64_t tile = next_tile(P, P.counters + 0, P.n_tiles_lfa, iter, &s_next);
    if (tile >= P.n_tiles_lfa) break;
    if (tid < 64) {
      const int64_t s = find_source_wave(SS, P.n_src, tile, true);
      if (tid == 0) {
        const SrcDev& S = SS[s];
        sh.src = s;
        sh.k0 = S.lfa_kb + (tile - S.lfa_t0) * kTileLfa;
        sh.cnt = (int32_t)min((int64_t)kTileLfa, S.lfa_ke - sh.k0);
        double sn, cs;
        sincos(2.0 * S.psi, &sn, &cs);
        sh.c2 = cs;
        sh.s2 = sn;
        double sc = c_stden[st];
        for (int q = 0; q < P.stencil_m; ++q) sc *= S.dt;
        sh.inv_scale = 1.0 / sc;
        sh.inv_scale2 = 1.0 / (sc * (c_stden2[st] / c_stden[st]) * S.dt * S.dt);
        sh.kH = P.mode == 2 ? (S.t_hyb - S.t0) / S.dt : -INFINITY;
      }
    }
    __syncthreads();
    const SrcDev& S = SS[sh.src];
    const int64_t k0 = sh.k0;
    const int cnt = sh.cnt;
    fit_geometry(P, S, (double)k0, (double)(k0 + cnt - 1), sh.F);

    // window of the derivative series from the six delays at both tile ends
    if (tid < 2) {
      const int64_t k = tid == 0 ? k0 : k0 + cnt - 1;
      const double s = ((double)k - sh.F.kc) * sh.F.ikh;
      double T3[3], xp3[3], xc3[3], mu3[3];
      lfa_geo(sh.F, s, T3, xp3, xc3, mu3);
      double qmin = 1e300, qmax = -1e300;
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          double d, kp, kx;
          lfa_use(P, T3, xp3, xc3, mu3, l, side, 0.0, 0.0, d, kp, kx);
          qmin = fmin(qmin, d / S.dt);
          qmax = fmax(qmax, d / S.dt);
        }
      sh.qext[tid][0] = qmin;
      sh.qext[tid][1] = qmax;
    }
    __syncthreads();
    if (tid == 0) {
      const double qmin = fmin(sh.qext[0][0], sh.qext[1][0]);
      const double qmax = fmax(sh.qext[0][1], sh.qext[1][1]);
      const int margin = 2 + (int)ceil(4e-4 * (double)cnt);
      const int64_t g0 = k0 - (int64_t)ceil(qmax) - N / 2 + 1 - margin;
      const int64_t g1 = k0 + cnt - 1 - (int64_t)floor(qmin) + N / 2 + margin;
      sh.g0 = g0;
      sh.ng = (int32_t)(g1 - g0 + 1);
      sh.nh = sh.ng + 2 * hw;
      sh.bad = (sh.ng > P.cap_g || sh.nh > P.cap_hl) ? 1 : 0;
      if (sh.bad) report(P.err, 1, k0, sh.ng, sh.nh);
    }
    __syncthreads();
    const int64_t g0 = sh.g0;
    const int ng = sh.ng, nh = sh.nh;
    const bool bad = sh.bad != 0;
    const double kH = sh.kH;

    if (!bad) {
      const int64_t h0 = g0 - hw;
      for (int i = tid; i < nh; i += kBlock) {
        const int64_t j = h0 + i;
        const bool in = j >= 0 && j < S.n;
        hwin[2 * i] = in ? P.hp[S.off + j] : 0.0;
        hwin[2 * i + 1] = in ? P.hc[S.off + j] : 0.0;
      }
      __syncthreads();
      // unscaled central stencil sums; 1/(den dt^m) is folded into the coefficients
      for (int i = tid; i < ng; i += kBlock) {
        const int64_t j = g0 + i;
        double ap = 0.0, ac = 0.0, bp = 0.0, bc = 0.0;
        if (j >= 0 && j < S.n) {
          const int c1 = i + hw - hw1;         // first sample of the order-m stencil
#pragma unroll
          for (int s = 0; s < 7; ++s) {
            if (s <= 2 * hw1) {
              ap = fma(c_stnum[st][s], hwin[2 * (c1 + s)], ap);
              ac = fma(c_stnum[st][s], hwin[2 * (c1 + s) + 1], ac);
            }
          }
          if constexpr (NX) {
#pragma unroll
            for (int s = 0; s < 9; ++s) {
              if (s <= 2 * hw) {
                bp = fma(c_stnum2[st][s], hwin[2 * (i + s)], bp);
                bc = fma(c_stnum2[st][s], hwin[2 * (i + s) + 1], bc);
              }
            }
          }
        }
        gwin[NC * i] = (TC)ap;
        gwin[NC * i + 1] = (TC)ac;
        if constexpr (NX) {
          gwin[NC * i + 2] = (TC)bp;
          gwin[NC * i + 3] = (TC)bc;
        }
      }
    }
    __syncthreads();

    if constexpr (kF32) {
      // ------------------------------------------------------------------
      // FP32 bulk: per wave of 256 consecutive outputs (4 per lane, stride
      // 64) and per link, Lagrange weights at the wave's reference offset and
      // a second-order expansion in the per-output offset (|eps| < 0.02).
      // The wave tables reuse the (now free) h window.
      // ------------------------------------------------------------------
      WaveParams* wp = reinterpret_cast<WaveParams*>(dyn + wave * kWaveParamsBytes);
      float4* wts = reinterpret_cast<float4*>(dyn + 4 * kWaveParamsBytes) + wave * 3 * N;
      const int64_t kw0 = k0 + (int64_t)wave * kWaveOut;
      const int wcnt = (int)max((int64_t)0, min((int64_t)kWaveOut, k0 + cnt - kw0));
      // model points: first, middle and last output of the wave (inside the fit)
      const double hr = 0.5 * (double)(wcnt - 1);
      const double kw = (double)kw0 + hr;
      if (!bad && wcnt > 0) {
        if (lane < 3) {
          const double r = (double)(lane - 1) * hr;
          const double s = (kw + r - sh.F.kc) * sh.F.ikh;
          double T3[3], xp3[3], xc3[3], mu3[3], kn3[3];
          lfa_geo(sh.F, s, T3, xp3, xc3, mu3);
          if constexpr (NX) lfa_kn(sh.F, s, kn3);
#pragma unroll
          for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int side = 0; side < 2; ++side) {
              double d, kp, kx;
              lfa_use(P, T3, xp3, xc3, mu3, l, side, sh.c2, sh.s2, d, kp, kx);
              const int u = 2 * l + side;
              wp->vals[lane][u][0] = d / S.dt;
              wp->vals[lane][u][1] = kp * sh.inv_scale;
              wp->vals[lane][u][2] = kx * sh.inv_scale;
              if constexpr (NX) {
                const double kap = lfa_kappa(P, T3, kn3, l, side) * sh.inv_scale2;
                wp->vals[lane][u][3] = kp * kap;
                wp->vals[lane][u][4] = kx * kap;
              }
            }
        }
        wave_sync();
        constexpr int NQ = NX ? 5 : 3;         // modelled quantities per use
        if (lane < 6 * NQ) {
          const int u = lane / NQ, qi = lane % NQ;
          const double v0 = wp->vals[0][u][qi], v1 = wp->vals[1][u][qi], v2 = wp->vals[2][u][qi];
          const double c1 = hr > 0.0 ? (v2 - v0) / (2.0 * hr) : 0.0;
          const double c2q = hr > 0.0 ? (v2 - 2.0 * v1 + v0) / (2.0 * hr * hr) : 0.0;
          if (qi == 0) {
            const int l = u / 2;
            const double qbar = 0.5 * (wp->vals[1][2 * l][0] + wp->vals[1][2 * l + 1][0]);
            const double mb = ceil(qbar);
            wp->delta[u] = (float)(qbar - v1);
            wp->a1[u] = (float)c1;
            wp->a2[u] = (float)c2q;
            if ((u & 1) == 0) {
              wp->mbar[l] = (int64_t)mb;
              wp->xbar[l] = (float)(mb - qbar);
            }
          } else if (qi == 1) {
            wp->kp0[u] = (float)v1;
            wp->kp1[u] = (float)c1;
            wp->kp2[u] = (float)c2q;
          } else if (qi == 2) {
            wp->kx0[u] = (float)v1;
            wp->kx1[u] = (float)c1;
            wp->kx2[u] = (float)c2q;
          } else if (qi == 3) {
            wp->kq0[u] = (float)v1;
            wp->kq1[u] = (float)c1;
            wp->kq2[u] = (float)c2q;
          } else {
            wp->kz0[u] = (float)v1;
            wp->kz1[u] = (float)c1;
            wp->kz2[u] = (float)c2q;
          }
        }
        wave_sync();
        // weights l_j, l'_j, l''_j at xbar of each link; lanes cover (link, tap)
        for (int e = lane; e < 3 * N; e += 64) {
          const int l = e / N, a = e % N;
          const double x = (double)wp->xbar[l];
          double p = lag_norm<N>(a), p1 = 0.0, p2 = 0.0;
          for (int b = 0; b < N; ++b) {
            if (b == a) continue;
            const double f = x - (double)(b - N / 2 + 1);
            p2 = p2 * f + 2.0 * p1;
            p1 = p1 * f + p;
            p = p * f;
          }
          wts[l * N + a] = make_float4((float)p, (float)p1, (float)p2, 0.0f);
        }
        wave_sync();

        float X0[4], X1[4], X2[4];
        bool near_end[4];                      // some read's nodes touch a series end
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          X0[s4] = X1[s4] = X2[s4] = 0.0f;
          near_end[s4] = false;
        }
        const float* gf = reinterpret_cast<const float*>(gwin);
        bool okall = true;
#pragma unroll 1
        for (int l = 0; l < 3; ++l) {
          const int64_t mb = wp->mbar[l];
          int base[4];
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int64_t k = kw0 + lane + 64 * s4;
            const int64_t b = k - mb - N / 2 + 1 - g0;
            const bool live = (lane + 64 * s4) < wcnt;
            const bool inwin = b >= 0 && b + N <= ng;
            if (live && !inwin) { okall = false; report(P.err, 2, k, b, ng); }
            base[s4] = inwin ? (int)b : 0;
            // nodes j0 .. j0 + N - 1 (one more either side for the offset spread)
            // against the elements where the zero-extended stencil output jumps
            const int64_t j0 = k - mb - N / 2 + 1;
            near_end[s4] = near_end[s4] || (j0 - 1 <= hw + 1 && j0 + N >= -hw - 2) ||
                           (j0 - 1 <= S.n + hw + 1 && j0 + N >= S.n - hw - 2);
          }
          float A[4][NC], B[4][NC], Cc[4][NC];
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int q = 0; q < NC; ++q) A[s4][q] = B[s4][q] = Cc[s4][q] = 0.0f;
          const float4* wl = wts + l * N;
#pragma unroll 2
          for (int j = 0; j < N; ++j) {
            const float4 w = wl[j];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
#pragma unroll
              for (int q = 0; q < NC; ++q) {
                const float g = gf[NC * (base[s4] + j) + q];
                A[s4][q] = fmaf(w.x, g, A[s4][q]);
                B[s4][q] = fmaf(w.y, g, B[s4][q]);
                Cc[s4][q] = fmaf(w.z, g, Cc[s4][q]);
              }
            }
          }
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const int u = 2 * l + side;
            const int c = side == 0 ? (l + 2) % 3 : (l + 1) % 3;
            const float dl = wp->delta[u], a1 = wp->a1[u], a2 = wp->a2[u];
            const float p0 = wp->kp0[u], p1 = wp->kp1[u], p2 = wp->kp2[u];
            const float x0 = wp->kx0[u], x1 = wp->kx1[u], x2 = wp->kx2[u];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
              const float r = (float)(lane + 64 * s4) - (float)hr;
              const float eps = dl - r * fmaf(a2, r, a1);
              const float hh = 0.5f * eps;
              float I[NC];
#pragma unroll
              for (int q = 0; q < NC; ++q) I[q] = fmaf(eps, fmaf(hh, Cc[s4][q], B[s4][q]), A[s4][q]);
              const float kp = fmaf(r, fmaf(r, p2, p1), p0);
              const float kx = fmaf(r, fmaf(r, x2, x1), x0);
              float v = fmaf(kp, I[0], kx * I[1]);
              if constexpr (NX) {
                const float kq = fmaf(r, fmaf(r, wp->kq2[u], wp->kq1[u]), wp->kq0[u]);
                const float kz = fmaf(r, fmaf(r, wp->kz2[u], wp->kz1[u]), wp->kz0[u]);
                v = fmaf(kq, I[NC - 2], fmaf(kz, I[NC - 1], v));
              }
              if (c == 0) X0[s4] += v;
              else if (c == 1) X1[s4] += v;
              else X2[s4] += v;
            }
          }
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int i = lane + 64 * s4;
          if (i >= wcnt) continue;
          const int64_t k = kw0 + i;
          float x = X0[s4], y = X1[s4], z = X2[s4];
          if (near_end[s4]) {
            // the expansion in the offset needs smooth data: exact weights here
            double o[3];
            lfa_exact_out<N, TC, NX>(P, sh, S, gwin, g0, ng, k, o);
            x = (float)o[0];
            y = (float)o[1];
            z = (float)o[2];
          }
          if (!okall) x = y = z = __builtin_nanf("");
          if (P.mode == 2) {
            const double rel = (double)k - kH;
            if (rel <= 0.5 * P.T_s) {
              const double zz = rel / P.sigma_s;
              if (zz > -17.0) {       // below, 1/(1+e^z) rounds to 1 in FP32
                const float w = 1.0f / (1.0f + expf((float)zz));
                x *= w; y *= w; z *= w;
              }
            } else {
              x = y = z = 0.0f;
            }
          }
          store3<float>(P, S.off + k, x, y, z);
        }
      }
      if (bad) {
        for (int i = tid; i < cnt; i += kBlock)
          store3<float>(P, S.off + k0 + i, __builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""));
      }
    } else {
      // ------------------------------------------------------------------
      // FP64: exact per-output Lagrange weights for each of the six reads.
      // ------------------------------------------------------------------
      for (int i = tid; i < cnt; i += kBlock) {
        const int64_t k = k0 + i;
        double out[3] = {0.0, 0.0, 0.0};
        if (bad) {
          out[0] = out[1] = out[2] = __builtin_nan("");
        } else {
          lfa_exact_out<N, TC, NX>(P, sh, S, gwin, g0, ng, k, out);
        }
        if (P.mode == 2) {
          const double rel = (double)k - kH;
          if (rel <= 0.5 * P.T_s) {
            const double w = 1.0 / (1.0 + exp(rel / P.sigma_s));
            out[0] *= w;
            out[1] *= w;
            out[2] *= w;
          } else {
            out[0] = out[1] = out[2] = 0.0;
          }
        }
        store3<double>(P, S.off + k, out[0], out[1], out[2]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// LFA kernel, FP32 bulk path for sampling steps up to kFastDtMax
// ---------------------------------------------------------------------------
// Per chunk of kFChunk outputs (a tile holds four chunks and one geometry fit):
//  1. the strain window is staged in LDS in FP64;
//  2. an FP64 central stencil gives the derivative series g+, g_x of every
//     element, and the polarisation rotation and antenna patterns of link l,
//     evaluated at the output time whose retarded time is that element, fold
//     them into one FP32 series F_l per link, written over the strain window;
//  3. each lane reads F_l for nine consecutive outputs.  The Lagrange weights
//     come from a table of their Taylor coefficients (orders 0-3) at a grid
//     point xbar shared by the wave; each lane re-expands them at its own
//     offset and accumulates the value A and the x-derivative B of each output,
//     and each of the two uses of the link then applies its exact offset to
//     first order: I = A + delta B.
// F_l = c(t*) g interpolated at t - tau equals c(t) times the interpolated g up
// to the interpolation error of the smooth product (c varies on the orbital
// time scale), far below FP32 rounding.  Offsets: |eps_lane| <= 0.04 and
// |delta| <= 1e-3 samples for orbital drift below 2e-4 (checked on the host).
constexpr int kFR = 9;                 // outputs per lane (odd: conflict-free LDS stride)
constexpr int kFWave = 64 * kFR;       // outputs per wave
constexpr int kFChunk = 4 * kFWave;    // outputs per chunk (one per workgroup pass)
constexpr uint32_t kAllUses = (1u << (2 * kFR)) - 1u;   // both uses of each of a lane's outputs
constexpr int kSR = 11;                // stencil elements per thread (odd: conflict-free 16-byte stride)
static_assert(kFChunk == kFastChunk && kFR == kFastOutPerLane, "chunk shape");
static_assert(kSR * kBlock == kFastStencilSpan, "stencil sweep");

// Taylor coefficients (l, l', l''/2, l'''/6) of the N Lagrange basis
// polynomials at x = g / kWGrid, g = 0..kWGrid (filled by set_constants).
__constant__ float c_wtab4[kWGrid + 1][4][4];
__constant__ float c_wtab8[kWGrid + 1][8][4];
__constant__ float c_wtab16[kWGrid + 1][16][4];
__constant__ float c_wtab32[kWGrid + 1][32][4];

template <int N>
__device__ __forceinline__ const float4* wtab_row(int g) {
  if constexpr (N == 4) return reinterpret_cast<const float4*>(&c_wtab4[g][0][0]);
  else if constexpr (N == 8) return reinterpret_cast<const float4*>(&c_wtab8[g][0][0]);
  else if constexpr (N == 16) return reinterpret_cast<const float4*>(&c_wtab16[g][0][0]);
  else return reinterpret_cast<const float4*>(&c_wtab32[g][0][0]);
}

struct FastWave {
  int64_t mbar[3];         // integer base of each link's reads (samples)
  int32_t gi[3];           // table row of xbar
  int32_t wcnt;
  float dl[6], a1[6], a2[6];   // x_u(r) - xbar = dl - r (a1 + a2 r), r = k - wave centre
  float c0[6], c1[6];          // signed prefactor / stencil scale: c0 + r c1
  float hr;                    // wave centre relative to its first output
  int8_t cross[4];             // link l < 3: some use's offset from mbar may leave [0, 1); [3] = 0
};

// Parameters of one chunk, written by the pre-pass and copied to LDS by the
// main kernel.
struct FastChunk {
  int64_t g0;                  // first element (sample index) of the window
  int32_t ng, bad;             // window length; bad: it exceeds the staged capacity
  double ec[3];                // centres (element index) of the precombination quadratics
  double pc[3][2][3];          // link, {c+, c_x}, monomial coefficient in (e - ec)
  FastWave W[4];
};

struct FastTile {
  int64_t off, n, k0;          // source offset and length, first output of the tile
  double kH;                   // switch sample (hybrid), -inf otherwise
  int32_t cnt, nch;            // outputs and chunks of the tile
  FastChunk C[4];
};
static_assert(sizeof(FastChunk) % 8 == 0 && sizeof(FastTile) % 8 == 0, "record alignment");
static_assert(sizeof(FastTile) <= kFastTileBytesMax, "tile record bound");
constexpr int kChunkWords = (int)(sizeof(FastChunk) / 4);

// Geometry sample points of a chunk: 0-11 the first, middle and last output
// of each wave, 12-13 the chunk ends, 14-22 three points per link bracketing
// the chunk's element window (precombination models).
constexpr int kFPts = 23;

__device__ __forceinline__ double fast_point(int pt, int64_t kc0, int ccnt, int N, bool& live) {
  live = true;
  if (pt < 12) {
    const int w = pt / 3, p = pt % 3;
    const int wc = min(max(ccnt - w * kFWave, 0), kFWave);
    if (wc <= 0) {
      live = false;
      return 0.0;
    }
    const double hr = 0.5 * (double)(wc - 1);
    return (double)(kc0 + (int64_t)w * kFWave) + hr + (double)(p - 1) * hr;
  }
  if (pt < 14) return pt == 12 ? (double)kc0 : (double)(kc0 + ccnt - 1);
  const int p = (pt - 14) % 3;
  return p == 0 ? (double)(kc0 - N / 2 - 4)
                : (p == 1 ? (double)kc0 + 0.5 * (double)(ccnt - 1) : (double)(kc0 + ccnt - 1 + N / 2 + 4));
}

template <int N>
__host__ __device__ constexpr int kFitPad() { return N / 2 + 8; }

// ---------------------------------------------------------------------------
// Pre-pass of the fast LFA kernel.  Per tile: the degree-6 geometry fit (in
// LDS only) over the tile and the elements read around it, and from it every
// chunk's window, each wave's offset and prefactor models and the per-link
// precombination quadratics, written to P.lfa_tiles.  The fit holds only what
// the fast path reads: T, xi+ and xi_x of the three positive links and k.R/c
// of the three spacecraft (21 node evaluations per tile).  Up to seven tiles
// per pass (P.prep_tiles, fewer for short batches), three workgroups per CU.
// ---------------------------------------------------------------------------
constexpr int kPQ = 12;
constexpr int kPrepNodes = kNodes * 3;
__host__ __device__ constexpr int pT(int l) { return l; }
__host__ __device__ constexpr int pXp(int l) { return 3 + l; }
__host__ __device__ constexpr int pXc(int l) { return 6 + l; }
__host__ __device__ constexpr int pKR(int i) { return 9 + i; }

struct PrepShared {
  double vals[kPrepTiles][kNodes][kPQ];
  double coef[kPrepTiles][kPQ][kNodes];
  double kc[kPrepTiles], ikh[kPrepTiles];
  double c2[kPrepTiles], s2[kPrepTiles], isc[kPrepTiles], idt[kPrepTiles];
  int64_t src[kPrepTiles], k0[kPrepTiles];
  int32_t cnt[kPrepTiles], live[kPrepTiles];
  double wv[kPrepTiles][4][4][3][6][2];   // tile, chunk, wave, point, use, {delay, coefficient}
  double qx[kPrepTiles][4][2][2];         // tile, chunk, end, {min, max delay}
  double pe[kPrepTiles][4][3][3][3];      // tile, chunk, link, point, {element, c+, c_x}
};

__device__ __forceinline__ double prep_eval(const double c[kPQ][kNodes], int q, double s) {
  double v = c[q][kNodes - 1];
#pragma unroll
  for (int m = kNodes - 2; m >= 0; --m) v = fma(v, s, c[q][m]);
  return v;
}

template <int N>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_lfa_prep(const KParams* __restrict__ Pp) {
  const KParams& P = *Pp;
  const SrcDev* __restrict__ SS = sources_of(Pp);
  FastTile* __restrict__ TT = static_cast<FastTile*>(P.lfa_tiles);
  __shared__ PrepShared sh;
  const int tid = threadIdx.x;
  const int st = 2 * (P.stencil_m == 3 ? 1 : 0) + (P.stencil_p == 4 ? 1 : 0);
  const int ntp = min(max(P.prep_tiles, 1), kPrepTiles);   // tiles per pass
  for (int64_t tb = (int64_t)blockIdx.x * ntp; tb < P.n_tiles_lfa; tb += (int64_t)gridDim.x * ntp) {
    // tile headers: one wave per tile
    for (int lt = tid >> 6; lt < ntp; lt += kBlock / 64) {
      const int64_t tile = tb + lt;
      const bool live = tile < P.n_tiles_lfa;
      const int64_t s = live ? find_source_wave(SS, P.n_src, tile, true) : 0;
      if ((tid & 63) == 0) sh.live[lt] = live ? 1 : 0;
      if (live && (tid & 63) == 0) {
        const SrcDev& S = SS[s];
        const int64_t k0 = S.lfa_kb + (tile - S.lfa_t0) * P.tile_fast;
        const int32_t cnt = (int32_t)min((int64_t)P.tile_fast, S.lfa_ke - k0);
        double kc, kh;
        fit_span((double)(k0 - kFitPad<N>()), (double)(k0 + cnt - 1 + kFitPad<N>()), kc, kh);
        sh.kc[lt] = kc;
        sh.ikh[lt] = 1.0 / kh;
        sh.src[lt] = s;
        sh.k0[lt] = k0;
        sh.cnt[lt] = cnt;
        sh.c2[lt] = S.c2psi;
        sh.s2[lt] = S.s2psi;
        double sc = c_stden[st];
        for (int q = 0; q < P.stencil_m; ++q) sc *= S.dt;
        sh.isc[lt] = 1.0 / sc;
        sh.idt[lt] = 1.0 / S.dt;
        FastTile& T = TT[tile];
        T.off = S.off;
        T.n = S.n;
        T.k0 = k0;
        T.kH = P.mode == 2 ? (S.t_hyb - S.t0) / S.dt : -INFINITY;
        T.cnt = cnt;
        T.nch = (cnt + kFChunk - 1) / kFChunk;
      }
    }
    __syncthreads();
    // node values (node j, positive link l) and fit
    for (int e = tid; e < ntp * kPrepNodes; e += kBlock) {
      const int lt = e / kPrepNodes, j = (e % kPrepNodes) / 3, l = e % 3;
      if (!sh.live[lt]) continue;
      const SrcDev& S = SS[sh.src[lt]];
      const double kh = 1.0 / sh.ikh[lt];
      const double t = S.t0 + (sh.kc[lt] + c_snode[j] * kh) * S.dt;
      double g[5];
      node_geometry(P.orb, S.beta, S.lam, t, l, g);
      sh.vals[lt][j][pT(l)] = g[0];
      sh.vals[lt][j][pXp(l)] = g[1];
      sh.vals[lt][j][pXc(l)] = g[2];
      sh.vals[lt][j][pKR(l)] = g[4];
    }
    __syncthreads();
    for (int e = tid; e < ntp * kPQ * kNodes; e += kBlock) {
      const int t = e / (kPQ * kNodes), c = e % (kPQ * kNodes);
      if (sh.live[t]) sh.coef[t][c / kNodes][c % kNodes] = fit_coef<kPQ>(sh.vals[t], c);
    }
    __syncthreads();
    // geometry, delays and prefactors at the sample points of every chunk
    for (int e = tid; e < ntp * 4 * kFPts; e += kBlock) {
      const int t = e / (4 * kFPts), c = (e / kFPts) % 4, pt = e % kFPts;
      if (!sh.live[t]) continue;
      const int ccnt = min(kFChunk, sh.cnt[t] - c * kFChunk);
      if (ccnt <= 0) continue;
      const int64_t kc0 = sh.k0[t] + (int64_t)c * kFChunk;
      bool live;
      const double kq = fast_point(pt, kc0, ccnt, N, live);
      if (!live) continue;
      const double s = (kq - sh.kc[t]) * sh.ikh[t];
      double kR[3], T3[3], mu3[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) kR[i] = prep_eval(sh.coef[t], pKR(i), s);
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        T3[l] = prep_eval(sh.coef[t], pT(l), s);
        mu3[l] = 0.5 * (kR[snd_of(l)] + kR[rcv_of(l)]);
      }
      double qd[6], sp[6];
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          double d, g;
          lfa_delay(P, T3, mu3, l, side, d, g);
          qd[2 * l + side] = d * sh.idt[t];
          sp[2 * l + side] = g * sh.isc[t];
        }
      if (pt < 12) {
        const int w = pt / 3, p = pt % 3;
#pragma unroll
        for (int u = 0; u < 6; ++u) {
          sh.wv[t][c][w][p][u][0] = qd[u];
          sh.wv[t][c][w][p][u][1] = sp[u];
        }
      } else if (pt < 14) {
        double qmin = qd[0], qmax = qd[0];
#pragma unroll
        for (int u = 1; u < 6; ++u) {
          qmin = fmin(qmin, qd[u]);
          qmax = fmax(qmax, qd[u]);
        }
        sh.qx[t][c][pt - 12][0] = qmin;
        sh.qx[t][c][pt - 12][1] = qmax;
      } else {
        const int l = (pt - 14) / 3, p = (pt - 14) % 3;
        const double ql = 0.5 * (sel3(qd[0], qd[2], qd[4], l) + sel3(qd[1], qd[3], qd[5], l));
        const double xp = prep_eval(sh.coef[t], pXp(l), s), xc = prep_eval(sh.coef[t], pXc(l), s);
        sh.pe[t][c][l][p][0] = kq - ql;
        sh.pe[t][c][l][p][1] = xp * sh.c2[t] + xc * sh.s2[t];
        sh.pe[t][c][l][p][2] = xc * sh.c2[t] - xp * sh.s2[t];
      }
    }
    __syncthreads();
    // chunk records: window (kind 0), wave models (1..12), precombination (13..15)
    for (int e = tid; e < ntp * 4 * 16; e += kBlock) {
      const int t = e / 64, c = (e / 16) % 4, kind = e % 16;
      if (!sh.live[t]) continue;
      const int ccnt = min(kFChunk, sh.cnt[t] - c * kFChunk);
      if (ccnt <= 0) continue;
      const int64_t kc0 = sh.k0[t] + (int64_t)c * kFChunk;
      FastChunk& R = TT[tb + t].C[c];
      if (kind == 0) {
        const double qmin = fmin(sh.qx[t][c][0][0], sh.qx[t][c][1][0]);
        const double qmax = fmax(sh.qx[t][c][0][1], sh.qx[t][c][1][1]);
        const int margin = 2 + (int)ceil(4e-4 * (double)ccnt);
        const int64_t g0 = kc0 - (int64_t)ceil(qmax) - N / 2 + 1 - margin;
        const int64_t g1 = kc0 + ccnt - 1 - (int64_t)floor(qmin) + N / 2 + margin;
        const int64_t ng = g1 - g0 + 1;
        R.g0 = g0;
        R.ng = (int32_t)min(ng, (int64_t)INT32_MAX);
        R.bad = ng > P.cap_g ? 1 : 0;
        if (R.bad) report(P.err, 1, kc0, ng, P.cap_g);
      } else if (kind <= 12) {
        const int w = (kind - 1) / 3, l = (kind - 1) % 3;
        const int wc = min(max(ccnt - w * kFWave, 0), kFWave);
        FastWave& Wv = R.W[w];
        if (l == 0) {
          Wv.wcnt = wc;
          Wv.hr = 0.5f * (float)(wc - 1);
          Wv.cross[3] = 0;
        }
        if (wc > 0) {
          const double hr = 0.5 * (double)(wc - 1);
          const double qbar = 0.5 * (sh.wv[t][c][w][1][2 * l][0] + sh.wv[t][c][w][1][2 * l + 1][0]);
          const double mb = ceil(qbar);
          const int gi = min(max((int)rint((mb - qbar) * (double)kWGrid), 0), kWGrid);
          const double xbar = (double)gi / (double)kWGrid;
          Wv.mbar[l] = (int64_t)mb;
          Wv.gi[l] = gi;
          // differences in FP64, scaling in FP32 (the models are stored in FP32)
          const float ih = hr > 0.0 ? 0.5f / (float)hr : 0.0f;
          // the split puts each use's integer base at ceil(q), offset mb - q in
          // [0, 1) when the base is mb; at the wave's first and last outputs the
          // offsets are mb - v0 and mb - v2 (the models are quadratic in r with
          // negligible curvature), so a link whose offsets come within 1e-3 of 0
          // or 1 is flagged for the main kernel's per-use base check
          bool cross = false;
          for (int side = 0; side < 2; ++side) {
            const int u = 2 * l + side;
            const double v0 = sh.wv[t][c][w][0][u][0], v2 = sh.wv[t][c][w][2][u][0];
            const double xa = mb - v0, xb = mb - v2;
            cross = cross || fmin(xa, xb) < 1e-3 || fmax(xa, xb) >= 1.0 - 1e-3;
          }
          Wv.cross[l] = cross ? 1 : 0;
          for (int side = 0; side < 2; ++side) {
            const int u = 2 * l + side;
            const double v0 = sh.wv[t][c][w][0][u][0], v1 = sh.wv[t][c][w][1][u][0], v2 = sh.wv[t][c][w][2][u][0];
            const double e0 = sh.wv[t][c][w][0][u][1], e1 = sh.wv[t][c][w][1][u][1], e2 = sh.wv[t][c][w][2][u][1];
            Wv.dl[u] = (float)((mb - v1) - xbar);
            Wv.a1[u] = (float)(v2 - v0) * ih;
            Wv.a2[u] = (float)(v2 - 2.0 * v1 + v0) * (2.0f * ih * ih);
            Wv.c0[u] = (float)e1;
            Wv.c1[u] = (float)(e2 - e0) * ih;
          }
        }
      } else {
        const int l = kind - 13;
        const double x0 = sh.pe[t][c][l][0][0], x1 = sh.pe[t][c][l][1][0], x2 = sh.pe[t][c][l][2][0];
        R.ec[l] = x1;
        for (int q = 0; q < 2; ++q) {
          const double f0 = sh.pe[t][c][l][0][q + 1], f1 = sh.pe[t][c][l][1][q + 1], f2 = sh.pe[t][c][l][2][q + 1];
          // quadratic through the three samples, in u = e - x1
          const double d01 = (x1 > x0) ? (f1 - f0) / (x1 - x0) : 0.0;
          const double d12 = (x2 > x1) ? (f2 - f1) / (x2 - x1) : 0.0;
          const double d012 = (x2 > x0) ? (d12 - d01) / (x2 - x0) : 0.0;
          R.pc[l][q][0] = f1;
          R.pc[l][q][1] = d01 + (x1 - x0) * d012;
          R.pc[l][q][2] = d012;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Main kernel of the fast LFA path: per chunk, the record written by the
// pre-pass and the strain window are staged, then stencil + precombination
// and the interpolation described above.
// ---------------------------------------------------------------------------
constexpr int kEdgeMax = 64;   // >= N + kFR + 2 hw + 8 for every supported N

// Exact read near an end of the series: the oracle's split, Lagrange weights
// w_j = norm_j P(x) / (x - x_j) with P(x) = prod_i (x - x_i) (x = 0 reads the
// node), on the raw pairs, and the polarisation coefficients at the output
// time.  j0 is the absolute element of tap 0, ne the number of stored pairs;
// ge[0] holds the pairs of elements 0..ne-1, ge[1] those of n-ne..n-1.
__device__ __forceinline__ bool edge_pair(const float2 (*ge)[kEdgeMax], int64_t j, int64_t n, int ne, float2& g) {
  if (j < 0 || j >= n) { g = make_float2(0.0f, 0.0f); return true; }
  if (j < ne) { g = ge[0][j]; return true; }
  if (j >= n - ne) { g = ge[1][j - (n - ne)]; return true; }
  return false;
}

template <int N>
__device__ __forceinline__ bool edge_read(const float2 (*ge)[kEdgeMax], int64_t j0, int64_t n, int ne, double x,
                                          double& sp, double& sx) {
  sp = sx = 0.0;
  float2 g;
  if (x == 0.0) {
    if (!edge_pair(ge, j0 + N / 2 - 1, n, ne, g)) return false;
    sp = g.x;
    sx = g.y;
    return true;
  }
  double Pn = 1.0;
#pragma unroll 1
  for (int i = 0; i < N; ++i) Pn *= x - (double)(i - N / 2 + 1);
  // unit-spaced nodes: norm_j = (-1)^(N-1-j) / (j! (N-1-j)!), so
  // norm_{j+1} = -norm_j (N-1-j) / (j+1), starting from norm_0 = lag_norm<N>(0)
  double nj = lag_norm<N>(0);
  bool ok = true;
#pragma unroll 1
  for (int j = 0; j < N; ++j) {
    ok = edge_pair(ge, j0 + j, n, ne, g) && ok;
    const double w = nj * Pn / (x - (double)(j - N / 2 + 1));
    sp = fma(w, (double)g.x, sp);
    sx = fma(w, (double)g.y, sx);
    nj = -nj * (double)(N - 1 - j) / (double)(j + 1);
  }
  return ok;
}

template <int N>
__global__ __launch_bounds__(kBlock, 3) void k_lfa_fast(const KParams* __restrict__ Pp) {
  const KParams& P = *Pp;
  const FastTile* __restrict__ TT = static_cast<const FastTile*>(P.lfa_tiles);
  __shared__ FastChunk ch;                      // the current chunk's record
  __shared__ float2 gedge[2][kEdgeMax];         // raw (g+, g_x) next to the series ends
  __shared__ int64_t s_next;
  extern __shared__ __align__(16) char dyn[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  float* Fw = reinterpret_cast<float*>(dyn);                        // [3][ngp], FP32
  const int st = 2 * (P.stencil_m == 3 ? 1 : 0) + (P.stencil_p == 4 ? 1 : 0);
  const int hw = c_sthw[st];
  // all seven stencil weights, zero beyond 2 hw (a pair-summed form saves
  // FP64 FMAs but costs registers, and measured slower)
  double stn[7];
#pragma unroll
  for (int s = 0; s < 7; ++s) stn[s] = c_stnum[st][s];
  const int ne = N + kFR + 2 * hw + 8;          // raw pairs kept at each end

  int64_t iter = 0;
  for (;;) {
    const int64_t tile = next_tile(P, P.counters + 0, P.n_tiles_lfa, iter, &s_next);
    if (tile >= P.n_tiles_lfa) break;
    const FastTile& T = TT[tile];
    const int64_t off = T.off, n = T.n, k0 = T.k0;
    const double kH = T.kH;
    const int cnt = T.cnt, nch = T.nch;

    for (int c = 0; c < nch; ++c) {
      const int64_t kc0 = k0 + (int64_t)c * kFChunk;
      const int ccnt = min(kFChunk, cnt - c * kFChunk);
      const FastChunk& R = T.C[c];
      const int64_t g0 = R.g0;
      const int ng = R.ng, ngp = ng + kFR + 1;
      const bool bad = R.bad != 0;
      // the chunk record goes to LDS (read after the barrier below)
      if (tid < kChunkWords) reinterpret_cast<int32_t*>(&ch)[tid] = reinterpret_cast<const int32_t*>(&R)[tid];

      if (!bad) {
        // ---- stencil and precombination, kSR consecutive elements per thread,
        // the strain read straight from global memory (neighbouring threads
        // overlap by 2 hw samples; the cache absorbs the re-reads)
        // the coefficients vary on the orbital time scale: FP32 models suffice
        // (F_l is stored in FP32); the stencil sums stay FP64
        float pcv[3][2][3], ecv[3];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          ecv[l] = (float)(R.ec[l] - (double)g0);   // relative to the window start
#pragma unroll
          for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int m = 0; m < 3; ++m) pcv[l][q][m] = (float)R.pc[l][q][m];
        }
        constexpr int kSM = kSR / 2;                 // middle element of a thread's run
        for (int base = 0; base < ng; base += kSR * kBlock) {
          const int i0 = base + kSR * tid;
          if (i0 < ng) {
            // this thread's elements e (absolute j0 + e) inside the series: [elo, ehi);
            // raw pairs kept for e < es0 (first ne elements) and e >= es1 (last ne)
            const int64_t j0 = g0 + i0;
            const int elo = (int)min(max(-j0, (int64_t)0), (int64_t)kSR);
            const int ehi = (int)min(max(n - j0, (int64_t)0), (int64_t)kSR);
            const int es0 = (int)min(max((int64_t)ne - j0, (int64_t)0), (int64_t)kSR);
            const int es1 = (int)min(max(n - ne - j0, (int64_t)0), (int64_t)kSR);
            const bool near_end = es0 > 0 || es1 < kSR;
            // the coefficients over the thread's kSR elements: tangent lines of the
            // chunk's quadratics at the middle element (the curvature term over
            // +-5 samples is ~1e-10 of the coefficient)
            float cpm[3], cpd[3], cxm[3], cxd[3];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
              const float u = (float)(i0 + kSM) - ecv[l];
              cpm[l] = fmaf(u, fmaf(u, pcv[l][0][2], pcv[l][0][1]), pcv[l][0][0]);
              cpd[l] = fmaf(2.0f * u, pcv[l][0][2], pcv[l][0][1]);
              cxm[l] = fmaf(u, fmaf(u, pcv[l][1][2], pcv[l][1][1]), pcv[l][1][0]);
              cxd[l] = fmaf(2.0f * u, pcv[l][1][2], pcv[l][1][1]);
            }
            // samples j0 - 3 + m, m < kSR + 6, inside the series for m in [mlo, mhi)
            const int mlo = (int)min(max((int64_t)hw - j0, (int64_t)0), (int64_t)(kSR + 6));
            const int mhi = (int)min(max(n - j0 + hw, (int64_t)0), (int64_t)(kSR + 6));
            const double* __restrict__ hpb = P.hp + off + (j0 - hw);
            const double* __restrict__ hcb = P.hc + off + (j0 - hw);
            double hp_[kSR + 6], hc_[kSR + 6];
            // the strain loads go out ahead of the other waves' arithmetic
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int m = 0; m < kSR + 6; ++m) {
              const bool in = m >= mlo && m < mhi;
              hp_[m] = in ? hpb[m] : 0.0;
              hc_[m] = in ? hcb[m] : 0.0;
            }
            __builtin_amdgcn_s_setprio(0);
#pragma unroll
            for (int e = 0; e < kSR; ++e) {
              double ap = 0.0, ac = 0.0;
#pragma unroll
              for (int s = 0; s < 7; ++s) {
                ap = fma(stn[s], hp_[e + s], ap);
                ac = fma(stn[s], hc_[e + s], ac);
              }
              const bool in = e >= elo && e < ehi;
              if (!in) ap = ac = 0.0;
              const float gp = (float)ap, gx = (float)ac;
              if (near_end && in) {
                if (e < es0) gedge[0][(int)(j0 + e)] = make_float2(gp, gx);
                if (e >= es1) gedge[1][(int)(j0 + e - (n - ne))] = make_float2(gp, gx);
              }
#pragma unroll
              for (int l = 0; l < 3; ++l) {
                const float cp = fmaf((float)(e - kSM), cpd[l], cpm[l]);
                const float cx = fmaf((float)(e - kSM), cxd[l], cxm[l]);
                if (i0 + e < ng) Fw[l * ngp + i0 + e] = fmaf(cp, gp, cx * gx);
              }
            }
          }
        }
      }
      __syncthreads();

      if (!bad) {

        // ---- E: interpolation, TDI combination, hybrid weight -------------
        const FastWave& Wv = ch.W[wave];
        const int wcnt = Wv.wcnt;
        const int64_t kw0 = kc0 + (int64_t)wave * kFWave;
        if (wcnt > 0) {
          const int nl = min(max(wcnt - kFR * lane, 0), kFR);
          const float rL = (float)(kFR * lane + kFR / 2) - Wv.hr;
          float Xa[kFR], Xb[kFR], Xc[kFR];
#pragma unroll
          for (int q = 0; q < kFR; ++q) Xa[q] = Xb[q] = Xc[q] = 0.0f;
          bool ok = true;
          int l = 0, pass = 0;
#pragma unroll 1
          for (;;) {
            // Near the ends of the series the zero extension makes F_l jump: the
            // expansion in the offset does not hold for such broadband data, so a
            // lane whose reads touch an end takes no use here; the exact split and
            // weights give its uses after the link loop.
            const int64_t e_lo = kw0 + kFR * lane - Wv.mbar[l] - N / 2 + 1;
            const int64_t e_hi = e_lo + kFR + N - 2;
            const bool edge = nl > 0 && ((e_lo <= hw + 1 && e_hi >= -hw - 2) ||
                                         (e_lo <= n + hw + 1 && e_hi >= n - hw - 2));
            // The split puts each use's integer base at ceil(q), i.e. its offset x
            // from the base in [0, 1); the wave shares the base mbar (x = xbar + e).
            // When a delay crosses an integer inside the wave (the pre-pass flags
            // the link) the uses with x outside [0, 1) belong to the neighbouring
            // base, whose node set is shifted by one sample.  A second pass takes
            // them with that base's window and the table row at the integer end
            // (x = 1 for base mbar + 1, x = 0 for mbar - 1); the first pass takes
            // the rest.  For data the taps resolve the two interpolants agree;
            // near a merger they do not.  Edge lanes take neither pass.
            const int gi = __builtin_amdgcn_readfirstlane(Wv.gi[l]);
            const int npass = __builtin_amdgcn_readfirstlane((int)Wv.cross[l]) != 0 ? 2 : 1;
            // x near 0 (gi <= kWGrid / 2): the neighbouring base is mbar + 1, else mbar - 1
            const int s_alt = 2 * gi <= kWGrid ? 1 : -1;
            uint32_t own = edge ? 0u : kAllUses;   // bit side * kFR + q: the use is on base mbar
            if (npass == 2 && !edge) {
              const float xbar = (float)gi * (1.0f / (float)kWGrid);
              own = 0u;
#pragma unroll
              for (int side = 0; side < 2; ++side) {
                const int u = 2 * l + side;
#pragma unroll
                for (int q = 0; q < kFR; ++q) {
                  const float r = rL + (float)(q - kFR / 2);
                  const float x = xbar + (Wv.dl[u] - r * fmaf(Wv.a2[u], r, Wv.a1[u]));
                  if (s_alt > 0 ? x >= 0.0f : x < 1.0f) own |= 1u << (side * kFR + q);
                }
              }
            }
            static_assert(2 * kFR <= 32, "use mask");
            const int grow = pass ? (s_alt > 0 ? kWGrid : 0) : gi;
            const float eoff =
                pass ? (float)(gi - grow) * (1.0f / (float)kWGrid) + (float)s_alt : 0.0f;
            const uint32_t take = edge ? 0u : (pass ? ~own : own);
            const int64_t b64 = kw0 + kFR * lane - Wv.mbar[l] - N / 2 + 1 - g0 - (pass ? s_alt : 0);
            const uint32_t live = nl > 0 ? take & (((1u << nl) - 1u) * ((1u << kFR) + 1u)) : 0u;
            if (live != 0u && (b64 < 0 || b64 + nl + N - 2 >= ng)) {
              ok = false;
              report(P.err, 2, kw0 + kFR * lane, b64, ng);
            }
            const int b = (int)min(max(b64, (int64_t)0), (int64_t)(ngp - (kFR + N - 1)));
            const float* Fl = Fw + l * ngp + b;
            float win[kFR + N - 1];
#pragma unroll
            for (int t = 0; t < kFR + N - 1; ++t) win[t] = Fl[t];
            const int u0 = 2 * l, u1 = 2 * l + 1;
            const float e0 = Wv.dl[u0] - rL * fmaf(Wv.a2[u0], rL, Wv.a1[u0]);
            const float e1 = Wv.dl[u1] - rL * fmaf(Wv.a2[u1], rL, Wv.a1[u1]);
            const float eLm = 0.5f * (e0 + e1);
            const float eL = eLm + eoff;
            // the pass's table row, read by scalar loads (SGPR operands)
            const float4* row = wtab_row<N>(grow);
            float A[kFR], B[kFR];
#pragma unroll
            for (int q = 0; q < kFR; ++q) A[q] = B[q] = 0.0f;
#pragma unroll
            for (int j = 0; j < N; ++j) {
              const float4 c = row[j];
              // w = p(e) = c.x + c.y e + c.z e^2 + c.w e^3 by Horner; its slope
              // p'(e) = c.y + 2 c.z e + 3 c.w e^2 is taken as b1 + e b2 = c.y + 2 c.z e
              // + 2 c.w e^2: it only multiplies the per-use offset delta (<= 1e-3),
              // so the dropped c.w e^2 delta is of fifth order in the offsets.  The
              // slope must be that of the same N-node interpolant: a shorter stencil
              // differs from it by O(1) of the local jump where the data have a kink
              // (a merger cut), and parity with the oracle's exact read is lost there.
              const float b2 = fmaf(eL, c.w, c.z);
              const float b1 = fmaf(eL, b2, c.y);
              const float w = fmaf(eL, b1, c.x);
              const float wd = fmaf(eL, b2, b1);
#pragma unroll
              for (int q = 0; q < kFR; ++q) {
                A[q] = fmaf(w, win[j + q], A[q]);
                B[q] = fmaf(wd, win[j + q], B[q]);
              }
            }
            // per use: I = A + delta B, delta linear in the output index over
            // the lane's kFR outputs (the offset's curvature over 2 kFR samples
            // is below 1e-8 samples)
            float Iv[2][kFR];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
              const int u = 2 * l + side;
              const float a1 = Wv.a1[u], a2 = Wv.a2[u];
              const float d0 = (side == 0 ? e0 : e1) - eLm;
              const float sl = fmaf(2.0f * a2, rL, a1);
#pragma unroll
              for (int q = 0; q < kFR; ++q)
                Iv[side][q] = fmaf(fmaf((float)(kFR / 2 - q), sl, d0), B[q], A[q]);
            }
            // side 0 feeds channel (l+2)%3 (Xa), side 1 channel (l+1)%3 (Xb); most
            // waves take every use (no crossing, no edge) and skip the mask tests
            if (__ballot(take != kAllUses) == 0) {
#pragma unroll
              for (int side = 0; side < 2; ++side) {
                const int u = 2 * l + side;
                const float c1 = Wv.c1[u], cL = fmaf(rL, c1, Wv.c0[u]);
#pragma unroll
                for (int q = 0; q < kFR; ++q) {
                  const float cf = fmaf((float)(q - kFR / 2), c1, cL);
                  if (side == 0) Xa[q] = fmaf(cf, Iv[0][q], Xa[q]);
                  else Xb[q] = fmaf(cf, Iv[1][q], Xb[q]);
                }
              }
            } else {
#pragma unroll
              for (int side = 0; side < 2; ++side) {
                const int u = 2 * l + side;
                const float c1 = Wv.c1[u], cL = fmaf(rL, c1, Wv.c0[u]);
#pragma unroll
                for (int q = 0; q < kFR; ++q) {
                  const float cf = fmaf((float)(q - kFR / 2), c1, cL);
                  if ((take >> (side * kFR + q)) & 1u) {
                    if (side == 0) Xa[q] = fmaf(cf, Iv[0][q], Xa[q]);
                    else Xb[q] = fmaf(cf, Iv[1][q], Xb[q]);
                  }
                }
              }
            }
            if (++pass < npass) continue;
            pass = 0;
            // the next link's (side 0, side 1) channels are this link's (Xc, Xa)
#pragma unroll
            for (int q = 0; q < kFR; ++q) {
              const float t = Xc[q];
              Xc[q] = Xb[q];
              Xb[q] = Xa[q];
              Xa[q] = t;
            }
            if (++l == 3) break;
          }
          // Edge lanes: raw pairs with the coefficients at the output time (the
          // precombined F_l is exact only for band-limited data).  A link's edge
          // lanes hold 2 kFR uses each; they are spread over the 64 lanes of the
          // wave, 64 at a time, and each c * value goes back to its lane by a
          // shuffle.  After the link loop X = Xc, Y = Xb, Z = Xa, and side 0 of
          // link l feeds channel (l + 2) % 3, side 1 channel (l + 1) % 3.
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            const int64_t e_lo = kw0 + kFR * lane - Wv.mbar[l] - N / 2 + 1;
            const int64_t e_hi = e_lo + kFR + N - 2;
            const bool edge = nl > 0 && ((e_lo <= hw + 1 && e_hi >= -hw - 2) ||
                                         (e_lo <= n + hw + 1 && e_hi >= n - hw - 2));
            const uint64_t emask = __ballot(edge);
            if (emask == 0) continue;
            const double mq = (double)Wv.mbar[l] - (double)Wv.gi[l] / (double)kWGrid;
            const int total = __popcll(emask) * (2 * kFR);
            const int my_rank = edge ? __popcll(emask & ((1ull << lane) - 1ull)) : -1;
#pragma unroll 1
            for (int rb = 0; rb < total; rb += 64) {
              const int id = rb + lane;
              float v = 0.0f;
              int good = 1;
              if (id < total) {
                const int rank = id / (2 * kFR), side = (id / kFR) % 2, q = id % kFR;
                uint64_t mm = emask;
                for (int i = 0; i < rank; ++i) mm &= mm - 1ull;
                const int ol = __ffsll((unsigned long long)mm) - 1;      // the use's lane
                if (q < min(max(wcnt - kFR * ol, 0), kFR)) {
                  const int u = 2 * l + side;
                  const float r = ((float)(kFR * ol + kFR / 2) - Wv.hr) + (float)(q - kFR / 2);
                  const int64_t k = kw0 + kFR * ol + q;
                  const double qf = mq - (double)(Wv.dl[u] - r * fmaf(Wv.a2[u], r, Wv.a1[u]));   // delay in samples
                  const double mc = ceil(qf);
                  const int64_t j0 = k - (int64_t)mc - N / 2 + 1;
                  double sp, sx;
                  if (!edge_read<N>(gedge, j0, n, ne, mc - qf, sp, sx)) {
                    good = 0;
                    report(P.err, 2, k, j0, n);
                  } else {
                    const double uu = ((double)k - qf) - ch.ec[l];
                    const double cp = fma(uu, fma(uu, ch.pc[l][0][2], ch.pc[l][0][1]), ch.pc[l][0][0]);
                    const double cx = fma(uu, fma(uu, ch.pc[l][1][2], ch.pc[l][1][1]), ch.pc[l][1][0]);
                    v = fmaf(r, Wv.c1[u], Wv.c0[u]) * (float)fma(cp, sp, cx * sx);
                  }
                }
              }
              // constant indices keep the channels in registers
#pragma unroll
              for (int idx = 0; idx < 2 * kFR; ++idx) {
                const int src = my_rank * (2 * kFR) + idx - rb;
                const float got = __shfl(v, src & 63, 64);
                const int gok = __shfl(good, src & 63, 64);
                if (my_rank >= 0 && src >= 0 && src < 64) {
                  const int q = idx % kFR;
                  const int chn = idx < kFR ? (l + 2) % 3 : (l + 1) % 3;
                  if (chn == 0) Xc[q] += got;
                  else if (chn == 1) Xb[q] += got;
                  else Xa[q] += got;
                  if (!gok) ok = false;
                }
              }
            }
          }
          // after three links: X = Xc, Y = Xb, Z = Xa.  Hybrid: w+ = 1/(1+e^z),
          // z = (k - kH)/sigma, zero beyond k - kH = T/2; a wave whose outputs all
          // have z <= -17 (w+ rounds to 1 in FP32) skips the weight.
          const double relL = (double)(kw0 + kFR * lane) - kH;   // k - kH of the lane's first output
          const double isg = 1.0 / P.sigma_s;
          const bool weigh = P.mode == 2 && ((double)(kw0 + wcnt - 1) - kH) * isg > -17.0;
          const int64_t o0 = off + kw0 + kFR * lane;
#pragma unroll
          for (int q = 0; q < kFR; ++q) {
            if (q >= nl) continue;
            float x = Xc[q], y = Xb[q], z = Xa[q];
            if (!ok) x = y = z = __builtin_nanf("");
            if (weigh) {
              const double rel = relL + (double)q;
              if (rel <= 0.5 * P.T_s) {
                const float zz = (float)(rel * isg);
                if (zz > -17.0f) {
                  const float wgt = 1.0f / (1.0f + expf(zz));
                  x *= wgt; y *= wgt; z *= wgt;
                }
              } else {
                x = y = z = 0.0f;
              }
            }
            store3<float>(P, o0 + q, x, y, z);
          }
        }
      } else {
        for (int i = tid; i < ccnt; i += kBlock)
          store3<float>(P, off + kc0 + i, __builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""));
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// TDI 2.0 LFA from the TDI 1.5 LFA series, Eq. (relation_X20_X15_nonequal_
// timedelays): X2.0(t_k) = 2 (T2+T3)(t_k) I_N[D1 X1.5](k - (T2+T3)(t_k)/dt),
// Y and Z by cyclic relabelling (equal arms: 4L/c and 2L/c).  The TDI 1.5 LFA
// series of every sample of each source comes from an earlier FP64 launch of
// the LFA kernel into P.x15 (three channel arrays of P.x15_stride doubles).
// Per tile of kTileLfa outputs its window is staged in LDS, differentiated by
// the central first-derivative stencil of accuracy p (zero outside the series),
// and read at the fractional delay with exact FP64 Lagrange weights.
// ---------------------------------------------------------------------------
struct X20Shared {
  GeoFit F;
  int64_t src, k0, g0;
  int32_t cnt, nw, bad;
  double kH;
  double qext[2][2];
};

template <int N, typename TC>
__global__ __launch_bounds__(kBlock, 2) void k_x20(const KParams* __restrict__ Pp) {
  const KParams& P = *Pp;
  const SrcDev* __restrict__ SS = sources_of(Pp);
  __shared__ X20Shared sh;
  __shared__ int64_t s_next;
  extern __shared__ __align__(16) char dyn[];
  const int cap = P.cap_g;
  double* xw = reinterpret_cast<double*>(dyn);            // [3][cap]: X1.5 window
  double* dw = xw + 3 * (size_t)cap;                       // [3][cap]: its first derivative
  const int tid = threadIdx.x;
  double sc[7], den;
  int hw;
  stencil_coeffs(1, P.stencil_p, sc, hw, den);

  int64_t iter = 0;
  for (;;) {
    const int64_t tile = next_tile(P, P.counters + 0, P.n_tiles_lfa, iter, &s_next);
    if (tile >= P.n_tiles_lfa) break;
    if (tid < 64) {
      const int64_t s = find_source_wave(SS, P.n_src, tile, true);
      if (tid == 0) {
        const SrcDev& S = SS[s];
        sh.src = s;
        sh.k0 = S.lfa_kb + (tile - S.lfa_t0) * kTileLfa;
        sh.cnt = (int32_t)min((int64_t)kTileLfa, S.lfa_ke - sh.k0);
        sh.kH = P.mode == 2 ? (S.t_hyb - S.t0) / S.dt : -INFINITY;
      }
    }
    __syncthreads();
    const SrcDev& S = SS[sh.src];
    const int64_t k0 = sh.k0;
    const int cnt = sh.cnt;
    fit_geometry(P, S, (double)k0, (double)(k0 + cnt - 1), sh.F);
    // window of the derivative series from the three channel delays at both ends
    if (tid < 2) {
      const int64_t k = tid == 0 ? k0 : k0 + cnt - 1;
      const double s = ((double)k - sh.F.kc) * sh.F.ikh;
      double qmin = 1e300, qmax = -1e300;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double Ta = P.equal_arms ? P.orb.L_over_c : geo_eval(sh.F, qT((c + 1) % 3), s);
        const double Tb = P.equal_arms ? P.orb.L_over_c : geo_eval(sh.F, qT((c + 2) % 3), s);
        qmin = fmin(qmin, (Ta + Tb) / S.dt);
        qmax = fmax(qmax, (Ta + Tb) / S.dt);
      }
      sh.qext[tid][0] = qmin;
      sh.qext[tid][1] = qmax;
    }
    __syncthreads();
    if (tid == 0) {
      const double qmin = fmin(sh.qext[0][0], sh.qext[1][0]);
      const double qmax = fmax(sh.qext[0][1], sh.qext[1][1]);
      const int margin = 2 + (int)ceil(4e-4 * (double)cnt);
      sh.g0 = k0 - (int64_t)ceil(qmax) - N / 2 + 1 - margin;
      const int64_t g1 = k0 + cnt - 1 - (int64_t)floor(qmin) + N / 2 + margin;
      sh.nw = (int32_t)(g1 - sh.g0 + 1);
      sh.bad = sh.nw + 2 * hw > cap ? 1 : 0;
      if (sh.bad) report(P.err, 1, k0, sh.nw, cap);
    }
    __syncthreads();
    const int64_t g0 = sh.g0;
    const int nw = sh.nw;
    const bool bad = sh.bad != 0;
    const double kH = sh.kH;
    if (!bad) {
      for (int i = tid; i < nw + 2 * hw; i += kBlock) {
        const int64_t j = g0 - hw + i;
        const bool in = j >= 0 && j < S.n;
#pragma unroll
        for (int c = 0; c < 3; ++c)
          xw[c * cap + i] = in ? P.x15[(size_t)c * P.x15_stride + S.off + j] : 0.0;
      }
      __syncthreads();
      const double iden = 1.0 / (den * S.dt);
      for (int i = tid; i < nw; i += kBlock) {
        const int64_t j = g0 + i;
        const bool in = j >= 0 && j < S.n;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double a = 0.0;
          for (int q = 0; q <= 2 * hw; ++q) a = fma(sc[q], xw[c * cap + i + q], a);
          dw[c * cap + i] = in ? a * iden : 0.0;
        }
      }
      __syncthreads();
    }
    for (int i = tid; i < cnt; i += kBlock) {
      const int64_t k = k0 + i;
      double out[3];
      if (bad) {
        out[0] = out[1] = out[2] = __builtin_nan("");
      } else {
        const double s = ((double)k - sh.F.kc) * sh.F.ikh;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double Ta = P.equal_arms ? P.orb.L_over_c : geo_eval(sh.F, qT((c + 1) % 3), s);
          const double Tb = P.equal_arms ? P.orb.L_over_c : geo_eval(sh.F, qT((c + 2) % 3), s);
          int64_t i0;
          double x;
          split(k, Ta + Tb, S.dt, i0, x);
          const int64_t b = i0 - N / 2 + 1 - g0;
          double v;
          if (b < 0 || b + N > nw) {
            report(P.err, 2, k, b, nw);
            v = __builtin_nan("");
          } else if (x == 0.0) {
            v = dw[c * cap + b + N / 2 - 1];
          } else {
            lag_interp<N, 1, double>(x, dw + c * cap + b, &v);
          }
          out[c] = 2.0 * (Ta + Tb) * v;
        }
      }
      if (P.mode == 2) {
        const double rel = (double)k - kH;
        if (rel <= 0.5 * P.T_s) {
          const double w = 1.0 / (1.0 + exp(rel / P.sigma_s));
          out[0] *= w;
          out[1] *= w;
          out[2] *= w;
        } else {
          out[0] = out[1] = out[2] = 0.0;
        }
      }
      store3<TC>(P, S.off + k, (TC)out[0], (TC)out[1], (TC)out[2]);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Full-response kernel
// ---------------------------------------------------------------------------
struct FullShared {
  GeoFit F;
  int64_t src, k0, y0, w0;
  int32_t cnt, ny, nh, bad;
  double c2, s2, kH;
  double dext[4];
};

template <int N, typename TC>
__device__ __forceinline__ void interp2(const TC* win, int64_t b, double x, TC& vp, TC& vc) {
  if (x == 0.0) {
    vp = win[2 * (b + N / 2 - 1)];
    vc = win[2 * (b + N / 2 - 1) + 1];
    return;
  }
  TC v[2];
  lag_interp<N, 2, TC>(x, win + 2 * b, v);
  vp = v[0];
  vc = v[1];
}

// Channel c of full-response output o.  Hybrid: add w- X^Full to the LFA part
// that the LFA kernel wrote inside its window (k - kH <= T/2), else store.
template <typename TC>
__device__ __forceinline__ void full_store(const KParams& P, int64_t o, int c, double v, double rel) {
  TC* out = static_cast<TC*>(c == 0 ? P.X : (c == 1 ? P.Y : P.Z));
  if (P.mode == 2) {
    const double w = 1.0 / (1.0 + exp(-rel / P.sigma_s));
    const bool has_lfa = rel <= 0.5 * P.T_s;
    if constexpr (sizeof(TC) == 8) {
      out[o] = (has_lfa ? out[o] : 0.0) + w * v;
    } else {
      out[o] = (has_lfa ? out[o] : 0.0f) + (float)w * (float)v;
    }
  } else {
    out[o] = (TC)v;
  }
}

// TP: the hybrid's variant (tiles of at most kTileFullHybrid outputs): stage 1
// per (sample, receiving spacecraft), stage 2 per (output, channel, term) with
// the term values in LDS.  The FULL mode's variant (larger tiles) takes one
// work item per sample in stage 1 and one per output in stage 2.
template <int N, typename TC, bool TP>
__global__ __launch_bounds__(kBlock, 2) void k_full(const KParams* __restrict__ Pp) {
  const KParams& P = *Pp;
  const SrcDev* __restrict__ SS = sources_of(Pp);
  __shared__ FullShared sh;
  __shared__ int64_t s_next;
  extern __shared__ __align__(16) char dyn[];
  const int tid = threadIdx.x;
  const int cap_y = P.cap_y;
  TC* hwin = reinterpret_cast<TC*>(dyn);                                        // [cap_hf][2]
  TC* ywin = reinterpret_cast<TC*>(dyn + align16((size_t)P.cap_hf * 2 * sizeof(TC)));  // [6][cap_y]
  double* Tc = reinterpret_cast<double*>(dyn + align16((size_t)P.cap_hf * 2 * sizeof(TC)) +
                                         align16((size_t)cap_y * 6 * sizeof(TC)));       // [9][kTileFull]
  TC* tv = reinterpret_cast<TC*>(Tc + 9 * kTileFull);   // hybrid: [tile * 3][terms] signed term values

  int64_t iter = 0;
  for (;;) {
    const int64_t tile = next_tile(P, P.counters + 1, P.n_tiles_full, iter, &s_next);
    if (tile >= P.n_tiles_full) break;
    if (tid < 64) {
      const int64_t s = find_source_wave(SS, P.n_src, tile, false);
      if (tid == 0) {
        const SrcDev& S = SS[s];
        sh.src = s;
        sh.k0 = S.full_kb + (tile - S.full_t0) * P.tile_full;
        sh.cnt = (int32_t)min((int64_t)P.tile_full, S.full_ke - sh.k0);
        const int margin = 2 + (int)ceil(4e-4 * (double)sh.cnt);
        sh.y0 = sh.k0 - (int64_t)ceil(P.D2_bound / S.dt) - N / 2 + 1 - margin;
        sh.ny = (int32_t)(sh.k0 + sh.cnt - 1 + N / 2 + margin - sh.y0 + 1);
        double sn, cs;
        sincos(2.0 * S.psi, &sn, &cs);
        sh.c2 = cs;
        sh.s2 = sn;
        sh.kH = P.mode == 2 ? (S.t_hyb - S.t0) / S.dt : -INFINITY;
      }
    }
    __syncthreads();
    const SrcDev& S = SS[sh.src];
    const int64_t k0 = sh.k0, y0 = sh.y0;
    const int cnt = sh.cnt, ny = sh.ny;
    fit_geometry(P, S, (double)y0, (double)(y0 + ny - 1), sh.F);

    // h window from the stage-1 delays at both ends of the y window
    if (tid < 2) {
      const int64_t i = tid == 0 ? y0 : y0 + ny - 1;
      const double s = ((double)i - sh.F.kc) * sh.F.ikh;
      double kR[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) kR[q] = geo_eval(sh.F, qKR(q), s);
      double dmin = 1e300, dmax = -1e300;
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const double T = geo_eval(sh.F, qT(a), s);
        const double ds = T + kR[snd_of(a)], dr = kR[rcv_of(a)];
        dmin = fmin(dmin, fmin(ds, dr));
        dmax = fmax(dmax, fmax(ds, dr));
      }
      sh.dext[2 * tid] = dmin;
      sh.dext[2 * tid + 1] = dmax;
    }
    __syncthreads();
    if (tid == 0) {
      const double dmin = fmin(sh.dext[0], sh.dext[2]), dmax = fmax(sh.dext[1], sh.dext[3]);
      const int margin = 2 + (int)ceil(4e-4 * (double)ny);
      const int64_t w0 = y0 - (int64_t)ceil(dmax / S.dt) - N / 2 + 1 - margin;
      const int64_t w1 = y0 + ny - 1 - (int64_t)floor(dmin / S.dt) + N / 2 + margin;
      sh.w0 = w0;
      sh.nh = (int32_t)(w1 - w0 + 1);
      sh.bad = (sh.nh > P.cap_hf || ny > cap_y) ? 1 : 0;
      if (sh.bad) report(P.err, 4, k0, ny, sh.nh);
    }
    __syncthreads();
    const int64_t w0 = sh.w0;
    const int nh = sh.nh;
    const bool bad = sh.bad != 0;
    const double dt = S.dt;

    if (!bad) {
      for (int i = tid; i < nh; i += kBlock) {
        const int64_t j = w0 + i;
        const bool in = j >= 0 && j < S.n;
        hwin[2 * i] = (TC)(in ? P.hp[S.off + j] : 0.0);
        hwin[2 * i + 1] = (TC)(in ? P.hc[S.off + j] : 0.0);
      }
      __syncthreads();
      // Stage 1: y_l[i] = [H_l(t_i - ds) - H_l(t_i - dr)] / (2 (1 - k.n)), zero
      // outside the series; antenna patterns at the reception time t_i.  The
      // receiver read is shared by the two links into each spacecraft.
      const double c2 = sh.c2, s2 = sh.s2;
      if constexpr (TP) {
        // hybrid tiles: one work item per (sample, receiving spacecraft), so
        // that a small tile still spreads over the workgroup
        for (int it = tid; it < ny * 3; it += kBlock) {
          const int ii = it / 3, r = it - 3 * ii;
          const int64_t i = y0 + ii;
          // the links received by spacecraft r (slots with rcv_of(a) == r)
          const int la = r == 0 ? 2 : (r == 1 ? 0 : 1), lb = r == 0 ? 4 : (r == 1 ? 5 : 3);
          if (!(i >= 0 && i < S.n)) {
            ywin[la * cap_y + ii] = (TC)0;
            ywin[lb * cap_y + ii] = (TC)0;
            continue;
          }
          const double s = ((double)i - sh.F.kc) * sh.F.ikh;
          TC hr[2];
          {
            int64_t i0;
            double x;
            split(i, geo_eval(sh.F, qKR(r), s), dt, i0, x);
            const int64_t b = i0 - N / 2 + 1 - w0;
            if (b < 0 || b + N > nh) {
              report(P.err, 8, i, b, nh);
              hr[0] = hr[1] = (TC)__builtin_nan("");
            } else {
              interp2<N, TC>(hwin, b, x, hr[0], hr[1]);
            }
          }
  #pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int a = q == 0 ? la : lb;
            const double T = geo_eval(sh.F, qT(a), s);
            if (i >= k0 && i < k0 + cnt) Tc[a * kTileFull + (int)(i - k0)] = T;
            int64_t i0;
            double x;
            split(i, T + geo_eval(sh.F, qKR(snd_of(a)), s), dt, i0, x);
            const int64_t b = i0 - N / 2 + 1 - w0;
            TC vp, vc;
            if (b < 0 || b + N > nh) {
              report(P.err, 8, i, b, nh);
              vp = vc = (TC)__builtin_nan("");
            } else {
              interp2<N, TC>(hwin, b, x, vp, vc);
            }
            const double xp = geo_eval(sh.F, qXp(a), s), xc = geo_eval(sh.F, qXc(a), s);
            const TC A = (TC)(xp * c2 + xc * s2), B = (TC)(xc * c2 - xp * s2);
            const TC Hs = A * vp + B * vc;
            const TC Hr = A * hr[0] + B * hr[1];
            ywin[a * cap_y + ii] = (Hs - Hr) / (TC)geo_eval(sh.F, qD(a), s);
          }
        }
      } else {
        // FULL tiles: one work item per sample (its three receiver reads and
        // six links), the geometry evaluated once per sample
        for (int ii = tid; ii < ny; ii += kBlock) {
          const int64_t i = y0 + ii;
          if (!(i >= 0 && i < S.n)) {
#pragma unroll
            for (int a = 0; a < 6; ++a) ywin[a * cap_y + ii] = (TC)0;
            continue;
          }
          const double s = ((double)i - sh.F.kc) * sh.F.ikh;
          const double kR0 = geo_eval(sh.F, qKR(0), s), kR1 = geo_eval(sh.F, qKR(1), s),
                       kR2 = geo_eval(sh.F, qKR(2), s);
          // the receiver read is shared by the two links into each spacecraft
          TC hr[6];
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            int64_t i0;
            double x;
            split(i, sel3(kR0, kR1, kR2, q), dt, i0, x);
            const int64_t b = i0 - N / 2 + 1 - w0;
            if (b < 0 || b + N > nh) {
              report(P.err, 8, i, b, nh);
              hr[2 * q] = hr[2 * q + 1] = (TC)__builtin_nan("");
            } else {
              interp2<N, TC>(hwin, b, x, hr[2 * q], hr[2 * q + 1]);
            }
          }
#pragma unroll 1
          for (int a = 0; a < 6; ++a) {
            const double T = geo_eval(sh.F, qT(a), s);
            if (i >= k0 && i < k0 + cnt) Tc[a * kTileFull + (int)(i - k0)] = T;
            int64_t i0;
            double x;
            split(i, T + sel3(kR0, kR1, kR2, snd_of(a)), dt, i0, x);
            const int64_t b = i0 - N / 2 + 1 - w0;
            TC vp, vc;
            if (b < 0 || b + N > nh) {
              report(P.err, 8, i, b, nh);
              vp = vc = (TC)__builtin_nan("");
            } else {
              interp2<N, TC>(hwin, b, x, vp, vc);
            }
            const double xp = geo_eval(sh.F, qXp(a), s), xc = geo_eval(sh.F, qXc(a), s);
            const TC A = (TC)(xp * c2 + xc * s2), B = (TC)(xc * c2 - xp * s2);
            const int r = rcv_of(a);
            const TC hrp = r == 0 ? hr[0] : (r == 1 ? hr[2] : hr[4]);
            const TC hrc = r == 0 ? hr[1] : (r == 1 ? hr[3] : hr[5]);
            const TC Hs = A * vp + B * vc;
            const TC Hr = A * hrp + B * hrc;
            ywin[a * cap_y + ii] = (Hs - Hr) / (TC)geo_eval(sh.F, qD(a), s);
          }
        }
      }
    }
    __syncthreads();

    // Stage 2: sum of +-y_l at the term delays, light times at the output time
    // (or time-nested: each light time from the fit at its retarded sample).
    const int nterms = P.gen == 20 ? 16 : 8;
    const double kH = sh.kH;
    if constexpr (TP) {
      // the signed value of term t of channel c at output i (T6: the light times
      // at the output)
      auto term = [&](int i, int c, int t, const double (&T6)[6]) -> TC {
        const int64_t k = k0 + i;
        double d = 0.0;
        int slot, sign;
        if (P.nested) {
#pragma unroll 1
          for (int q = 0; q < c_nlen[t]; ++q) {
            const double sq = ((double)k - d / dt - sh.F.kc) * sh.F.ikh;
            d += geo_eval(sh.F, qT(rot_slot(c_nseq[t][q], c)), sq);
          }
          slot = c_nlink[t];
          sign = c_nsign[t];
        } else {
#pragma unroll
          for (int a = 0; a < 6; ++a) d += (double)c_tcoef[t][unrot_slot(a, c)] * T6[a];
          slot = c_tlink[t];
          sign = c_tsign[t];
        }
        const TC* ys = ywin + rot_slot(slot, c) * cap_y;
        TC v;
        if (d == 0.0) {
          v = ys[k - y0];
        } else {
          int64_t i0;
          double x;
          split(k, d, dt, i0, x);
          const int64_t b = i0 - N / 2 + 1 - y0;
          if (b < 0 || b + N > ny) {
            report(P.err, 16, k, b, ny);
            v = (TC)__builtin_nan("");
          } else if (x == 0.0) {
            v = ys[b + N / 2 - 1];
          } else {
            TC vv[1];
            lag_interp<N, 1, TC>(x, ys + b, vv);
            v = vv[0];
          }
        }
        return sign > 0 ? v : -v;
      };
      // Hybrid tiles (at most kTileFullHybrid outputs) take one work item per
      // (output, channel, term), so that a tile's latency is a few reads rather
      // than all of a channel's terms in sequence; the terms are then summed in
      // their order, as the per-(output, channel) loop below does.
      if (!bad) {
        for (int it = tid; it < cnt * 3 * nterms; it += kBlock) {
          const int t = it % nterms, ic = it / nterms, i = ic / 3, c = ic - 3 * i;
          const double rel = (double)(k0 + i) - kH;
          if (P.mode == 2 && !(rel >= -0.5 * P.T_s)) continue;
          double T6[6];
#pragma unroll
          for (int a = 0; a < 6; ++a) T6[a] = Tc[a * kTileFull + i];
          tv[it] = term(i, c, t, T6);
        }
        __syncthreads();
      }
      for (int it = tid; it < cnt * 3; it += kBlock) {
        const int i = it / 3, c = it - 3 * i;
        const int64_t k = k0 + i;
        const double rel = (double)k - kH;
        if (P.mode == 2 && !(rel >= -0.5 * P.T_s)) continue;
        double outc;
        if (bad) {
          outc = __builtin_nan("");
        } else {
          TC sum = (TC)0;
          for (int t = 0; t < nterms; ++t) sum += tv[it * nterms + t];
          outc = (double)sum;
        }
        if (P.aet) {
          // A, E, T mix the channels: the three items of an output meet in LDS
          Tc[(6 + c) * kTileFull + i] = outc;
          continue;
        }
        full_store<TC>(P, S.off + k, c, outc, rel);
      }
    } else {
      // FULL tiles: one work item per output, its three channels in turn
      for (int i = tid; i < cnt; i += kBlock) {
        const int64_t k = k0 + i;
        const double rel = (double)k - kH;
        if (P.mode == 2 && !(rel >= -0.5 * P.T_s)) continue;
        double out[3];
        if (bad) {
          out[0] = out[1] = out[2] = __builtin_nan("");
        } else {
          double T6[6];
#pragma unroll
          for (int a = 0; a < 6; ++a) T6[a] = Tc[a * kTileFull + i];
#pragma unroll 1
          for (int c = 0; c < 3; ++c) {
            TC sum = (TC)0;
#pragma unroll 1
            for (int t = 0; t < nterms; ++t) {
              double d = 0.0;
              int slot, sign;
              if (P.nested) {
#pragma unroll 1
                for (int q = 0; q < c_nlen[t]; ++q) {
                  const double sq = ((double)k - d / dt - sh.F.kc) * sh.F.ikh;
                  d += geo_eval(sh.F, qT(rot_slot(c_nseq[t][q], c)), sq);
                }
                slot = c_nlink[t];
                sign = c_nsign[t];
              } else {
#pragma unroll
                for (int a = 0; a < 6; ++a) d += (double)c_tcoef[t][unrot_slot(a, c)] * T6[a];
                slot = c_tlink[t];
                sign = c_tsign[t];
              }
              const TC* ys = ywin + rot_slot(slot, c) * cap_y;
              TC v;
              if (d == 0.0) {
                v = ys[k - y0];
              } else {
                int64_t i0;
                double x;
                split(k, d, dt, i0, x);
                const int64_t b = i0 - N / 2 + 1 - y0;
                if (b < 0 || b + N > ny) {
                  report(P.err, 16, k, b, ny);
                  v = (TC)__builtin_nan("");
                } else if (x == 0.0) {
                  v = ys[b + N / 2 - 1];
                } else {
                  TC vv[1];
                  lag_interp<N, 1, TC>(x, ys + b, vv);
                  v = vv[0];
                }
              }
              sum += sign > 0 ? v : -v;
            }
            if (c == 0) out[0] = (double)sum; else if (c == 1) out[1] = (double)sum; else out[2] = (double)sum;
          }
        }
        if (P.aet) to_aet<double>(out[0], out[1], out[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) full_store<TC>(P, S.off + k, c, out[c], rel);
      }
    }
    if constexpr (TP) {
      // A, E, T of the term-parallel items
      if (P.aet) {
        __syncthreads();
        for (int i = tid; i < cnt; i += kBlock) {
          const int64_t k = k0 + i;
          const double rel = (double)k - kH;
          if (P.mode == 2 && !(rel >= -0.5 * P.T_s)) continue;
          double o3[3] = {Tc[6 * kTileFull + i], Tc[7 * kTileFull + i], Tc[8 * kTileFull + i]};
          to_aet<double>(o3[0], o3[1], o3[2]);
#pragma unroll
          for (int c = 0; c < 3; ++c) full_store<TC>(P, S.off + k, c, o3[c], rel);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Link outputs: the six single links y_slr on the grid of each source.
//   full:   Eq. (yslr), y = [H_l(t - delta_s) - H_l(t - delta_r)] / (2 (1 - k.n)),
//           H_l from Eq. (H) with the antenna patterns at the reception time;
//   LFA:    Eq. (yslr_strain_derivatives) for every link,
//           y = -(T_l / 2) [xi+ h+'(t - T_l/2 - mu_l) + xi_x hx'(...)],
//           mu_l = k.(R_s + R_r)/(2c), h' the first derivative by the central
//           stencil of accuracy p on the grid (zero outside the series);
//           with two terms, the next term of Eq. (yslr_with_tau_derivatives),
//           (T_l (1 - k.n_l) / 2)^2 / 6 times the third derivative, joins h';
//   hybrid: Eq. (hybridized_yslr) with the windows and weights of the TDI hybrid.
// One workgroup per tile of kTileLinks outputs (one geometry fit per tile), each
// thread taking every kBlock-th output.
// FP32-bulk LFA (leading term): the two links of an arm (l and -l) read the
// derivative series at delays that differ by (T_l - T_-l) / 2, ~1e-4 samples.
// Per arm the two components are read once, at the mean offset of the two
// links, with weights from the Taylor table (a row shared by the wave,
// re-expanded per lane): values A+-, slopes B+-; each link takes A + (its
// offset - the mean) B with its own polarisation factors (those of l and -l
// differ through aberration, so the components are not precombined per arm).  Reads whose nodes touch a series end, whose two offsets straddle
// an integer, or whose lane is far from the wave's table row take the exact
// two-component path.
// ---------------------------------------------------------------------------
struct LinkShared {
  GeoFit F;
  int64_t src, k0, w0;
  int32_t cnt, nh, bad, pad;
  double c2, s2, kH;
  double dext[4];
};

// ARM: the FP32 per-arm read of the leading-term LFA (launched for the LFA and
// hybrid modes in FP32-bulk); without it the kernel is the exact path alone.
template <int N, typename TC, bool ARM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ARM ? 2 : 1))) void k_links(const KParams* __restrict__ Pp) {
  const KParams& P = *Pp;
  const SrcDev* __restrict__ SS = sources_of(Pp);
  __shared__ LinkShared sh;
  extern __shared__ __align__(16) char dyn[];
  const int tid = threadIdx.x;
  const int cap = P.cap_lk;
  TC* hwin = reinterpret_cast<TC*>(dyn);                                              // [cap][2]
  TC* gwin = reinterpret_cast<TC*>(dyn + align16((size_t)cap * 2 * sizeof(TC)));     // [cap][2]
  TC* g3win = reinterpret_cast<TC*>(dyn + 2 * align16((size_t)cap * 2 * sizeof(TC)));  // [cap][2]
  const int64_t tile = blockIdx.x;
  if (tile >= P.n_tiles_lfa) return;
  const bool want_lfa = P.mode != 0, want_full = P.mode != 1;
  // the per-arm read: FP32, leading LFA term
  static_assert(!ARM || sizeof(TC) == 4, "the per-arm read is FP32");
  const bool arm_fast = ARM && want_lfa && P.lfa_terms != 2;
  if (tid < 64) {
    const int64_t s = find_source_wave(SS, P.n_src, tile, true);
    if (tid == 0) {
      const SrcDev& S = SS[s];
      sh.src = s;
      sh.k0 = (tile - S.lfa_t0) * kTileLinks;
      sh.cnt = (int32_t)min((int64_t)kTileLinks, S.n - sh.k0);
      sh.c2 = S.c2psi;
      sh.s2 = S.s2psi;
      sh.kH = P.mode == 2 ? (S.t_hyb - S.t0) / S.dt : 0.0;
    }
  }
  __syncthreads();
  const SrcDev& S = SS[sh.src];
  const int64_t k0 = sh.k0;
  const int cnt = sh.cnt;
  fit_geometry(P, S, (double)k0, (double)(k0 + cnt - 1), sh.F);
  // read window from every delay at both ends of the tile
  if (tid < 2) {
    const int64_t i = tid == 0 ? k0 : k0 + cnt - 1;
    const double s = ((double)i - sh.F.kc) * sh.F.ikh;
    double kR[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) kR[q] = geo_eval(sh.F, qKR(q), s);
    double dmin = 1e300, dmax = -1e300;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const double T = geo_eval(sh.F, qT(a), s);
      const double Tl = P.equal_arms ? P.orb.L_over_c : T;
      const double ds = T + kR[snd_of(a)], dr = kR[rcv_of(a)];
      const double dl = 0.5 * Tl + 0.5 * (kR[snd_of(a)] + kR[rcv_of(a)]);
      dmin = fmin(dmin, fmin(fmin(ds, dr), dl));
      dmax = fmax(dmax, fmax(fmax(ds, dr), dl));
    }
    sh.dext[2 * tid] = dmin;
    sh.dext[2 * tid + 1] = dmax;
  }
  __syncthreads();
  if (tid == 0) {
    const double dmin = fmin(sh.dext[0], sh.dext[2]), dmax = fmax(sh.dext[1], sh.dext[3]);
    const int margin = 2 + (int)ceil(4e-4 * (double)cnt);
    const int64_t w0 = k0 - (int64_t)ceil(dmax / S.dt) - N / 2 + 1 - margin;
    const int64_t w1 = k0 + cnt - 1 - (int64_t)floor(dmin / S.dt) + N / 2 + margin;
    sh.w0 = w0;
    sh.nh = (int32_t)(w1 - w0 + 1);
    sh.bad = sh.nh > cap ? 1 : 0;
    if (sh.bad) report(P.err, 16, k0, 0, sh.nh);
  }
  __syncthreads();
  const int64_t w0 = sh.w0;
  const int nh = sh.nh;
  const double dt = S.dt;
  const int64_t stride = P.link_stride;
  TC* Yo = static_cast<TC*>(P.X);
  if (sh.bad) {
    for (int o = tid; o < cnt; o += kBlock)
      for (int a = 0; a < 6; ++a) Yo[a * stride + S.off + k0 + o] = (TC)__builtin_nan("");
    return;
  }
  // strain window (full part) and first-derivative window (LFA part), the
  // derivative taken in FP64 on the grid from the strain in global memory
  double st[7], st3[7];
  int hw, hw3;
  double den, den3;
  stencil_coeffs(1, P.stencil_p, st, hw, den);
  stencil_coeffs(3, P.stencil_p, st3, hw3, den3);
  const double gscale = 1.0 / (den * dt), g3scale = 1.0 / (den3 * dt * dt * dt);
  // the stencils on the seven offsets -3..3 (zero beyond the half width), so
  // that the tap loops index them with constants
  double sc1[7], sc3[7];
#pragma unroll
  for (int o = 0; o < 7; ++o) {
    sc1[o] = hw == 3 ? st[o] : (hw == 2 ? (o >= 1 && o <= 5 ? st[o - 1] : 0.0) : (o >= 2 && o <= 4 ? st[o - 2] : 0.0));
    sc3[o] = hw3 == 3 ? st3[o]
                      : (hw3 == 2 ? (o >= 1 && o <= 5 ? st3[o - 1] : 0.0) : (o >= 2 && o <= 4 ? st3[o - 2] : 0.0));
  }
  const bool nlo = want_lfa && P.lfa_terms == 2;
  // the window loads go out ahead of the other resident workgroups' arithmetic
  __builtin_amdgcn_s_setprio(1);
  for (int i = tid; i < nh; i += kBlock) {
    const int64_t j = w0 + i;
    const bool in = j >= 0 && j < S.n;
    if (want_full) {
      hwin[2 * i] = (TC)(in ? P.hp[S.off + j] : 0.0);
      hwin[2 * i + 1] = (TC)(in ? P.hc[S.off + j] : 0.0);
    }
    if (want_lfa) {
      double gp = 0.0, gc = 0.0;
      if (in) {
#pragma unroll
        for (int o = 0; o < 7; ++o) {
          const int64_t jj = j + o - 3;
          if (sc1[o] != 0.0 && jj >= 0 && jj < S.n) {
            gp += sc1[o] * P.hp[S.off + jj];
            gc += sc1[o] * P.hc[S.off + jj];
          }
        }
      }
      gwin[2 * i] = (TC)(gp * gscale);
      gwin[2 * i + 1] = (TC)(gc * gscale);
    }
    if (nlo) {
      double gp = 0.0, gc = 0.0;
      if (in) {
#pragma unroll
        for (int o = 0; o < 7; ++o) {
          const int64_t jj = j + o - 3;
          if (sc3[o] != 0.0 && jj >= 0 && jj < S.n) {
            gp += sc3[o] * P.hp[S.off + jj];
            gc += sc3[o] * P.hc[S.off + jj];
          }
        }
      }
      g3win[2 * i] = (TC)(gp * g3scale);
      g3win[2 * i + 1] = (TC)(gc * g3scale);
    }
  }
  __builtin_amdgcn_s_setprio(0);
  __syncthreads();
  for (int o = tid; o < cnt; o += kBlock) {
    const int64_t k = k0 + o;
    const double s = ((double)k - sh.F.kc) * sh.F.ikh;
    const double rel = (double)k - sh.kH;
    const bool lfa = P.mode == 1 || (P.mode == 2 && rel <= 0.5 * P.T_s);
    const bool full = P.mode == 0 || (P.mode == 2 && rel >= -0.5 * P.T_s);
    double wp = 1.0, wm = 1.0;
    if (P.mode == 2) {
      wp = 1.0 / (1.0 + exp(rel / P.sigma_s));
      wm = 1.0 / (1.0 + exp(-rel / P.sigma_s));
    }
    const double kR[3] = {geo_eval(sh.F, qKR(0), s), geo_eval(sh.F, qKR(1), s), geo_eval(sh.F, qKR(2), s)};
    const double c2 = sh.c2, s2 = sh.s2;
    // LFA values of the six links from the per-arm reads (bit a of xmask set:
    // link a takes the exact two-component read below instead)
    float yl[6];
    uint32_t xmask = 0x3fu;
#pragma unroll
    for (int a = 0; a < 6; ++a) yl[a] = 0.0f;
    if (arm_fast && lfa) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double Tp = P.equal_arms ? P.orb.L_over_c : geo_eval(sh.F, qT(a), s);
        const double Tm = P.equal_arms ? P.orb.L_over_c : geo_eval(sh.F, qT(a + 3), s);
        const double mu = 0.5 * (kR[snd_of(a)] + kR[rcv_of(a)]);
        const double qp = (0.5 * Tp + mu) / dt, qm = (0.5 * Tm + mu) / dt;
        const double qbar = 0.5 * (qp + qm), hd = 0.5 * (qp - qm);
        int64_t i0;
        double xbar;
        split(k, qbar * dt, dt, i0, xbar);
        const int64_t b = i0 - N / 2 + 1 - w0;
        const int64_t jlo = i0 - N / 2 + 1, jhi = i0 + N / 2;
        const bool edge = (jlo <= hw + 1 && jhi >= -hw - 2) || (jlo <= S.n + hw + 1 && jhi >= S.n - hw - 2);
        // the wave's table row, and this lane's expansion offset from it
        const int gl = min(max((int)rint(xbar * (double)kWGrid), 0), kWGrid);
        const int g = __builtin_amdgcn_readfirstlane(gl);
        const float e = (float)(xbar - (double)g / (double)kWGrid);
        const bool ok = !edge && b >= 0 && b + N <= nh && fabsf(e) <= 0.04f && xbar - fabs(hd) >= 0.0 &&
                        xbar + fabs(hd) < 1.0;
        if (__ballot(ok) == 0) continue;
        if (ok) {
          float Ap = 0.0f, Ac = 0.0f, Bp = 0.0f, Bc = 0.0f;
          const float4* row = wtab_row<N>(g);
          const float* Ga = reinterpret_cast<const float*>(gwin) + 2 * b;
#pragma unroll
          for (int j2 = 0; j2 < N; ++j2) {
            const float4 c = row[j2];
            const float b2 = fmaf(e, c.w, c.z);
            const float b1 = fmaf(e, b2, c.y);
            const float w = fmaf(e, b1, c.x);
            const float wd = fmaf(e, b2, b1);
            const float gp = Ga[2 * j2], gc = Ga[2 * j2 + 1];
            Ap = fmaf(w, gp, Ap);
            Ac = fmaf(w, gc, Ac);
            Bp = fmaf(wd, gp, Bp);
            Bc = fmaf(wd, gc, Bc);
          }
          // link a reads at xbar - hd, link a + 3 at xbar + hd, each with its
          // own polarisation factors at the output time
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const int l = a + 3 * side;
            const double xp = geo_eval(sh.F, qXp(l), s), xc = geo_eval(sh.F, qXc(l), s);
            const float cp = (float)(xp * c2 + xc * s2), cx = (float)(xc * c2 - xp * s2);
            const float dl = side == 0 ? -(float)hd : (float)hd;
            const float v = fmaf(cp, fmaf(dl, Bp, Ap), cx * fmaf(dl, Bc, Ac));
            yl[l] = (float)(wp * (-0.5 * (side == 0 ? Tp : Tm))) * v;
          }
          xmask &= ~((1u << a) | (1u << (a + 3)));
        }
      }
    }
#pragma unroll 1
    for (int a = 0; a < 6; ++a) {
      TC y = (TC)0;
      const bool exact = ((xmask >> a) & 1u) != 0;
      if (lfa && !exact) {
        float ysel = yl[0];
#pragma unroll
        for (int q = 1; q < 6; ++q) ysel = a == q ? yl[q] : ysel;
        y = (TC)ysel;
        if (!full) {
          Yo[a * stride + S.off + k] = y;
          continue;
        }
      }
      const double T = geo_eval(sh.F, qT(a), s);
      const double xp = geo_eval(sh.F, qXp(a), s), xc = geo_eval(sh.F, qXc(a), s);
      const TC A = (TC)(xp * c2 + xc * s2), B = (TC)(xc * c2 - xp * s2);
      const int sn = snd_of(a), rc = rcv_of(a);
      if (lfa && exact) {
        const double Tl = P.equal_arms ? P.orb.L_over_c : T;
        int64_t i0;
        double x;
        split(k, 0.5 * Tl + 0.5 * (kR[sn] + kR[rc]), dt, i0, x);
        const int64_t b = i0 - N / 2 + 1 - w0;
        TC vp, vc, v3p = (TC)0, v3c = (TC)0;
        if (b < 0 || b + N > nh) {
          report(P.err, 16, k, b, nh);
          vp = vc = (TC)__builtin_nan("");
        } else {
          interp2<N, TC>(gwin, b, x, vp, vc);
          if (nlo) interp2<N, TC>(g3win, b, x, v3p, v3c);
        }
        TC lf = A * vp + B * vc;
        if (nlo) {
          // (T (1 - k.n) / 2)^2 / 6 with 1 - k.n = D / 2
          const double e = 0.25 * Tl * geo_eval(sh.F, qD(a), s);
          lf += (TC)(e * e / 6.0) * (A * v3p + B * v3c);
        }
        y += (TC)(wp * (-0.5 * Tl)) * lf;
      }
      if (full) {
        TC v[4];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          int64_t i0;
          double x;
          split(k, e == 0 ? T + kR[sn] : kR[rc], dt, i0, x);
          const int64_t b = i0 - N / 2 + 1 - w0;
          if (b < 0 || b + N > nh) {
            report(P.err, 16, k, b, nh);
            v[2 * e] = v[2 * e + 1] = (TC)__builtin_nan("");
          } else {
            interp2<N, TC>(hwin, b, x, v[2 * e], v[2 * e + 1]);
          }
        }
        const TC Hs = A * v[0] + B * v[1], Hr = A * v[2] + B * v[3];
        y += (TC)wm * ((Hs - Hr) / (TC)geo_eval(sh.F, qD(a), s));
      }
      Yo[a * stride + S.off + k] = y;
    }
  }
}

template <int N, typename TC>
int launch_lfa_t(const KParams* dp, int nx, int grid, size_t lds, hipStream_t st) {
  if (nx) hipLaunchKernelGGL((k_lfa<N, TC, true>), dim3(grid), dim3(kBlock), lds, st, dp);
  else hipLaunchKernelGGL((k_lfa<N, TC, false>), dim3(grid), dim3(kBlock), lds, st, dp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N, typename TC>
int launch_x20_t(const KParams* dp, int grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k_x20<N, TC>), dim3(grid), dim3(kBlock), lds, st, dp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N, typename TC>
int occ_x20_t(size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_x20<N, TC>), kBlock, lds) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

template <int N, typename TC>
int launch_full_t(const KParams* dp, int tp, int grid, size_t lds, hipStream_t st) {
  if (tp) hipLaunchKernelGGL((k_full<N, TC, true>), dim3(grid), dim3(kBlock), lds, st, dp);
  else hipLaunchKernelGGL((k_full<N, TC, false>), dim3(grid), dim3(kBlock), lds, st, dp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N, typename TC>
int launch_links_t(const KParams* dp, int arm, int64_t grid, size_t lds, hipStream_t st) {
  if constexpr (sizeof(TC) == 4) {
    if (arm) {
      hipLaunchKernelGGL((k_links<N, TC, true>), dim3((unsigned)grid), dim3(kBlock), lds, st, dp);
      return hipGetLastError() == hipSuccess ? 0 : -1;
    }
  }
  hipLaunchKernelGGL((k_links<N, TC, false>), dim3((unsigned)grid), dim3(kBlock), lds, st, dp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
int launch_lfa_fast_t(const KParams* dp, int grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k_lfa_fast<N>), dim3(grid), dim3(kBlock), lds, st, dp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
int launch_lfa_fit_t(const KParams* dp, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_lfa_prep<N>), dim3(grid), dim3(kBlock), 0, st, dp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
int occ_lfa_fit_t() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_lfa_prep<N>), kBlock, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

template <int N>
int occ_lfa_fast_t(size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_lfa_fast<N>), kBlock, lds) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

template <int N, typename TC>
int occ_lfa_t(int nx, size_t lds) {
  int n = 0;
  const void* f = nx ? reinterpret_cast<const void*>(&k_lfa<N, TC, true>)
                     : reinterpret_cast<const void*>(&k_lfa<N, TC, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kBlock, lds) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

template <int N, typename TC>
int occ_full_t(int tp, size_t lds) {
  int n = 0;
  const void* f = tp ? reinterpret_cast<const void*>(&k_full<N, TC, true>)
                     : reinterpret_cast<const void*>(&k_full<N, TC, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kBlock, lds) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

template <int N, typename TC>
size_t wave_bytes_t() {
  return sizeof(TC) == 4 ? wave_tables_bytes<N>() : 0;
}

#define TDI_DISPATCH(taps, fp32, FN, ...)          \
  do {                                             \
    if (fp32) {                                    \
      switch (taps) {                              \
        case 4: return FN<4, float>(__VA_ARGS__);  \
        case 8: return FN<8, float>(__VA_ARGS__);  \
        case 16: return FN<16, float>(__VA_ARGS__); \
        case 32: return FN<32, float>(__VA_ARGS__); \
      }                                            \
    } else {                                       \
      switch (taps) {                              \
        case 4: return FN<4, double>(__VA_ARGS__); \
        case 8: return FN<8, double>(__VA_ARGS__); \
        case 16: return FN<16, double>(__VA_ARGS__); \
        case 32: return FN<32, double>(__VA_ARGS__); \
      }                                            \
    }                                              \
  } while (0)

size_t wave_bytes(int taps, int fp32) {
  TDI_DISPATCH(taps, fp32, wave_bytes_t);
  return 0;
}

#define TDI_DISPATCH_FAST(taps, FN, ...)           \
  do {                                             \
    switch (taps) {                                \
      case 4: return FN<4>(__VA_ARGS__);           \
      case 8: return FN<8>(__VA_ARGS__);           \
      case 16: return FN<16>(__VA_ARGS__);         \
      case 32: return FN<32>(__VA_ARGS__);         \
    }                                              \
  } while (0)

// Taylor coefficients of the Lagrange basis on nodes j - N/2 + 1 at x = g / kWGrid:
// l_j(x + y) = norm_j prod_{i != j} (x - x_i + y), expanded to y^3.
template <int N>
void lagrange_taylor_table(float out[kWGrid + 1][N][4]) {
  for (int g = 0; g <= kWGrid; ++g) {
    const long double x = (long double)g / (long double)kWGrid;
    for (int j = 0; j < N; ++j) {
      long double c[4] = {1.0L, 0.0L, 0.0L, 0.0L};
      long double den = 1.0L;
      for (int i = 0; i < N; ++i) {
        if (i == j) continue;
        const long double a = x - (long double)(i - N / 2 + 1);
        for (int d = 3; d >= 1; --d) c[d] = c[d] * a + c[d - 1];
        c[0] *= a;
        den *= (long double)(j - i);
      }
      for (int d = 0; d < 4; ++d) out[g][j][d] = (float)(c[d] / den);
    }
  }
}

template <int N>
int upload_taylor_table(const void* symbol) {
  static float tab[kWGrid + 1][N][4];
  lagrange_taylor_table<N>(tab);
  return hipMemcpyToSymbol(symbol, tab, sizeof(tab)) == hipSuccess ? 0 : -1;
}

}  // namespace

int set_constants() {
  // Chebyshev nodes of the first kind (the middle one is exactly 0) and the
  // inverse of the Vandermonde matrix V[j][m] = s_j^m.
  double s[kNodes], V[kNodes][2 * kNodes];
  for (int j = 0; j < kNodes; ++j) {
    s[j] = cos(M_PI * (2.0 * j + 1.0) / (2.0 * kNodes));
    if (j == kNodes / 2) s[j] = 0.0;
  }
  for (int j = 0; j < kNodes; ++j)
    for (int m = 0; m < 2 * kNodes; ++m)
      V[j][m] = m < kNodes ? pow(s[j], (double)m) : (m - kNodes == j ? 1.0 : 0.0);
  for (int c = 0; c < kNodes; ++c) {          // Gauss-Jordan with partial pivoting
    int piv = c;
    for (int r = c + 1; r < kNodes; ++r)
      if (fabs(V[r][c]) > fabs(V[piv][c])) piv = r;
    for (int m = 0; m < 2 * kNodes; ++m) {
      const double t = V[c][m];
      V[c][m] = V[piv][m];
      V[piv][m] = t;
    }
    const double d = V[c][c];
    for (int m = 0; m < 2 * kNodes; ++m) V[c][m] /= d;
    for (int r = 0; r < kNodes; ++r) {
      if (r == c) continue;
      const double f = V[r][c];
      for (int m = 0; m < 2 * kNodes; ++m) V[r][m] -= f * V[c][m];
    }
  }
  double inv[kNodes][kNodes];                 // coefficient m = sum_j inv[m][j] value_j
  for (int m = 0; m < kNodes; ++m)
    for (int j = 0; j < kNodes; ++j) inv[m][j] = V[m][kNodes + j];
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_vinv), inv, sizeof(inv)) != hipSuccess) return -1;
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_snode), s, sizeof(s)) != hipSuccess) return -1;
  if (upload_taylor_table<4>(HIP_SYMBOL(c_wtab4)) != 0) return -1;
  if (upload_taylor_table<8>(HIP_SYMBOL(c_wtab8)) != 0) return -1;
  if (upload_taylor_table<16>(HIP_SYMBOL(c_wtab16)) != 0) return -1;
  if (upload_taylor_table<32>(HIP_SYMBOL(c_wtab32)) != 0) return -1;
  return 0;
}

size_t fast_tile_bytes() { return sizeof(FastTile); }

size_t lfa_lds_bytes(int taps, int cap_g, int cap_h, int fp32, int fast, int nx, int* goff) {
  if (fast) {                                // the three F_l series only
    if (goff) *goff = 0;
    return align16((size_t)3 * (cap_g + kFR + 1) * sizeof(float));
  }
  const size_t tcs = fp32 ? sizeof(float) : sizeof(double);
  size_t hb = align16((size_t)cap_h * 2 * sizeof(double));
  const size_t wb = align16(wave_bytes(taps, fp32));
  if (wb > hb) hb = wb;
  if (goff) *goff = (int)hb;
  return hb + align16((size_t)cap_g * (nx ? 4 : 2) * tcs);
}

size_t full_lds_bytes(int cap_h, int cap_y, int fp32, int hybrid) {
  const size_t tcs = fp32 ? sizeof(float) : sizeof(double);
  // light times of the tile's outputs (6 rows) and, for A, E, T, the three
  // channels; the hybrid's term-parallel stage 2 keeps every term's value
  return align16((size_t)cap_h * 2 * tcs) + align16((size_t)cap_y * 6 * tcs) +
         (size_t)9 * kTileFull * sizeof(double) + (hybrid ? (size_t)kTileFullHybrid * 3 * 16 * tcs : 0);
}

int launch_lfa(const KParams* dp, int taps, int fp32, int fast, int nx, int grid, size_t lds, void* stream) {
  if (fast) {
    if (!fp32 || nx) return -2;
    TDI_DISPATCH_FAST(taps, launch_lfa_fast_t, dp, grid, lds, (hipStream_t)stream);
    return -2;
  }
  TDI_DISPATCH(taps, fp32, launch_lfa_t, dp, nx, grid, lds, (hipStream_t)stream);
  return -2;
}

int launch_lfa_fit(const KParams* dp, int taps, int grid, void* stream) {
  TDI_DISPATCH_FAST(taps, launch_lfa_fit_t, dp, grid, (hipStream_t)stream);
  return -2;
}

int occupancy_lfa_fit(int taps) {
  TDI_DISPATCH_FAST(taps, occ_lfa_fit_t);
  return 1;
}

int launch_x20(const KParams* dp, int taps, int fp32, int grid, size_t lds, void* stream) {
  TDI_DISPATCH(taps, fp32, launch_x20_t, dp, grid, lds, (hipStream_t)stream);
  return -2;
}

int occupancy_x20(int taps, int fp32, size_t lds) {
  TDI_DISPATCH(taps, fp32, occ_x20_t, lds);
  return 1;
}

size_t x20_lds_bytes(int cap) { return (size_t)6 * cap * sizeof(double); }

int launch_full(const KParams* dp, int taps, int fp32, int hybrid, int grid, size_t lds, void* stream) {
  TDI_DISPATCH(taps, fp32, launch_full_t, dp, hybrid, grid, lds, (hipStream_t)stream);
  return -2;
}

int launch_links(const KParams* dp, int taps, int fp32, int arm, int64_t grid, size_t lds, void* stream) {
  if (grid <= 0) return 0;
  TDI_DISPATCH(taps, fp32, launch_links_t, dp, arm, grid, lds, (hipStream_t)stream);
  return -2;
}

size_t links_lds_bytes(int cap, int fp32, int windows) {
  const size_t e = fp32 ? 4 : 8;
  return align16((size_t)cap * 2 * e) * (size_t)windows;
}

int occupancy_lfa(int taps, int fp32, int fast, int nx, size_t lds) {
  if (fast) {
    TDI_DISPATCH_FAST(taps, occ_lfa_fast_t, lds);
    return 1;
  }
  TDI_DISPATCH(taps, fp32, occ_lfa_t, nx, lds);
  return 1;
}

int occupancy_full(int taps, int fp32, int hybrid, size_t lds) {
  TDI_DISPATCH(taps, fp32, occ_full_t, hybrid, lds);
  return 1;
}

}  // namespace tdi
