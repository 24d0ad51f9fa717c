/*
 * FP64 CPU oracle of the hybrid time-domain LISA response (arXiv:2505.09600).
 *
 * TEST INFRASTRUCTURE ONLY (see tdi_oracle.h).  Written from the paper's
 * definitions, in their order and notation, for a reader to check by eye:
 *   - source triad and polarisation rotation          Sec. II.A, Eqs. (hplus_ssb, hcross_ssb)
 *   - antenna patterns and link projection            Sec. II.A, Eqs. (H, xi_plus, xi_cross)
 *   - single-link response and propagation delays     Sec. II.B, Eqs. (yslr, delta_s, delta_r)
 *   - Michelson X 1.5 / 2.0, delays evaluated at t    Sec. II.B, Eqs. (X1.5, X2.0)
 *     (optionally time-nested delays)
 *   - low-frequency response (central differences)    Sec. III, Eqs. (yslr_strain_derivatives,
 *                                                     X15_with_strain_derivatives,
 *                                                     X20_with_strain_derivatives);
 *                                                     App. B, Eqs. (X15_nonequal_timedelays,
 *                                                     X20_nonequal_timedelays)
 *   - sigmoid hybrid                                  Sec. IV, Eqs. (sigmoid, hybridized_xs)
 * Readings where the paper is silent or inconsistent are listed in the design doc
 * of the repository; each is restated at its point of use below.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math, no FMA contraction).
 */
#include "tdi_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_C 299792458.0   /* speed of light, m/s */
#define ORC_PI 3.14159265358979323846

static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Links.  Sec. II.B: link l joins sender s and receiver r, |l| is the index of
 * the spacecraft opposite the link and sgn(l) = eps_{s |l| r}.
 * ------------------------------------------------------------------------- */
static int levi_civita(int a, int b, int c) {
  if (a == b || b == c || a == c) return 0;
  if ((a == 1 && b == 2 && c == 3) || (a == 2 && b == 3 && c == 1) || (a == 3 && b == 1 && c == 2))
    return 1;
  return -1;
}

void orc_link_ends(int l, int* s, int* r) {
  int a = l > 0 ? l : -l;
  int o1 = a % 3 + 1, o2 = (a + 1) % 3 + 1;     /* the two spacecraft other than |l| */
  if (levi_civita(o1, a, o2) == (l > 0 ? 1 : -1)) { *s = o1; *r = o2; }
  else { *s = o2; *r = o1; }
}

/* link label -> slot in the 6-arrays: +1,+2,+3,-1,-2,-3 */
static int link_slot(int l) { return l > 0 ? l - 1 : 2 - l; }

/* Cyclic relabelling 1->2->3->1 applied c times (Y: c = 1, Z: c = 2), sign kept. */
static int rotate_link(int l, int c) {
  int a = l > 0 ? l : -l;
  int b = (a - 1 + c) % 3 + 1;
  return l > 0 ? b : -b;
}

/* ---------------------------------------------------------------------------
 * Triad (Sec. II.A).  k = -e_r, u = -e_phi, v = -e_theta with beta = pi/2 - theta
 * and lambda = phi.  The printed components carry two sign slips (k_z and u_y)
 * that contradict both the stated definitions and orthonormality; the
 * definitions are used.
 * ------------------------------------------------------------------------- */
void orc_triad(double beta, double lam, double k[3], double u[3], double v[3]) {
  double cb = cos(beta), sb = sin(beta), cl = cos(lam), sl = sin(lam);
  k[0] = -cb * cl; k[1] = -cb * sl; k[2] = -sb;
  u[0] = sl;       u[1] = -cl;      u[2] = 0.0;
  v[0] = -sb * cl; v[1] = -sb * sl; v[2] = cb;
}

/* ---------------------------------------------------------------------------
 * Orbits.  The paper uses an equal-arm analytic orbit (Sec. II.B) without
 * printing it; the first-order-in-eccentricity analytic form of its cited
 * reference is used: alpha = Omega t + kappa0, beta_i = 2 pi (i-1)/3 + lambda0,
 * e = L / (2 sqrt(3) R).  FROZEN takes the positions at t_freeze.
 * ------------------------------------------------------------------------- */
void orc_positions(const orc_orbit* o, double t, double R[3][3]) {
  if (o->kind == ORC_ORBIT_TABLE) {
    /* Sampled orbit: 8-point Lagrange interpolation in time on the samples
     * around t (the same product-form weights as the fractional delays). */
    double u = (t - o->table_t0) / o->table_dt;
    int64_t i0 = (int64_t)floor(u);
    double x = u - (double)i0, w[8];
    int64_t j0 = i0 - 3;
    if (j0 < 0) { x += (double)j0; j0 = 0; }
    if (j0 > o->n_table - 8) { x += (double)(j0 - (o->n_table - 8)); j0 = o->n_table - 8; }
    orc_lagrange_weights(x, 8, w);
    for (int i = 0; i < 3; ++i)
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int m = 0; m < 8; ++m) acc += w[m] * o->table[9 * (j0 + m) + 3 * i + c];
        R[i][c] = acc;
      }
    return;
  }
  double tt = (o->kind == ORC_ORBIT_FROZEN) ? o->t_freeze : t;
  double e = o->L / (2.0 * sqrt(3.0) * o->R);
  double alpha = o->omega * tt + o->kappa0;
  for (int i = 0; i < 3; ++i) {
    double b = 2.0 * ORC_PI * (double)i / 3.0 + o->lambda0;
    R[i][0] = o->R * cos(alpha) + 0.5 * e * o->R * (cos(2.0 * alpha - b) - 3.0 * cos(b));
    R[i][1] = o->R * sin(alpha) + 0.5 * e * o->R * (sin(2.0 * alpha - b) - 3.0 * sin(b));
    R[i][2] = -sqrt(3.0) * e * o->R * cos(alpha - b);
  }
}

/* Light time T_l(t) = L_l(t)/c: photon received by r at t, emitted by s at
 * t - T; fixed-point iteration T <- |R_r(t) - R_s(t - T)| / c from L/c.
 * FROZEN: equal constant arms, T = L/c. */
double orc_light_time(const orc_orbit* o, int l, double t) {
  if (o->kind == ORC_ORBIT_FROZEN) return o->L / ORC_C;
  int s, r;
  orc_link_ends(l, &s, &r);
  double Rr[3][3], Rs[3][3];
  orc_positions(o, t, Rr);
  double T = o->L / ORC_C;
  for (int it = 0; it < 12; ++it) {
    orc_positions(o, t - T, Rs);
    double d[3] = {Rr[r - 1][0] - Rs[s - 1][0], Rr[r - 1][1] - Rs[s - 1][1],
                   Rr[r - 1][2] - Rs[s - 1][2]};
    double Tn = sqrt(dot3(d, d)) / ORC_C;
    double dT = Tn - T;
    T = Tn;
    if (fabs(dT) <= 4e-15) break;
  }
  return T;
}

/* Geometry at time t (Sec. II.A/B): n_l is the photon direction
 * (R_r(t) - R_s(t - T_l)) / (c T_l); xi+ = (u.n)^2 - (v.n)^2, xi_x = 2 (u.n)(v.n);
 * delta_s = T_l + k.R_s(t)/c, delta_r = k.R_r(t)/c (Eqs. delta_s, delta_r). */
void orc_geometry(const orc_orbit* o, double beta, double lam, double t, orc_geom* g) {
  static const int L6[6] = {1, 2, 3, -1, -2, -3};
  double k[3], u[3], v[3];
  orc_triad(beta, lam, k, u, v);
  orc_positions(o, t, g->R);
  for (int a = 0; a < 6; ++a) {
    int l = L6[a], s, r;
    orc_link_ends(l, &s, &r);
    double T = orc_light_time(o, l, t);
    double Re[3][3];
    orc_positions(o, t - T, Re);
    double nn[3];
    for (int i = 0; i < 3; ++i) nn[i] = (g->R[r - 1][i] - Re[s - 1][i]) / (ORC_C * T);
    double un = dot3(u, nn), vn = dot3(v, nn);
    g->T[a] = T;
    for (int i = 0; i < 3; ++i) g->n[a][i] = nn[i];
    g->xi_p[a] = un * un - vn * vn;
    g->xi_c[a] = 2.0 * un * vn;
    g->kn[a] = dot3(k, nn);
    g->ds[a] = T + dot3(k, g->R[s - 1]) / ORC_C;
    g->dr[a] = dot3(k, g->R[r - 1]) / ORC_C;
    if (a < 3) g->mu[a] = (dot3(k, g->R[s - 1]) + dot3(k, g->R[r - 1])) / (2.0 * ORC_C);
  }
}

/* ---------------------------------------------------------------------------
 * Fractional delay.  A delay d (s) at output sample k is read at grid position
 * k - d/dt = i0 + x with i0 = k - ceil(d/dt), x in [0, 1).  The absolute time
 * t_k - d is never formed.
 * ------------------------------------------------------------------------- */
void orc_split(int64_t k, double d, double dt, int64_t* i0, double* x) {
  double q = d / dt;
  double m = ceil(q);
  *i0 = k - (int64_t)m;
  *x = m - q;
}

/* Lagrange interpolation with N taps (degree N-1) on the nodes
 * j = -N/2+1 .. N/2 around i0: l_j(x) = prod_{m != j} (x - m)/(j - m).
 * Written as a product of ratios so that x = 0 returns s[i0] exactly. */
void orc_lagrange_weights(double x, int N, double* w) {
  int jlo = -N / 2 + 1;
  for (int a = 0; a < N; ++a) {
    int j = jlo + a;
    double p = 1.0;
    for (int b = 0; b < N; ++b) {
      int m = jlo + b;
      if (m == j) continue;
      p *= (x - (double)m) / (double)(j - m);
    }
    w[a] = p;
  }
}

double orc_lagrange(const double* s, int64_t n, int64_t i0, double x, int N) {
  double w[64];
  orc_lagrange_weights(x, N, w);
  int jlo = -N / 2 + 1;
  double acc = 0.0;
  for (int a = 0; a < N; ++a) {
    int64_t i = i0 + jlo + a;
    if (i >= 0 && i < n) acc += w[a] * s[i];   /* zero outside the series */
  }
  return acc;
}

/* ---------------------------------------------------------------------------
 * Central finite-difference stencils of derivative order m and accuracy p
 * (the numerical derivatives of Sec. III).  Coefficients over offsets
 * -h..h, numerator / denominator.
 * ------------------------------------------------------------------------- */
static int stencil_coeffs(int m, int p, double* num, double* den) {
  /* orders 4 and 5: the strain derivatives of the next LFA term */
  if (m == 4 && p == 2) { double c[] = {1, -4, 6, -4, 1}; memcpy(num, c, sizeof c); *den = 1; return 2; }
  if (m == 4 && p == 4) { double c[] = {-1, 12, -39, 56, -39, 12, -1}; memcpy(num, c, sizeof c); *den = 6; return 3; }
  if (m == 5 && p == 2) { double c[] = {-1, 4, -5, 0, 5, -4, 1}; memcpy(num, c, sizeof c); *den = 2; return 3; }
  if (m == 5 && p == 4) { double c[] = {1, -9, 26, -29, 0, 29, -26, 9, -1}; memcpy(num, c, sizeof c); *den = 6; return 4; }
  if (m == 1 && p == 2) { double c[] = {-1, 0, 1}; memcpy(num, c, sizeof c); *den = 2; return 1; }
  if (m == 1 && p == 4) { double c[] = {1, -8, 0, 8, -1}; memcpy(num, c, sizeof c); *den = 12; return 2; }
  if (m == 2 && p == 2) { double c[] = {1, -2, 1}; memcpy(num, c, sizeof c); *den = 1; return 1; }
  if (m == 2 && p == 4) { double c[] = {-1, 16, -30, 16, -1}; memcpy(num, c, sizeof c); *den = 12; return 2; }
  if (m == 3 && p == 2) { double c[] = {-1, 2, 0, -2, 1}; memcpy(num, c, sizeof c); *den = 2; return 2; }
  if (m == 3 && p == 4) { double c[] = {1, -8, 13, 0, -13, 8, -1}; memcpy(num, c, sizeof c); *den = 8; return 3; }
  return -1;
}

static double stencil_at(const double* h, int64_t n, int64_t i, const double* num, int hw, double scale) {
  double acc = 0.0;
  for (int s = -hw; s <= hw; ++s) {
    int64_t j = i + s;
    if (j >= 0 && j < n) acc += num[s + hw] * h[j];
  }
  return acc / scale;
}

void orc_stencil(const double* h, int64_t n, int m, int p, double dt, double* g) {
  double num[9], den;
  int hw = stencil_coeffs(m, p, num, &den);
  if (hw < 0) { for (int64_t i = 0; i < n; ++i) g[i] = NAN; return; }
  double scale = den * pow(dt, (double)m);
  for (int64_t i = 0; i < n; ++i) g[i] = stencil_at(h, n, i, num, hw, scale);
}

/* ---------------------------------------------------------------------------
 * TDI term lists, transcribed from Eqs. (X1.5) and (X2.0): each term is
 * sign * y_link(t - sum of the listed delays), with every L evaluated at t.
 * Links: y_{1-32} is l = -3, y_{231} is l = +3, y_{123} is l = +2,
 * y_{3-21} is l = -2.  Y and Z follow by cyclic relabelling.
 * ------------------------------------------------------------------------- */
typedef struct { int sign, link, nd, d[7]; } orc_term;

static const orc_term X15_TERMS[8] = {
    {+1, -3, 3, {-2, +2, +3}},
    {-1, -3, 1, {+3}},
    {+1, +3, 2, {+2, -2}},
    {-1, +3, 0, {0}},
    {+1, +2, 1, {-2}},
    {-1, +2, 3, {-2, -3, +3}},
    {+1, -2, 0, {0}},
    {-1, -2, 2, {-3, +3}},
};

static const orc_term X20_EXTRA_TERMS[8] = {
    {+1, -3, 5, {-2, +2, +3, +3, -3}},
    {-1, -3, 7, {+3, +3, -3, -2, -2, +2, +2}},
    {+1, +3, 4, {-2, +2, +3, -3}},
    {-1, +3, 6, {+3, -3, -2, -2, +2, +2}},
    {+1, +2, 7, {-2, -2, +2, +3, +3, -3, -3}},
    {-1, +2, 5, {+3, -3, -2, -2, +2}},
    {+1, -2, 6, {-2, +2, +3, +3, -3, -3}},
    {-1, -2, 4, {+3, -3, -2, +2}},
};

static int n_terms(int gen) { return gen == 20 ? 16 : 8; }
static const orc_term* term_at(int t) { return t < 8 ? &X15_TERMS[t] : &X20_EXTRA_TERMS[t - 8]; }

/* ---------------------------------------------------------------------------
 * The same combinations with time-nested delays (an option: the paper takes
 * every delay at t, Sec. II.B, text after Eq. X2.0).  A delay operator shifts
 * by the light time of its link at the time it is applied,
 *   D_l f(t) = f(t - T_l(t)),   D_a D_b f(t) = f(t - T_a(t) - T_b(t - T_a(t))),
 * so the leftmost factor is taken at the output time.  With the two round
 * trips from spacecraft 1,
 *   A = D_{+3} D_{-3}  (out along 1->2, back along 2->1, which arrives at t),
 *   B = D_{-2} D_{+2}  (out along 1->3, back along 3->1),
 * and the two one-arm signals received at spacecraft 1,
 *   eta2 = y_{231} + D_{+3} y_{1-32},   eta3 = y_{3-21} + D_{-2} y_{123},
 * Eq. (X1.5) is (B - 1) eta2 - (A - 1) eta3 and Eq. (X2.0) adds
 * (B A - A B B) eta2 + (B A A - A B) eta3.  Expanded, every product carries the
 * delays of one printed term above, in a definite order.
 * ------------------------------------------------------------------------- */
typedef struct { int sign; const char* word; int eta; } orc_word;

static const orc_word NESTED_WORDS[8] = {
    {+1, "B", 2}, {-1, "", 2}, {+1, "", 3}, {-1, "A", 3},            /* X1.5 */
    {+1, "BA", 2}, {-1, "ABB", 2}, {+1, "BAA", 3}, {-1, "AB", 3},     /* added by X2.0 */
};

void orc_nested_term(int t, int* sign, int* link, int* nd, int d[8]) {
  const orc_word* w = &NESTED_WORDS[t / 2];
  int n = 0;
  for (const char* ch = w->word; *ch; ++ch) {
    if (*ch == 'A') { d[n++] = +3; d[n++] = -3; }
    else            { d[n++] = -2; d[n++] = +2; }
  }
  /* even t: the link received at spacecraft 1; odd t: the far link, reached
   * through one more leg into spacecraft 1, applied last */
  const int near = w->eta == 2 ? +3 : -2, far = w->eta == 2 ? -3 : +2;
  if (t % 2 == 0) {
    *link = near;
  } else {
    *link = far;
    d[n++] = near;
  }
  *sign = w->sign;
  *nd = n;
}

/* ---------------------------------------------------------------------------
 * Evaluation context: h_SSB, lazily filled link series y and LFA derivative
 * series g (each entry computed at most once).
 * ------------------------------------------------------------------------- */
typedef struct {
  const orc_config* c;
  const orc_orbit* o;
  const orc_source* s;
  int64_t n;
  double* hp_ssb;
  double* hc_ssb;
  double* y;          /* 6 * n */
  unsigned char* y_ok;
  double* gp;
  double* gc;
  unsigned char* g_ok;
  int m;              /* LFA derivative order */
  void* nt;           /* LFA with the next term: context of derivative order m + 2 */
  void* sc;           /* TDI 2.0 LFA from TDI 1.5: the shortcut's series (orc_x20) */
} orc_ctx;

static void ctx_init(orc_ctx* x, const orc_config* c, const orc_orbit* o, const orc_source* s,
                     int64_t n, const double* hp, const double* hc) {
  x->c = c; x->o = o; x->s = s; x->n = n;
  x->hp_ssb = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  x->hc_ssb = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  /* Eqs. (hplus_ssb, hcross_ssb): rotation by the polarisation angle. */
  double c2 = cos(2.0 * s->psi), s2 = sin(2.0 * s->psi);
  for (int64_t i = 0; i < n; ++i) {
    x->hp_ssb[i] = hp[i] * c2 - hc[i] * s2;
    x->hc_ssb[i] = hp[i] * s2 + hc[i] * c2;
  }
  x->y = NULL; x->y_ok = NULL; x->gp = NULL; x->gc = NULL; x->g_ok = NULL;
  x->m = (c->tdi_gen == 20) ? 3 : 2;
  x->nt = NULL;
  x->sc = NULL;
}

static void sc_free(void* p);

static void ctx_free(orc_ctx* x) {
  free(x->hp_ssb); free(x->hc_ssb); free(x->y); free(x->y_ok);
  free(x->gp); free(x->gc); free(x->g_ok);
  if (x->nt) { ctx_free((orc_ctx*)x->nt); free(x->nt); }
  if (x->sc) sc_free(x->sc);
}

/* X, Y, Z LFA with the next term (lfa_terms = 2): a second context holding the
 * derivative series of order m + 2 of the same source. */
static void ctx_next_term(orc_ctx* x, int64_t n, const double* hp, const double* hc) {
  if (x->c->lfa_terms != 2 || x->c->mode == ORC_FULL) return;
  orc_ctx* t = (orc_ctx*)malloc(sizeof(orc_ctx));
  ctx_init(t, x->c, x->o, x->s, n, hp, hc);
  t->m = x->m + 2;
  x->nt = t;
}

static double t_of(const orc_ctx* x, int64_t k) { return x->s->t0 + (double)k * x->s->dt; }

/* Stage 1 at grid sample i, Eq. (yslr) with Eq. (H): for each link,
 * y = [H_l(t - delta_s) - H_l(t - delta_r)] / (2 (1 - k.n)), where H_l at a
 * retarded time uses the antenna patterns at the reception time t_i and the
 * N-tap Lagrange value of h_SSB. */
static void stage1_at(orc_ctx* x, int64_t i, double y6[6]) {
  orc_geom g;
  orc_geometry(x->o, x->s->beta, x->s->lam, t_of(x, i), &g);
  int N = x->c->taps;
  double dt = x->s->dt;
  for (int a = 0; a < 6; ++a) {
    int64_t i0; double fx;
    orc_split(i, g.ds[a], dt, &i0, &fx);
    double Hs = g.xi_p[a] * orc_lagrange(x->hp_ssb, x->n, i0, fx, N) +
                g.xi_c[a] * orc_lagrange(x->hc_ssb, x->n, i0, fx, N);
    orc_split(i, g.dr[a], dt, &i0, &fx);
    double Hr = g.xi_p[a] * orc_lagrange(x->hp_ssb, x->n, i0, fx, N) +
                g.xi_c[a] * orc_lagrange(x->hc_ssb, x->n, i0, fx, N);
    y6[a] = (Hs - Hr) / (2.0 * (1.0 - g.kn[a]));
  }
}

static void ensure_y_alloc(orc_ctx* x) {
  if (x->y) return;
  size_t n = (size_t)(x->n > 0 ? x->n : 1);
  x->y = (double*)malloc(sizeof(double) * 6 * n);
  x->y_ok = (unsigned char*)calloc(n, 1);
}

static void ensure_y_range(orc_ctx* x, int64_t lo, int64_t hi) {
  ensure_y_alloc(x);
  if (lo < 0) lo = 0;
  if (hi > x->n) hi = x->n;
  for (int64_t i = lo; i < hi; ++i) {
    if (x->y_ok[i]) continue;
    double y6[6];
    stage1_at(x, i, y6);
    for (int a = 0; a < 6; ++a) x->y[(size_t)a * x->n + i] = y6[a];
    x->y_ok[i] = 1;
  }
}

static int in_parallel(void) {
#ifdef _OPENMP
  return omp_in_parallel();
#else
  return 1;
#endif
}

/* Fill y for every grid index >= lo (in parallel when not nested). */
static void fill_y_from(orc_ctx* x, int64_t lo) {
  ensure_y_alloc(x);
  int64_t n = x->n;
  if (lo < 0) lo = 0;
#pragma omp parallel for schedule(static) if (n - lo > 4096 && !in_parallel())
  for (int64_t i = lo; i < n; ++i) {
    if (x->y_ok[i]) continue;
    double y6[6];
    stage1_at(x, i, y6);
    for (int a = 0; a < 6; ++a) x->y[(size_t)a * n + i] = y6[a];
    x->y_ok[i] = 1;
  }
}

static double lagrange_y(orc_ctx* x, int slot, int64_t i0, double fx) {
  int N = x->c->taps;
  ensure_y_range(x, i0 - N / 2 + 1, i0 + N / 2 + 1);
  return orc_lagrange(x->y + (size_t)slot * x->n, x->n, i0, fx, N);
}

/* Term t of channel c at output sample k: sign, link of y and total delay.
 * Delays at t_k (the paper's choice): the light times of the term are summed.
 * Time-nested: each light time is taken at t_k less the delays applied before
 * it.  The retarded time is formed in absolute time only as the argument of
 * the slowly varying light time; the split uses the delay alone. */
static void term_delay(const orc_ctx* x, const orc_geom* g, int c, int t, int64_t k,
                       int* sign, int* link, double* d) {
  double acc = 0.0;
  if (x->c->nested_delays) {
    int nd, dl[8];
    orc_nested_term(t, sign, link, &nd, dl);
    for (int q = 0; q < nd; ++q) acc += orc_light_time(x->o, rotate_link(dl[q], c), t_of(x, k) - acc);
  } else {
    const orc_term* tm = term_at(t);
    for (int q = 0; q < tm->nd; ++q) acc += g->T[link_slot(rotate_link(tm->d[q], c))];
    *sign = tm->sign;
    *link = tm->link;
  }
  *link = rotate_link(*link, c);
  *d = acc;
}

/* Stage 2 at output sample k, Eqs. (X1.5)/(X2.0): all delays L_l -> c T_l(t_k)
 * (or time-nested, above); a term's delays are summed first, then split.  If
 * absterms is non-null the sum of |term| per channel is returned there too. */
static void full_at(orc_ctx* x, int64_t k, double out[3], double* absterms) {
  orc_geom g;
  orc_geometry(x->o, x->s->beta, x->s->lam, t_of(x, k), &g);
  for (int c = 0; c < 3; ++c) {
    double acc = 0.0, aabs = 0.0;
    for (int t = 0; t < n_terms(x->c->tdi_gen); ++t) {
      int sign, link;
      double d;
      term_delay(x, &g, c, t, k, &sign, &link, &d);
      int64_t i0; double fx;
      orc_split(k, d, x->s->dt, &i0, &fx);
      double v = lagrange_y(x, link_slot(link), i0, fx);
      acc += (double)sign * v;
      aabs += fabs(v);
    }
    out[c] = acc;
    if (absterms) absterms[c] = aabs;
  }
}

/* LFA derivative series g_m = D^(m)_p [h_SSB] on the grid, zero outside. */
static void ensure_g_alloc(orc_ctx* x) {
  if (x->gp) return;
  size_t n = (size_t)(x->n > 0 ? x->n : 1);
  x->gp = (double*)malloc(sizeof(double) * n);
  x->gc = (double*)malloc(sizeof(double) * n);
  x->g_ok = (unsigned char*)calloc(n, 1);
}

static void ensure_g_range(orc_ctx* x, int64_t lo, int64_t hi) {
  ensure_g_alloc(x);
  if (lo < 0) lo = 0;
  if (hi > x->n) hi = x->n;
  double num[9], den;
  int hw = stencil_coeffs(x->m, x->c->stencil_order, num, &den);
  double scale = den * pow(x->s->dt, (double)x->m);
  for (int64_t i = lo; i < hi; ++i) {
    if (x->g_ok[i]) continue;
    x->gp[i] = stencil_at(x->hp_ssb, x->n, i, num, hw, scale);
    x->gc[i] = stencil_at(x->hc_ssb, x->n, i, num, hw, scale);
    x->g_ok[i] = 1;
  }
}

static void fill_g_all(orc_ctx* x) {
  ensure_g_alloc(x);
  ensure_g_range(x, 0, x->n);
}

/* Xi_l(k; d) = xi+_l(t_k) I_N[g+](k - d/dt) + xi_x_l(t_k) I_N[g_x](k - d/dt). */
static double Xi(orc_ctx* x, const orc_geom* g, int l, int64_t k, double d) {
  int N = x->c->taps;
  int64_t i0; double fx;
  orc_split(k, d, x->s->dt, &i0, &fx);
  ensure_g_range(x, i0 - N / 2 + 1, i0 + N / 2 + 1);
  int a = link_slot(l);
  return g->xi_p[a] * orc_lagrange(x->gp, x->n, i0, fx, N) +
         g->xi_c[a] * orc_lagrange(x->gc, x->n, i0, fx, N);
}

/* LFA at output sample k.  The single-link LFA of Eq. (yslr_strain_derivatives),
 * y_l(t) = -(T_l/2) [xi+ h+'(t - T_l/2 - mu_l) + xi_x hx'(...)], with
 * mu_l = k.(R_s + R_r)/(2c), substituted into Eqs. (X15_nonequal_timedelays)
 * and (X20_nonequal_timedelays) (T_i = L_i/c, positive-index links, geometry at
 * t_k, derivatives of the delays and antenna patterns dropped as in App. B):
 *   X1.5 = -2 T2 T3        [Xi_2^(2)(k; T2+T3+mu_2)     - Xi_3^(2)(k; T2+T3+mu_3)]
 *   X2.0 = -4 T2 T3 (T2+T3) [Xi_2^(3)(k; 2(T2+T3)+mu_2) - Xi_3^(3)(k; 2(T2+T3)+mu_3)]
 * where Xi^(m) interpolates the m-th strain derivative taken on the grid by a
 * central stencil (derivative first, then fractional delay).  Equal arms set
 * every T_i to L/c.  Y, Z: links (2,3) -> (3,1) -> (1,2). */
/* Next term (lfa_terms = 2), from the same central expansion carried one order
 * further.  Expanding the eight terms of Eqs. (X1.5l2), (X1.5l3) about their
 * group centres to third order in the delays, with the two-term link series of
 * Eq. (yslr_with_tau_derivatives) and the link-reversal symmetry of the delays
 * used for Eq. (X15_nonequal_timedelays), gives for the link-2 group of X
 *   -2 T2 T3 [Xi_2^(2) + kappa_2 Xi_2^(4)](k; T2+T3+mu_2),
 *   kappa_2 = T3^2/6 + T2^2/8 + T2^2 (1 + (k.n_2)^2)/24:
 * T3^2/6 + T2^2/8 from the third-order terms of the TDI combination, the last
 * term the m = 1 link term [T2 (1 -+ k.n_2)/2]^2/6 averaged over the two
 * directions of arm 2.  TDI 2.0 follows from X2.0(t) = X1.5(t) - X1.5(t - D),
 * D = 2(T2+T3) (constant link-symmetric delays), expanded about t - D/2 to
 * third order: the same form with m = 3 and kappa + (T2+T3)^2/6.  The link-3
 * group exchanges T2 and T3.  What remains is third order in 2 pi f L/c and
 * proportional to k.n (the link asymmetry of the m = 1 terms), fourth order
 * when k.n vanishes on both arms. */
static double lfa_kappa(int gen, double Tl, double To, double kn) {
  double kap = To * To / 6.0 + Tl * Tl / 8.0 + Tl * Tl * (1.0 + kn * kn) / 24.0;
  if (gen == 20) kap += (Tl + To) * (Tl + To) / 6.0;
  return kap;
}

static void lfa_at(orc_ctx* x, int64_t k, double out[3]) {
  orc_geom g;
  orc_geometry(x->o, x->s->beta, x->s->lam, t_of(x, k), &g);
  orc_ctx* nt = (orc_ctx*)x->nt;
  for (int c = 0; c < 3; ++c) {
    int la = (c + 1) % 3 + 1, lb = (c + 2) % 3 + 1;
    double Ta = x->c->equal_arms ? x->o->L / ORC_C : g.T[la - 1];
    double Tb = x->c->equal_arms ? x->o->L / ORC_C : g.T[lb - 1];
    double pref, d;
    if (x->c->tdi_gen == 20) { pref = -4.0 * Ta * Tb * (Ta + Tb); d = 2.0 * (Ta + Tb); }
    else { pref = -2.0 * Ta * Tb; d = Ta + Tb; }
    double va = Xi(x, &g, la, k, d + g.mu[la - 1]);
    double vb = Xi(x, &g, lb, k, d + g.mu[lb - 1]);
    if (nt) {
      va += lfa_kappa(x->c->tdi_gen, Ta, Tb, g.kn[la - 1]) * Xi(nt, &g, la, k, d + g.mu[la - 1]);
      vb += lfa_kappa(x->c->tdi_gen, Tb, Ta, g.kn[lb - 1]) * Xi(nt, &g, lb, k, d + g.mu[lb - 1]);
    }
    out[c] = pref * (va - vb);
  }
}

/* TDI 2.0 LFA from the TDI 1.5 LFA, Eq. (relation_X20_X15_nonequal_timedelays):
 *   X2.0(t) = 2 (T2 + T3) dX1.5/dt (t - T2 - T3),
 * in the stencil-first form used throughout: X1.5 is the LFA TDI 1.5 series on
 * the grid (zero outside [0, n-1]), its first derivative is taken there by the
 * central stencil of accuracy p, and that series is read at the fractional
 * delay T2 + T3 by N-tap Lagrange, the light times at the output time (equal
 * arms: 4L/c and 2L/c, Eq. relation_X20_X15_equal_timedelays).  Y, Z cyclic. */
typedef struct {
  orc_config c15;     /* the same configuration at TDI 1.5, LFA */
  orc_ctx x15;        /* its context (derivative order 2) */
  double* v;          /* X1.5, Y1.5, Z1.5 on the grid, 3 n */
  double* d;          /* their first derivatives, 3 n */
  unsigned char* v_ok;
  unsigned char* d_ok;
  int absmode;        /* rounding-scale evaluation: magnitudes throughout */
} orc_x20;

static void abs_lfa_at(orc_ctx* x, int64_t k, double out[3]);
static double lagrange_abs(const double* s, int64_t n, int64_t i0, double x, int N);

static void sc_free(void* p) {
  orc_x20* s = (orc_x20*)p;
  ctx_free(&s->x15);
  free(s->v); free(s->d); free(s->v_ok); free(s->d_ok);
  free(s);
}

static void ctx_shortcut(orc_ctx* x, int64_t n, const double* hp, const double* hc) {
  if (!x->c->x20_from_x15 || x->c->tdi_gen != 20 || x->c->mode == ORC_FULL) return;
  orc_x20* s = (orc_x20*)calloc(1, sizeof(orc_x20));
  s->c15 = *x->c;
  s->c15.tdi_gen = 15;
  s->c15.mode = ORC_LFA;
  s->c15.x20_from_x15 = 0;
  ctx_init(&s->x15, &s->c15, x->o, x->s, n, hp, hc);
  size_t m = (size_t)(n > 0 ? n : 1);
  s->v = (double*)malloc(sizeof(double) * 3 * m);
  s->d = (double*)malloc(sizeof(double) * 3 * m);
  s->v_ok = (unsigned char*)calloc(m, 1);
  s->d_ok = (unsigned char*)calloc(m, 1);
  x->sc = s;
}

static void sc_ensure_v(orc_x20* s, int64_t n, int64_t lo, int64_t hi) {
  if (lo < 0) lo = 0;
  if (hi > n) hi = n;
  for (int64_t i = lo; i < hi; ++i) {
    if (s->v_ok[i]) continue;
    double r[3];
    if (s->absmode) abs_lfa_at(&s->x15, i, r);
    else lfa_at(&s->x15, i, r);
    for (int c = 0; c < 3; ++c) s->v[(size_t)c * n + i] = r[c];
    s->v_ok[i] = 1;
  }
}

static void sc_ensure_d(orc_x20* s, int64_t n, double dt, int p, int64_t lo, int64_t hi) {
  double num[9], den;
  int hw = stencil_coeffs(1, p, num, &den);
  if (s->absmode)
    for (int q = 0; q < 2 * hw + 1; ++q) num[q] = fabs(num[q]);
  if (lo < 0) lo = 0;
  if (hi > n) hi = n;
  for (int64_t i = lo; i < hi; ++i) {
    if (s->d_ok[i]) continue;
    sc_ensure_v(s, n, i - hw, i + hw + 1);
    for (int c = 0; c < 3; ++c) s->d[(size_t)c * n + i] = stencil_at(s->v + (size_t)c * n, n, i, num, hw, den * dt);
    s->d_ok[i] = 1;
  }
}

static void x20_at(orc_ctx* x, int64_t k, double out[3]) {
  orc_x20* s = (orc_x20*)x->sc;
  orc_geom g;
  orc_geometry(x->o, x->s->beta, x->s->lam, t_of(x, k), &g);
  int N = x->c->taps;
  for (int c = 0; c < 3; ++c) {
    int la = (c + 1) % 3 + 1, lb = (c + 2) % 3 + 1;
    double Ta = x->c->equal_arms ? x->o->L / ORC_C : g.T[la - 1];
    double Tb = x->c->equal_arms ? x->o->L / ORC_C : g.T[lb - 1];
    int64_t i0; double fx;
    orc_split(k, Ta + Tb, x->s->dt, &i0, &fx);
    sc_ensure_d(s, x->n, x->s->dt, x->c->stencil_order, i0 - N / 2 + 1, i0 + N / 2 + 1);
    const double* dc = s->d + (size_t)c * x->n;
    out[c] = 2.0 * (Ta + Tb) * (s->absmode ? lagrange_abs(dc, x->n, i0, fx, N) : orc_lagrange(dc, x->n, i0, fx, N));
  }
}

static void lfa_out(orc_ctx* x, int64_t k, double out[3]) {
  if (x->sc) x20_at(x, k, out);
  else lfa_at(x, k, out);
}

/* Hybrid weights and windows, Eqs. (sigmoid, hybridized_xs), in sample units:
 * z = (k - k_H)/sigma, w+ = 1/(1+e^z), w- = 1/(1+e^-z); LFA part where
 * k - k_H <= T/2, full part where k - k_H >= -T/2 (both inclusive, weights
 * applied everywhere).  k_H = (t_Hyb - t0)/dt. */
static void output_at(orc_ctx* x, int64_t k, double out[3]) {
  int mode = x->c->mode;
  if (mode == ORC_FULL) { full_at(x, k, out, NULL); return; }
  if (mode == ORC_LFA) { lfa_out(x, k, out); return; }
  double kH = (x->s->t_hyb - x->s->t0) / x->s->dt;
  double rel = (double)k - kH;
  double z = rel / x->c->sigma_samples;
  double wp = 1.0 / (1.0 + exp(z));
  double wm = 1.0 / (1.0 + exp(-z));
  double r[3] = {0.0, 0.0, 0.0};
  if (rel <= 0.5 * x->c->T_samples) {
    double a[3];
    lfa_out(x, k, a);
    for (int c = 0; c < 3; ++c) r[c] += wp * a[c];
  }
  if (rel >= -0.5 * x->c->T_samples) {
    double b[3];
    full_at(x, k, b, NULL);
    for (int c = 0; c < 3; ++c) r[c] += wm * b[c];
  }
  for (int c = 0; c < 3; ++c) out[c] = r[c];
}

/* First grid index of y that the full part can read, or n if none: the full
 * part starts at k_H - T/2 and a TDI 2.0 term reaches back at most seven arm
 * light times (bounded generously by ten L/c) plus N/2 taps. */
static int64_t first_y_needed(const orc_ctx* x) {
  if (x->c->mode == ORC_FULL) return 0;
  if (x->c->mode == ORC_LFA) return x->n;
  double kH = (x->s->t_hyb - x->s->t0) / x->s->dt;
  double k0 = kH - 0.5 * x->c->T_samples;
  if (!(k0 <= (double)(x->n - 1))) return x->n;       /* also catches NaN */
  if (k0 < 0.0) return 0;
  double back = 10.0 * x->o->L / ORC_C / x->s->dt + x->c->taps / 2 + 2;
  double lo = floor(k0 - back);
  return lo < 0.0 ? 0 : (int64_t)lo;
}

/* Single-link LFA at output sample k, Eq. (yslr_strain_derivatives) for each
 * link: y_l(t_k) = -(T_l/2) [xi+_l(t_k) h+'(t_k - T_l/2 - mu_l) +
 * xi_x_l(t_k) hx'(...)], T_l = L_l(t_k)/c (L/c for equal arms),
 * mu_l = k.(R_s + R_r)/(2c) (the same for l and -l), h' the first derivative
 * of h_SSB by the central stencil of accuracy p on the grid (the context's
 * derivative order must be 1), read at the retarded time by N-tap Lagrange. */
static void lfa_links_at(orc_ctx* x, orc_ctx* x3, int64_t k, double y6[6]) {
  static const int L6[6] = {1, 2, 3, -1, -2, -3};
  orc_geom g;
  orc_geometry(x->o, x->s->beta, x->s->lam, t_of(x, k), &g);
  for (int a = 0; a < 6; ++a) {
    int l = L6[a];
    double T = x->c->equal_arms ? x->o->L / ORC_C : g.T[a];
    double mu = g.mu[(l > 0 ? l : -l) - 1];
    double v = Xi(x, &g, l, k, 0.5 * T + mu);
    /* Next term of Eq. (yslr_with_tau_derivatives), m = 1: (1/3!) times
     * [L (1 - k.n) / (2c)]^2 times the third derivative of H, the
     * tau-derivatives taken as t-derivatives as in the leading term. */
    if (x3) {
      double e = 0.5 * T * (1.0 - g.kn[a]);
      v += e * e / 6.0 * Xi(x3, &g, l, k, 0.5 * T + mu);
    }
    y6[a] = -0.5 * T * v;
  }
}

/* ---------------------------------------------------------------------------
 * Public entry points.
 * ------------------------------------------------------------------------- */
void orc_link_outputs(const orc_config* c, const orc_orbit* o, const orc_source* s,
                      int64_t n, const double* hp, const double* hc, double* y) {
  orc_ctx x, x3;
  ctx_init(&x, c, o, s, n, hp, hc);
  x.m = 1;
  int nlo = c->lfa_terms == 2 && c->mode != ORC_FULL;
  if (nlo) { ctx_init(&x3, c, o, s, n, hp, hc); x3.m = 3; fill_g_all(&x3); }
  if (c->mode != ORC_FULL) fill_g_all(&x);      /* read-only below: safe across threads */
  double kH = (s->t_hyb - s->t0) / s->dt;
  #pragma omp parallel for schedule(dynamic, 256) if (!in_parallel())
  for (int64_t k = 0; k < n; ++k) {
    double r[6] = {0, 0, 0, 0, 0, 0}, a6[6];
    double rel = (double)k - kH, z = rel / c->sigma_samples;
    int lfa = c->mode == ORC_LFA || (c->mode == ORC_HYBRID && rel <= 0.5 * c->T_samples);
    int full = c->mode == ORC_FULL || (c->mode == ORC_HYBRID && rel >= -0.5 * c->T_samples);
    double wp = c->mode == ORC_HYBRID ? 1.0 / (1.0 + exp(z)) : 1.0;
    double wm = c->mode == ORC_HYBRID ? 1.0 / (1.0 + exp(-z)) : 1.0;
    if (lfa) { lfa_links_at(&x, nlo ? &x3 : NULL, k, a6); for (int a = 0; a < 6; ++a) r[a] += wp * a6[a]; }
    if (full) { stage1_at(&x, k, a6); for (int a = 0; a < 6; ++a) r[a] += wm * a6[a]; }
    for (int a = 0; a < 6; ++a) y[(size_t)a * (size_t)n + (size_t)k] = r[a];
  }
  if (nlo) ctx_free(&x3);
  ctx_free(&x);
}

void orc_links(const orc_config* c, const orc_orbit* o, const orc_source* s,
               int64_t n, const double* hp, const double* hc, double* y) {
  orc_ctx x;
  ctx_init(&x, c, o, s, n, hp, hc);
  fill_y_from(&x, 0);
  memcpy(y, x.y, sizeof(double) * 6 * (size_t)n);
  ctx_free(&x);
}

void orc_tdi_combine(int gen, int N, int64_t n, double dt, const double* y,
                     const double* T, double* X, double* Y, double* Z) {
  double* outs[3] = {X, Y, Z};
#pragma omp parallel for schedule(static) if (n > 4096 && !in_parallel())
  for (int64_t k = 0; k < n; ++k) {
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int t = 0; t < n_terms(gen); ++t) {
        const orc_term* tm = term_at(t);
        double d = 0.0;
        for (int q = 0; q < tm->nd; ++q) d += T[(size_t)link_slot(rotate_link(tm->d[q], c)) * n + k];
        int64_t i0; double fx;
        orc_split(k, d, dt, &i0, &fx);
        acc += (double)tm->sign *
               orc_lagrange(y + (size_t)link_slot(rotate_link(tm->link, c)) * n, n, i0, fx, N);
      }
      outs[c][k] = acc;
    }
  }
}

void orc_tdi_combine_nested(int gen, int N, int64_t n, double dt, const double* y,
                            const double* T, double* X, double* Y, double* Z) {
  double* outs[3] = {X, Y, Z};
#pragma omp parallel for schedule(static) if (n > 4096 && !in_parallel())
  for (int64_t k = 0; k < n; ++k) {
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int t = 0; t < n_terms(gen); ++t) {
        int sign, link, nd, dl[8];
        orc_nested_term(t, &sign, &link, &nd, dl);
        double d = 0.0;
        for (int q = 0; q < nd; ++q) {
          int64_t j0; double fj;
          orc_split(k, d, dt, &j0, &fj);
          d += orc_lagrange(T + (size_t)link_slot(rotate_link(dl[q], c)) * n, n, j0, fj, N);
        }
        int64_t i0; double fx;
        orc_split(k, d, dt, &i0, &fx);
        acc += (double)sign * orc_lagrange(y + (size_t)link_slot(rotate_link(link, c)) * n, n, i0, fx, N);
      }
      outs[c][k] = acc;
    }
  }
}

void orc_response(const orc_config* c, const orc_orbit* o, const orc_source* s,
                  int64_t n, const double* hp, const double* hc,
                  double* X, double* Y, double* Z) {
  if (n <= 0) return;
  orc_ctx x;
  ctx_init(&x, c, o, s, n, hp, hc);
  ctx_next_term(&x, n, hp, hc);
  ctx_shortcut(&x, n, hp, hc);
  int64_t ylo = first_y_needed(&x);
  if (ylo < n) fill_y_from(&x, ylo);
  if (c->mode != ORC_FULL) fill_g_all(&x);
  if (x.nt) fill_g_all((orc_ctx*)x.nt);
  if (x.sc) {
    /* every X1.5 sample, then its derivative, before the parallel reads */
    orc_x20* sc = (orc_x20*)x.sc;
    fill_g_all(&sc->x15);
#pragma omp parallel for schedule(static) if (n > 4096 && !in_parallel())
    for (int64_t i = 0; i < n; ++i) sc_ensure_v(sc, n, i, i + 1);
    sc_ensure_d(sc, n, s->dt, c->stencil_order, 0, n);
  }
#pragma omp parallel for schedule(static) if (n > 4096 && !in_parallel())
  for (int64_t k = 0; k < n; ++k) {
    double r[3];
    output_at(&x, k, r);
    X[k] = r[0]; Y[k] = r[1]; Z[k] = r[2];
  }
  ctx_free(&x);
}

void orc_response_at(const orc_config* c, const orc_orbit* o, const orc_source* s,
                     int64_t n, const double* hp, const double* hc,
                     int64_t nk, const int64_t* ks, double* X, double* Y, double* Z) {
  orc_ctx x;
  ctx_init(&x, c, o, s, n, hp, hc);
  ctx_next_term(&x, n, hp, hc);
  ctx_shortcut(&x, n, hp, hc);
  for (int64_t q = 0; q < nk; ++q) {
    double r[3];
    output_at(&x, ks[q], r);
    X[q] = r[0]; Y[q] = r[1]; Z[q] = r[2];
  }
  ctx_free(&x);
}

void orc_response_batch(const orc_config* c, const orc_orbit* o, int64_t n_sources,
                        const orc_source* src, const int64_t* offsets,
                        const double* hp, const double* hc,
                        double* X, double* Y, double* Z) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n_sources; ++i) {
    int64_t a = offsets[i], b = offsets[i + 1];
    orc_response(c, o, &src[i], b - a, hp + a, hc + a, X + a, Y + a, Z + a);
  }
}

void orc_full_terms_absmax(const orc_config* c, const orc_orbit* o, const orc_source* s,
                           int64_t n, const double* hp, const double* hc, double* absmax3) {
  orc_ctx x;
  ctx_init(&x, c, o, s, n, hp, hc);
  fill_y_from(&x, 0);
  absmax3[0] = absmax3[1] = absmax3[2] = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    double r[3], a[3];
    full_at(&x, k, r, a);
    for (int q = 0; q < 3; ++q) if (a[q] > absmax3[q]) absmax3[q] = a[q];
  }
  ctx_free(&x);
}

void orc_response_batch_at(const orc_config* c, const orc_orbit* o, int64_t n_sources,
                           const orc_source* src, const int64_t* offsets, const double* hp,
                           const double* hc, const int64_t* k_offsets, const int64_t* ks,
                           double* X, double* Y, double* Z) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n_sources; ++i) {
    int64_t a = offsets[i], b = offsets[i + 1];
    int64_t ka = k_offsets[i], kb = k_offsets[i + 1];
    orc_response_at(c, o, &src[i], b - a, hp + a, hc + a, kb - ka, ks + ka, X + ka, Y + ka, Z + ka);
  }
}

/* ===========================================================================
 * Rounding-error scale for FP64 comparisons (not part of the method).
 *
 * A_c(k) is the response evaluated with every input sample, interpolation
 * weight, stencil coefficient, antenna pattern and prefactor replaced by its
 * absolute value and every difference by a sum.  Any evaluation order of the
 * response in FP64 differs from the exact value by at most a modest multiple
 * of 2^-53 A_c(k) (the number of operations on the longest path), so
 * kappa_c = max_k A_c(k) / max_k |X_c(k)| is the conditioning of channel c.
 * ========================================================================= */
typedef struct {
  orc_ctx base;        /* geometry / configuration; its h_SSB holds |h_SSB| bounds */
} orc_abs;

static double lagrange_abs(const double* s, int64_t n, int64_t i0, double x, int N) {
  double w[64];
  orc_lagrange_weights(x, N, w);
  int jlo = -N / 2 + 1;
  double acc = 0.0;
  for (int a = 0; a < N; ++a) {
    int64_t i = i0 + jlo + a;
    if (i >= 0 && i < n) acc += fabs(w[a]) * fabs(s[i]);
  }
  return acc;
}

static void abs_init(orc_ctx* x, const orc_config* c, const orc_orbit* o, const orc_source* s,
                     int64_t n, const double* hp, const double* hc) {
  ctx_init(x, c, o, s, n, hp, hc);
  double c2 = fabs(cos(2.0 * s->psi)), s2 = fabs(sin(2.0 * s->psi));
  for (int64_t i = 0; i < n; ++i) {
    x->hp_ssb[i] = fabs(hp[i]) * c2 + fabs(hc[i]) * s2;
    x->hc_ssb[i] = fabs(hp[i]) * s2 + fabs(hc[i]) * c2;
  }
}

static void abs_stage1_at(orc_ctx* x, int64_t i, double y6[6]) {
  orc_geom g;
  orc_geometry(x->o, x->s->beta, x->s->lam, t_of(x, i), &g);
  int N = x->c->taps;
  double dt = x->s->dt;
  for (int a = 0; a < 6; ++a) {
    int64_t i0; double fx;
    double acc = 0.0;
    double d2[2] = {g.ds[a], g.dr[a]};
    for (int q = 0; q < 2; ++q) {
      orc_split(i, d2[q], dt, &i0, &fx);
      acc += fabs(g.xi_p[a]) * lagrange_abs(x->hp_ssb, x->n, i0, fx, N) +
             fabs(g.xi_c[a]) * lagrange_abs(x->hc_ssb, x->n, i0, fx, N);
    }
    y6[a] = acc / fabs(2.0 * (1.0 - g.kn[a]));
  }
}

static void abs_ensure_y(orc_ctx* x, int64_t lo, int64_t hi) {
  ensure_y_alloc(x);
  if (lo < 0) lo = 0;
  if (hi > x->n) hi = x->n;
  for (int64_t i = lo; i < hi; ++i) {
    if (x->y_ok[i]) continue;
    double y6[6];
    abs_stage1_at(x, i, y6);
    for (int a = 0; a < 6; ++a) x->y[(size_t)a * x->n + i] = y6[a];
    x->y_ok[i] = 1;
  }
}

static void abs_full_at(orc_ctx* x, int64_t k, double out[3]) {
  orc_geom g;
  orc_geometry(x->o, x->s->beta, x->s->lam, t_of(x, k), &g);
  int N = x->c->taps;
  for (int c = 0; c < 3; ++c) {
    double acc = 0.0;
    for (int t = 0; t < n_terms(x->c->tdi_gen); ++t) {
      int sign, link;
      double d;
      term_delay(x, &g, c, t, k, &sign, &link, &d);
      int64_t i0; double fx;
      orc_split(k, d, x->s->dt, &i0, &fx);
      abs_ensure_y(x, i0 - N / 2 + 1, i0 + N / 2 + 1);
      acc += lagrange_abs(x->y + (size_t)link_slot(link) * x->n, x->n, i0, fx, N);
    }
    out[c] = acc;
  }
}

static void abs_ensure_g(orc_ctx* x, int64_t lo, int64_t hi) {
  ensure_g_alloc(x);
  if (lo < 0) lo = 0;
  if (hi > x->n) hi = x->n;
  double num[9], den;
  int hw = stencil_coeffs(x->m, x->c->stencil_order, num, &den);
  double anum[9];
  for (int q = 0; q < 2 * hw + 1; ++q) anum[q] = fabs(num[q]);
  double scale = den * pow(x->s->dt, (double)x->m);
  for (int64_t i = lo; i < hi; ++i) {
    if (x->g_ok[i]) continue;
    x->gp[i] = stencil_at(x->hp_ssb, x->n, i, anum, hw, scale);
    x->gc[i] = stencil_at(x->hc_ssb, x->n, i, anum, hw, scale);
    x->g_ok[i] = 1;
  }
}

static void abs_lfa_at(orc_ctx* x, int64_t k, double out[3]) {
  orc_geom g;
  orc_geometry(x->o, x->s->beta, x->s->lam, t_of(x, k), &g);
  int N = x->c->taps;
  for (int c = 0; c < 3; ++c) {
    int la = (c + 1) % 3 + 1, lb = (c + 2) % 3 + 1;
    double Ta = x->c->equal_arms ? x->o->L / ORC_C : g.T[la - 1];
    double Tb = x->c->equal_arms ? x->o->L / ORC_C : g.T[lb - 1];
    double pref, d;
    if (x->c->tdi_gen == 20) { pref = 4.0 * Ta * Tb * (Ta + Tb); d = 2.0 * (Ta + Tb); }
    else { pref = 2.0 * Ta * Tb; d = Ta + Tb; }
    double acc = 0.0;
    int ls[2] = {la, lb};
    orc_ctx* nt = (orc_ctx*)x->nt;
    for (int q = 0; q < 2; ++q) {
      int64_t i0; double fx;
      orc_split(k, d + g.mu[ls[q] - 1], x->s->dt, &i0, &fx);
      abs_ensure_g(x, i0 - N / 2 + 1, i0 + N / 2 + 1);
      int a = link_slot(ls[q]);
      acc += fabs(g.xi_p[a]) * lagrange_abs(x->gp, x->n, i0, fx, N) +
             fabs(g.xi_c[a]) * lagrange_abs(x->gc, x->n, i0, fx, N);
      if (nt) {
        double Tl = q == 0 ? Ta : Tb, To = q == 0 ? Tb : Ta;
        double kap = lfa_kappa(x->c->tdi_gen, Tl, To, g.kn[ls[q] - 1]);
        abs_ensure_g(nt, i0 - N / 2 + 1, i0 + N / 2 + 1);
        acc += kap * (fabs(g.xi_p[a]) * lagrange_abs(nt->gp, nt->n, i0, fx, N) +
                      fabs(g.xi_c[a]) * lagrange_abs(nt->gc, nt->n, i0, fx, N));
      }
    }
    out[c] = pref * acc;
  }
}

void orc_response_abs_at(const orc_config* c, const orc_orbit* o, const orc_source* s,
                         int64_t n, const double* hp, const double* hc,
                         int64_t nk, const int64_t* ks, double* X, double* Y, double* Z) {
  orc_ctx x;
  abs_init(&x, c, o, s, n, hp, hc);
  if (c->lfa_terms == 2 && c->mode != ORC_FULL) {
    orc_ctx* t = (orc_ctx*)malloc(sizeof(orc_ctx));
    abs_init(t, c, o, s, n, hp, hc);
    t->m = x.m + 2;
    x.nt = t;
  }
  if (c->x20_from_x15 && c->tdi_gen == 20 && c->mode != ORC_FULL) {
    ctx_shortcut(&x, n, hp, hc);
    orc_x20* sc = (orc_x20*)x.sc;
    ctx_free(&sc->x15);
    abs_init(&sc->x15, &sc->c15, o, s, n, hp, hc);
    sc->absmode = 1;
  }
  for (int64_t q = 0; q < nk; ++q) {
    int64_t k = ks[q];
    double r[3] = {0.0, 0.0, 0.0}, a[3];
    if (c->mode == ORC_FULL) {
      abs_full_at(&x, k, r);
    } else if (c->mode == ORC_LFA) {
      if (x.sc) x20_at(&x, k, r);
      else abs_lfa_at(&x, k, r);
    } else {
      double kH = (s->t_hyb - s->t0) / s->dt;
      double rel = (double)k - kH, z = rel / c->sigma_samples;
      double wp = 1.0 / (1.0 + exp(z)), wm = 1.0 / (1.0 + exp(-z));
      if (rel <= 0.5 * c->T_samples) {
        if (x.sc) x20_at(&x, k, a);
        else abs_lfa_at(&x, k, a);
        for (int i = 0; i < 3; ++i) r[i] += wp * a[i];
      }
      if (rel >= -0.5 * c->T_samples) {
        abs_full_at(&x, k, a);
        for (int i = 0; i < 3; ++i) r[i] += wm * a[i];
      }
    }
    X[q] = r[0]; Y[q] = r[1]; Z[q] = r[2];
  }
  ctx_free(&x);
}
