/*
 * FP64 CPU oracle of the hybrid time-domain LISA response (arXiv:2505.09600).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct
 * re-statement of the paper's definitions (Sec. II "Full response",
 * Sec. III "Low-frequency response", Sec. IV "Hybrid response" and App. B).
 * It shares no code, header, table or constant with the HIP library; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg load it.
 */
#ifndef TDI_ORACLE_H
#define TDI_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_ORBIT_FROZEN = 0, ORC_ORBIT_ANALYTIC1 = 1, ORC_ORBIT_TABLE = 2 };
enum { ORC_FULL = 0, ORC_LFA = 1, ORC_HYBRID = 2 };

typedef struct {
  int32_t kind;      /* ORC_ORBIT_* */
  int32_t pad_;
  double L;          /* nominal arm length, m */
  double R;          /* orbital radius, m */
  double omega;      /* orbital angular velocity, rad/s */
  double kappa0;     /* initial orbital phase, rad */
  double lambda0;    /* initial constellation orientation, rad */
  double t_freeze;   /* FROZEN: positions are taken at this time, s */
  const double* table;   /* TABLE: positions [n_table][3][3] (sample, spacecraft, xyz), m */
  int64_t n_table;
  double table_t0, table_dt;
} orc_orbit;

typedef struct {
  int32_t tdi_gen;        /* 15 or 20 */
  int32_t mode;           /* ORC_FULL, ORC_LFA, ORC_HYBRID */
  int32_t taps;           /* N, even */
  int32_t stencil_order;  /* p in {2, 4} */
  int32_t equal_arms;     /* LFA only: 1 = equal constant delays L/c */
  int32_t lfa_terms;      /* LFA: 2 = keep the next term of the central series (links and X, Y, Z) */
  int32_t nested_delays;  /* full response: 1 = each delay at the time it is applied (time-nested),
                             0 = every delay at the output time (the paper's choice) */
  int32_t x20_from_x15;   /* LFA, TDI 2.0: 1 = X2.0 from the TDI 1.5 LFA series by
                             Eq. (relation_X20_X15_nonequal_timedelays) */
  double T_samples;       /* hybrid window length, samples */
  double sigma_samples;   /* sigmoid width, samples */
} orc_config;

typedef struct {
  double beta, lam, psi;  /* ecliptic latitude, longitude, polarisation (rad) */
  double t0, dt;          /* t_k = t0 + k dt */
  double t_hyb;           /* switch time (s); +inf pure LFA, -inf pure full */
} orc_source;

/* Link l in {+1,+2,+3,-1,-2,-3}: sender s and receiver r (1-based). */
void orc_link_ends(int l, int* s, int* r);

/* Propagation / polarisation triad of a source at (beta, lambda). */
void orc_triad(double beta, double lam, double k[3], double u[3], double v[3]);

/* Spacecraft positions R[i] (i = 0,1,2 for S/C 1,2,3) at time t. */
void orc_positions(const orc_orbit* o, double t, double R[3][3]);

/* Light time of link l received at time t (s). */
double orc_light_time(const orc_orbit* o, int l, double t);

/* Per-link geometry at time t, links ordered +1,+2,+3,-1,-2,-3. */
typedef struct {
  double T[6];        /* light time, s */
  double n[6][3];     /* photon direction sender -> receiver */
  double xi_p[6], xi_c[6];
  double kn[6];       /* k . n */
  double ds[6], dr[6];/* delta_s, delta_r (s) */
  double mu[3];       /* k.(R_s + R_r)/(2c) for links +1,+2,+3 */
  double R[3][3];
} orc_geom;
void orc_geometry(const orc_orbit* o, double beta, double lam, double t, orc_geom* g);

/* Retarded-index split of delay d (s) at output sample k. */
void orc_split(int64_t k, double d, double dt, int64_t* i0, double* x);

/* Lagrange interpolation of s (length n, zero outside) at i0 + x, N taps. */
double orc_lagrange(const double* s, int64_t n, int64_t i0, double x, int N);
void orc_lagrange_weights(double x, int N, double* w);

/* m-th derivative central stencil of accuracy p applied on the grid
 * (zero extension of h), result divided by dt^m; m in {1,2,3}, p in {2,4}. */
void orc_stencil(const double* h, int64_t n, int m, int p, double dt, double* g);

/* Stage 1 of the full response: the six link series y_l[k], l order as above. */
void orc_links(const orc_config* c, const orc_orbit* o, const orc_source* s,
               int64_t n, const double* hp, const double* hc, double* y /* 6*n */);

/* The six single-link outputs y[a*n + k] in the configuration's mode: full
 * (stage 1), LFA (Eq. yslr_strain_derivatives per link) or their hybrid
 * (Eq. hybridized_yslr); link order as above. */
void orc_link_outputs(const orc_config* c, const orc_orbit* o, const orc_source* s,
                      int64_t n, const double* hp, const double* hc, double* y /* 6*n */);

/* Stage 2 on arbitrary link series and per-sample light times T[l*n + k]. */
void orc_tdi_combine(int gen, int N, int64_t n, double dt, const double* y,
                     const double* T, double* X, double* Y, double* Z);

/* Term t of Eq. (X1.5) (t < 8) or of Eq. (X2.0) (t < 16) in time-nested form:
 * sign, link of y, and its delays in the order they are applied (d[0] is
 * taken at the output time, d[q] at the output time less the first q). */
void orc_nested_term(int t, int* sign, int* link, int* nd, int d[8]);

/* Stage 2 with time-nested delays: the light time of each later delay is read
 * from T at the retarded time by N-tap Lagrange interpolation (zero outside
 * [0, n), so only samples whose retarded reads stay inside are meaningful). */
void orc_tdi_combine_nested(int gen, int N, int64_t n, double dt, const double* y,
                            const double* T, double* X, double* Y, double* Z);

/* Whole response for one source (all samples). */
void orc_response(const orc_config* c, const orc_orbit* o, const orc_source* s,
                  int64_t n, const double* hp, const double* hc,
                  double* X, double* Y, double* Z);

/* Response at selected sample indices only (for sampled checks at full size). */
void orc_response_at(const orc_config* c, const orc_orbit* o, const orc_source* s,
                     int64_t n, const double* hp, const double* hc,
                     int64_t nk, const int64_t* ks, double* X, double* Y, double* Z);

/* Batch over sources (OpenMP across sources); offsets has n_sources + 1 entries. */
void orc_response_batch(const orc_config* c, const orc_orbit* o, int64_t n_sources,
                        const orc_source* src, const int64_t* offsets,
                        const double* hp, const double* hc,
                        double* X, double* Y, double* Z);

/* Sampled outputs of a batch: source i is evaluated at the k_offsets[i] ..
 * k_offsets[i+1]-1 entries of ks (sample indices within the source); results
 * are written at the same positions of X, Y, Z.  OpenMP across sources. */
void orc_response_batch_at(const orc_config* c, const orc_orbit* o, int64_t n_sources,
                           const orc_source* src, const int64_t* offsets, const double* hp,
                           const double* hc, const int64_t* k_offsets, const int64_t* ks,
                           double* X, double* Y, double* Z);

/* Rounding-error scale A(k) at selected samples: the response evaluated with
 * absolute values of every quantity and sums in place of differences (not part
 * of the method; used to bound FP64 evaluation-order differences). */
void orc_response_abs_at(const orc_config* c, const orc_orbit* o, const orc_source* s,
                         int64_t n, const double* hp, const double* hc,
                         int64_t nk, const int64_t* ks, double* X, double* Y, double* Z);

/* Per-channel condition number: max_k sum_terms |term_k| / max_k |X_k|. */
void orc_full_terms_absmax(const orc_config* c, const orc_orbit* o, const orc_source* s,
                           int64_t n, const double* hp, const double* hc,
                           double* absmax3 /* 3 */);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
