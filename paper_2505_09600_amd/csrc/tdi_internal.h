// Internal declarations shared by the host runtime (tdi_api.cpp) and the
// device kernels (tdi_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdi {

constexpr int kBlock = 256;       // threads per workgroup (4 waves of 64)
constexpr int kNodes = 7;         // Chebyshev nodes of the per-tile geometry fit (degree 6)
constexpr int kNQ = 27;           // fitted geometry quantities per tile
constexpr int kFitLen = kNQ * kNodes;   // coefficients of one tile fit
constexpr int kTileLfa = 1024;    // outputs per LFA tile (4 waves x 256)
constexpr int kTileFull = 256;    // outputs per full-response tile (FULL mode; the largest)
constexpr int kTileFullHybrid = 64;   // the hybrid's short full regions: small tiles, more workgroups
constexpr int kTileFullSmall = 16;    // hybrid batches with fewer full tiles than compute units
constexpr int kWaveOut = 256;     // LFA FP32: outputs per wave (4 per lane, stride 64)
// FP32 bulk LFA path (k_lfa_fast): chunks of 4 waves x 64 lanes x 9 outputs,
// four chunks per tile (one geometry fit); its stencil pass covers up to
// kFastStencilSpan elements in one sweep.
constexpr int kFastChunk = 2304;
constexpr int kTileLfaFast = 4 * kFastChunk;   // largest fast-path tile (the record holds 4 chunks)
constexpr int kFastStencilSpan = 11 * kBlock;
constexpr int kFastOutPerLane = 9;
constexpr int kWGrid = 16;                 // Lagrange Taylor table: rows per unit offset
constexpr double kFastDtMax = 40.0;        // s: quadratic chunk models stay below 1e-6 relative
constexpr double kFastRateMax = 2.0e-4;    // bound of |d delay / dt| for the offset expansions
constexpr size_t kFastTileBytesMax = 4096;  // bound of the fast path's per-tile record (checked in the kernels)
constexpr int kPrepTiles = 7;              // fast path pre-pass: most tiles per workgroup pass
constexpr int kTileLinks = 2048;           // link outputs: outputs per tile (kTileLinks / kBlock per thread)

// Orbit constants prepared once per plan.
struct OrbitDev {
  int32_t kind;          // 0 frozen, 1 first-order analytic, 2 sampled table
  int32_t pad;
  double L, R, omega, kappa0, t_freeze;
  double e;              // L / (2 sqrt(3) R)
  double cb[3], sb[3];   // cos / sin of beta_i = 2 pi i / 3 + lambda0
  double L_over_c;
  const double* tab;     // table: [ntab][3][3] positions (device)
  int64_t ntab;
  double tab_t0, tab_idt;  // time of sample 0, 1 / spacing
};

// Per-source record on the device, with the sample ranges and first global
// tile of each kernel (LFA and full response).
struct SrcDev {
  double beta, lam, psi, t0, dt, t_hyb;
  double c2psi, s2psi;   // cos 2 psi, sin 2 psi
  int64_t off;           // first sample in the flat arrays
  int64_t n;             // number of samples
  int64_t lfa_t0, lfa_kb, lfa_ke;     // LFA tiles cover samples [kb, ke)
  int64_t full_t0, full_kb, full_ke;  // full-response tiles cover samples [kb, ke)
};

// Kernel parameters, resident in device memory (one upload per run), followed
// by the SrcDev array.
struct KParams {
  // per run
  int64_t n_src;
  int64_t n_tiles_lfa, n_tiles_full;
  const double* hp;
  const double* hc;
  void* X;
  void* Y;
  void* Z;
  int32_t cap_g, cap_hl;               // LFA window capacities (samples): derivative, strain
  int32_t cap_hf, cap_y;               // full-response capacities: strain, link series
  int32_t lfa_goff;                    // byte offset of the LFA derivative window in LDS
                                       // (fast path: of the F_l series; 0 = over the strain)
  int32_t lfa_terms;                   // single-link LFA: 1 leading term, 2 with the next term
  // per plan
  int32_t* err;          // window-check report (8 ints)
  void* lfa_tiles;       // fast LFA path: per-tile records written by the pre-pass
  uint32_t* counters;    // work counters of the persistent kernels, zero at launch: [0] LFA tiles,
                         // [1] full tiles (the plan keeps them in front of the parameter block)
  OrbitDev orb;
  int32_t gen, mode, equal_arms, stencil_m, stencil_p, persistent;
  int32_t aet, cap_lk;   // aet: store A, E, T instead of X, Y, Z; cap_lk: link-output window
  int32_t nested;        // time-nested stage-2 delays
  int32_t tile_fast;     // fast LFA path: outputs per tile (1, 2 or 4 chunks of kFastChunk)
  int32_t tile_full;     // full-response outputs per tile (at most kTileFull)
  int32_t prep_tiles;    // fast LFA pre-pass: tiles per workgroup pass (1..kPrepTiles)
  int64_t link_stride;   // link outputs: elements between the six link arrays (X is their base)
  double T_s, sigma_s;
  double D2_bound;       // upper bound of a stage-2 delay (s)
  const double* x15;     // TDI 2.0 from TDI 1.5 (k_x20): the FP64 TDI 1.5 LFA series,
  int64_t x15_stride;    // three channel arrays x15_stride apart (same offsets as the outputs)
};

__host__ __device__ inline const SrcDev* sources_of(const KParams* p) {
  return reinterpret_cast<const SrcDev*>(p + 1);
}

// Launch entry points (defined in tdi_kernels.hip).
int set_constants();
// fast != 0 selects the FP32 bulk LFA kernel (fp32 must be 1)
// nx != 0: LFA with the next term (lfa_terms = 2; general kernel only)
int launch_lfa(const KParams* dp, int taps, int fp32, int fast, int nx, int grid, size_t lds_bytes, void* stream);
// hybrid != 0: the term-parallel stage 2 (tiles of at most kTileFullHybrid, LDS from
// full_lds_bytes(..., hybrid = 1))
int launch_full(const KParams* dp, int taps, int fp32, int hybrid, int grid, size_t lds_bytes, void* stream);
// TDI 2.0 LFA from the TDI 1.5 LFA series in KParams::x15 (window capacity cap_g)
int launch_x20(const KParams* dp, int taps, int fp32, int grid, size_t lds_bytes, void* stream);
int occupancy_x20(int taps, int fp32, size_t lds);
size_t x20_lds_bytes(int cap);
// link outputs: one workgroup per tile of kTileLinks samples (tile list in SrcDev::lfa_t0)
// arm != 0 (FP32, LFA or hybrid, leading term): the per-arm read of the LFA part
int launch_links(const KParams* dp, int taps, int fp32, int arm, int64_t grid, size_t lds, void* stream);
size_t links_lds_bytes(int cap, int fp32, int windows);
// pre-pass of the fast LFA path: per-tile records (geometry fits, chunk
// windows, wave models) for all LFA tiles (grid-stride over tiles)
int launch_lfa_fit(const KParams* dp, int taps, int grid, void* stream);
int occupancy_lfa_fit(int taps);   // resident pre-pass workgroups per CU
size_t fast_tile_bytes();     // bytes of one per-tile record
// LFA dynamic LDS: h window (FP64), reused for the FP32 wave tables, then the
// derivative window; goff receives the byte offset of the latter.  Fast path:
// h window and the three F_l series, overlaid when one stencil sweep suffices.
size_t lfa_lds_bytes(int taps, int cap_g, int cap_h, int fp32, int fast, int nx, int* goff);
// hybrid != 0 adds the per-term values of the term-parallel stage 2 (tiles of at
// most kTileFullHybrid outputs)
size_t full_lds_bytes(int cap_h, int cap_y, int fp32, int hybrid);
int occupancy_lfa(int taps, int fp32, int fast, int nx, size_t lds);
int occupancy_full(int taps, int fp32, int hybrid, size_t lds);

}  // namespace tdi
