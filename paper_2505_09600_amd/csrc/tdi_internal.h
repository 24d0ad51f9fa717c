// Internal declarations shared by the host runtime (tdi_api.cpp) and the
// device kernels (tdi_kernels.hip).  Not part of the public ABI.
#pragma once

#include <stdint.h>

namespace tdi {

// Orbit constants prepared once per plan.
struct OrbitDev {
  int32_t kind;          // 0 frozen, 1 first-order analytic
  int32_t pad;
  double L, R, omega, kappa0, t_freeze;
  double e;              // L / (2 sqrt(3) R)
  double cb[3], sb[3];   // cos / sin of beta_i = 2 pi i / 3 + lambda0
  double L_over_c;
};

// Per-source record on the device.
struct SrcDev {
  double beta, lam, psi, t0, dt, t_hyb;
  int64_t off;           // first sample in the flat arrays
  int64_t n;             // number of samples
  int64_t tile0;         // first global tile of this source
  int64_t pad;
};

constexpr int kMaxTaps = 32;
constexpr int kBlock = 256;

// Per-run values, uploaded with the source table in one copy so that a
// captured graph can be replayed for new batches.  The SrcDev array follows.
struct RunDesc {
  int64_t n_src;
  int64_t n_tiles;
  const double* hp;
  const double* hc;
  void* X;
  void* Y;
  void* Z;
  int32_t cap_g, cap_h, cap_y;   // LDS capacities (samples) of the staged windows
  int32_t pad;
};

struct KParams {
  const RunDesc* rd;
  const SrcDev* src;             // = (const SrcDev*)(rd + 1)
  int32_t* err_flag;       // set to 1 when a retarded window check fails
  uint32_t* counter;       // persistent work counter (reset before each run)
  OrbitDev orb;
  int32_t gen, mode, equal_arms, stencil_m;
  double T_s, sigma_s;
  double lag_c[kMaxTaps];  // Lagrange normalisation 1 / prod_{m != j} (j - m)
  double st_num[7];        // LFA stencil numerators over offsets -hw..hw
  double st_den;           // stencil denominator (times dt^m at run time)
  int32_t st_hw;
  int32_t tile;            // output samples per tile
  int32_t persistent;      // 1: loop over tiles with the work counter
};

// Launch entry points (defined in tdi_kernels.hip).
int launch_reset(uint32_t* counter, int32_t* err_flag, int reset_err, void* stream);
int launch_main(const KParams& p, int taps, int fp32, int grid, size_t lds_bytes, void* stream);
size_t lds_bytes_for(int tile, int cap_g, int cap_h, int cap_y, int fp32);
int max_lds_bytes();

}  // namespace tdi
