// Internal declarations of the noise-weighted inner product (host runtime
// tdi_ip.cpp and kernels tdi_ip_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdi_ip {

// Tile shapes of the two passes (T = float or double, complex elements in LDS).
// Pass 1 reads column blocks of the input (stride N2): a 128 KB tile, one
// workgroup of 1024 threads per compute unit, makes every row of a block a
// long contiguous read.  Pass 2 (and the one-pass path) reads whole rows: 64 KB
// tiles let two workgroups of 512 threads share a compute unit, so that one's
// transforms overlap the other's loads.
template <typename T, int Pass> struct Tile {
  static constexpr int kLogE = (sizeof(T) == 4 ? 13 : 12) + (Pass == 1 ? 1 : 0);
  static constexpr int kE = 1 << kLogE;
  static constexpr int kBlock = Pass == 1 ? 1024 : 512;
  static constexpr int kPerCu = Pass == 1 ? 1 : 2;     // resident workgroups per compute unit
};
// workgroup sizes by pass (single-argument names for __launch_bounds__)
template <typename T> constexpr int kBlock1 = Tile<T, 1>::kBlock;
template <typename T> constexpr int kBlock2 = Tile<T, 2>::kBlock;
// the LDS-stage twiddle table holds 2^log_tw roots of unity (the larger tile)
template <typename T> constexpr int log_tw() { return Tile<T, 1>::kLogE; }
constexpr int kReduceBlock = 256;

// Per-source record.  The zero-extended length N = 2^logN is split as
// N = N1 * N2 (N1 = 1: one pass straight from the input).
struct IpSrc {
  int64_t off, n;          // first sample and length in the input arrays
  int64_t ws;              // first workspace element (channel c at ws + c * N)
  int64_t t1, t2, part;    // first task of pass 1 and pass 2, first partial slot
  int64_t wofs;            // this length's weight table in IpParams::wt
  int32_t logN, logN1, logN2, cols;   // cols: columns of one pass-1 task
  int32_t n1, n2;          // pass-1 / pass-2 tasks per channel
};

// Parameters of one run, followed in device memory by IpSrc[n_src].
struct IpParams {
  int64_t n_src, n_t1, n_t2;
  const void* x[3];
  const void* y[3];
  void* ws;                // complex workspace of the two-pass transforms
  double* part;            // 3 partial sums per pass-2 task
  double* out;             // 9 per source: per channel <x|x>, <x|y>, <y|y>
  // weights 2^-wexp / S_n(f_k) in the transform precision, zero outside the
  // band, one table per length N laid out in the order of the second pass:
  // [class A/E, T][k1 < N1][k2 < N2/2] for bin k = k1 + N1 k2.  1/S_n is of
  // order 1e40, beyond FP32: the power-of-two scale keeps it in range and the
  // reduction undoes it exactly (wexp = 0 for FP64 tables).
  const void* wt;
  int32_t wexp, pad0;
  // twiddle tables in the transform precision (complex pairs):
  //   tw[m] = e^{-2 pi i m / 2^log_tw}, for the LDS stages;
  //   th[h] = e^{-2 pi i h 2^tbits / N_max}, tl[l] = e^{-2 pi i l / N_max}, for the
  //   four-step twiddle e^{-2 pi i m / N_max} = th[m >> tbits] tl[m mod 2^tbits]
  const void* tw;
  const void* th;
  const void* tl;
  int32_t logNmax, tbits;
  double dt, f_min, f_max;
};

__host__ __device__ inline const IpSrc* ip_sources(const IpParams* p) {
  return reinterpret_cast<const IpSrc*>(p + 1);
}

// persistent launches: at most `grid` workgroups (a multiple of 8) walk the tasks
int launch_pass1(const IpParams* dp, int fp64, int64_t tasks, int grid, void* stream);
int launch_pass2(const IpParams* dp, int fp64, int64_t tasks, int grid, void* stream);
int launch_reduce(const IpParams* dp, int64_t n_src, void* stream);

}  // namespace tdi_ip
