// Internal declarations of the noise-weighted inner product (host runtime
// tdi_ip.cpp and kernels tdi_ip_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdi_ip {

constexpr int kIpBlock = 512;            // threads per workgroup
// complex elements one workgroup holds in LDS (64 KB): FP32 and FP64
constexpr int kElemsF = 8192;
constexpr int kElemsD = 4096;

template <typename T> constexpr int elems_of() { return sizeof(T) == 4 ? kElemsF : kElemsD; }
template <typename T> constexpr int log_elems_of() { return sizeof(T) == 4 ? 13 : 12; }
// longest row of the second pass (two rows share the LDS)
template <typename T> constexpr int row_max() { return elems_of<T>() / 2; }

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
  // weights 1 / S_n(f_k), zero outside the band, one table per length N laid
  // out in the order of the second pass: [class A/E, T][k1 < N1][k2 < N2/2]
  // for bin k = k1 + N1 k2
  const double* wt;
  // twiddle tables in the transform precision (complex pairs):
  //   tw[m] = e^{-2 pi i m / E} (E = LDS elements), for the LDS stages;
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
