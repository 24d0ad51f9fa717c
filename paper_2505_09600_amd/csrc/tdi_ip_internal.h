// Internal declarations of the noise-weighted inner product (host runtime
// tdi_ip.cpp and kernels tdi_ip_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdi_ip {

constexpr int kIpBlock = 256;            // threads per workgroup
// complex elements one workgroup holds in LDS (64 KB): FP32 and FP64
constexpr int kElemsF = 8192;
constexpr int kElemsD = 4096;

template <typename T> constexpr int elems_of() { return sizeof(T) == 4 ? kElemsF : kElemsD; }
// longest row of the second pass (two rows share the LDS)
template <typename T> constexpr int row_max() { return elems_of<T>() / 2; }

// Per-source record.  The zero-extended length N = 2^logN is split as
// N = N1 * N2 (N1 = 1: one pass straight from the input).
struct IpSrc {
  int64_t off, n;          // first sample and length in the input arrays
  int64_t ws;              // first workspace element (channel c at ws + c * N)
  int64_t t1, t2, part;    // first task of pass 1 and pass 2, first partial slot
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
  const double* winv;      // 1 / S_n at f = k / (N_max dt): [2][K_max + 1] (A and E, T)
  int64_t kmax;
  int32_t logNmax, pad;
  double dt, f_min, f_max;
};

__host__ __device__ inline const IpSrc* ip_sources(const IpParams* p) {
  return reinterpret_cast<const IpSrc*>(p + 1);
}

int launch_pass1(const IpParams* dp, int fp64, int64_t tasks, void* stream);
int launch_pass2(const IpParams* dp, int fp64, int64_t tasks, void* stream);
int launch_reduce(const IpParams* dp, int64_t n_src, void* stream);

}  // namespace tdi_ip
