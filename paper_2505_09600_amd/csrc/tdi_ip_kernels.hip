// Noise-weighted inner product of two sets of A, E, T series on gfx950.
//
// <x|y> = 4 Re sum_k conj(x~_k) y~_k / S_n(f_k) df (Eq. scalar_product, App. on
// the scalar product), with x~ the discrete form of Eq. (defFT): dt times the
// DFT of the series zero-extended to N = 2^logN samples.
//
// x and y of one channel travel as one complex series z = x + i y, so one
// complex transform serves both; with Z = DFT(z) and P = Z_{N-k},
//   |x~_k|^2 = dt^2 |Z_k + conj P|^2 / 4,   |y~_k|^2 = dt^2 |Z_k - conj P|^2 / 4,
//   Re(conj(x~_k) y~_k) = dt^2 Im(Z_k P) / 2.
// Long series use the four-step split N = N1 N2: pass 1 transforms the N2
// columns (length N1, stride N2) and applies the twiddles e^{-2 pi i j2 k1 / N};
// pass 2 transforms the rows k1 (length N2), giving Z at k = k1 + N1 k2.  The
// spectrum is never written back: a pass-2 workgroup holds rows k1 and N1 - k1,
// which hold every partner N - k of its own bins, and reduces the three
// weighted sums on the spot.  Short series (N1 = 1) take one pass straight
// from the input.
//
// The transforms are radix-4 (plus one radix-2 stage for odd log2 length)
// Stockham passes in LDS with natural-order output, in the precision of the
// input (float or double); the weighted sums accumulate in double.
#include <hip/hip_runtime.h>

#include "tdi_ip_internal.h"

namespace tdi_ip {
namespace {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using V = float2; };
template <> struct Cplx<double> { using V = double2; };

__device__ __forceinline__ void sincospi_t(float a, float* s, float* c) { sincospif(a, s, c); }
__device__ __forceinline__ void sincospi_t(double a, double* s, double* c) { sincospi(a, s, c); }
__device__ __forceinline__ float ldexp_t(float a, int e) { return ldexpf(a, e); }
__device__ __forceinline__ double ldexp_t(double a, int e) { return ldexp(a, e); }

template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// e^{-2 pi i m / M} for 0 <= m < M, M a power of two: 2 m / M is exact in T.
template <typename T, typename V>
__device__ __forceinline__ V root(int64_t m, int logM) {
  const T a = ldexp_t((T)m, 1 - logM);
  T s, c;
  sincospi_t(a, &s, &c);
  V r;
  r.x = c;
  r.y = -s;
  return r;
}

template <typename V>
__device__ __forceinline__ void dft4(V* a) {
  V t0, t1, t2, t3;
  t0.x = a[0].x + a[2].x; t0.y = a[0].y + a[2].y;
  t1.x = a[0].x - a[2].x; t1.y = a[0].y - a[2].y;
  t2.x = a[1].x + a[3].x; t2.y = a[1].y + a[3].y;
  t3.x = a[1].x - a[3].x; t3.y = a[1].y - a[3].y;
  a[0].x = t0.x + t2.x; a[0].y = t0.y + t2.y;
  a[2].x = t0.x - t2.x; a[2].y = t0.y - t2.y;
  // y1 = t1 - i t3, y3 = t1 + i t3
  a[1].x = t1.x + t3.y; a[1].y = t1.y - t3.x;
  a[3].x = t1.x - t3.y; a[3].y = t1.y + t3.x;
}

template <typename V>
__device__ __forceinline__ void dft2(V* a) {
  V t;
  t.x = a[0].x - a[1].x; t.y = a[0].y - a[1].y;
  a[0].x += a[1].x; a[0].y += a[1].y;
  a[1] = t;
}

// One Stockham stage of radix R on B sequences of length L = 2^logL held in
// LDS; element e of sequence b sits at buf[b * bs + e * es].  Ns is the length
// of the sub-transforms already formed.  Butterfly q maps to sequence
// b = q mod B (B = 2^logB) and index j = q / B, so that neighbouring lanes touch
// neighbouring sequences (interleaved layout) or neighbouring elements.
template <typename T, int R>
__device__ void fft_stage(typename Cplx<T>::V* buf, int logL, int logNs, int logB, int bs, int es) {
  using V = typename Cplx<T>::V;
  constexpr int kMaxQ = elems_of<T>() / (R * kIpBlock);
  constexpr int kLogR = R == 4 ? 2 : 1;
  const int nb = 1 << (logL - kLogR);          // butterflies per sequence
  const int total = nb << logB;
  const int Ns = 1 << logNs;
  V v[kMaxQ][R];
#pragma unroll
  for (int i = 0; i < kMaxQ; ++i) {
    const int q = threadIdx.x + i * kIpBlock;
    if (q < total) {
      const int b = q & ((1 << logB) - 1), j = q >> logB;
      const V* src = buf + b * bs + j * es;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src[r * nb * es];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kMaxQ; ++i) {
    const int q = threadIdx.x + i * kIpBlock;
    if (q < total) {
      const int b = q & ((1 << logB) - 1), j = q >> logB;
      const int k = j & (Ns - 1);
      if (logNs > 0) {
        const V w1 = root<T, V>(k, logNs + kLogR);
        V w = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[i][r] = cmul(v[i][r], w);
          if (r + 1 < R) w = cmul(w, w1);
        }
      }
      if constexpr (R == 4) dft4(v[i]); else dft2(v[i]);
      V* dst = buf + b * bs + ((j - k) * R + k) * es;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns * es] = v[i][r];
    }
  }
  __syncthreads();
}

// Forward DFT (e^{-2 pi i j k / L}) of B sequences in place, natural order out.
template <typename T>
__device__ void lds_fft(typename Cplx<T>::V* buf, int logL, int logB, int bs, int es) {
  int logNs = 0;
  if (logL & 1) {
    fft_stage<T, 2>(buf, logL, 0, logB, bs, es);
    logNs = 1;
  }
  while (logNs < logL) {
    fft_stage<T, 4>(buf, logL, logNs, logB, bs, es);
    logNs += 2;
  }
}

// the source that owns a task: last s with first-task(s) <= task
template <int Pass>
__device__ __forceinline__ int64_t find_task_source(const IpSrc* S, int64_t n, int64_t task) {
  int64_t lo = 0, hi = n;            // answer in [lo, hi)
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    const int64_t t = Pass == 1 ? S[mid].t1 : S[mid].t2;
    if (t <= task) lo = mid; else hi = mid;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ T load_or_zero(const void* p, int64_t off, int64_t j, int64_t n) {
  return j < n ? static_cast<const T*>(p)[off + j] : (T)0;
}

// Pass 1: columns j2 in [c0, c0 + cols) of one channel of one source.
template <typename T>
__global__ void __launch_bounds__(kIpBlock) k_ip_pass1(const IpParams* __restrict__ P) {
  using V = typename Cplx<T>::V;
  __shared__ V buf[elems_of<T>()];
  const int64_t task = blockIdx.x;
  if (task >= P->n_t1) return;
  const IpSrc* SS = ip_sources(P);
  const IpSrc S = SS[find_task_source<1>(SS, P->n_src, task)];
  const int64_t local = task - S.t1;
  const int c = (int)(local / S.n1);
  const int blk = (int)(local - (int64_t)c * S.n1);
  const int logC = 31 - __builtin_clz(S.cols);
  const int C = S.cols, N1 = 1 << S.logN1;
  const int64_t N2 = (int64_t)1 << S.logN2;
  const int64_t c0 = (int64_t)blk * C;
  const void* xs = P->x[c];
  const void* ys = P->y[c];
  // element (j1, col) at buf[j1 * C + col]: neighbouring lanes read neighbouring samples
  for (int e = threadIdx.x; e < C * N1; e += kIpBlock) {
    const int j1 = e >> logC, col = e & (C - 1);
    const int64_t j = (int64_t)j1 * N2 + c0 + col;
    V z;
    z.x = load_or_zero<T>(xs, S.off, j, S.n);
    z.y = load_or_zero<T>(ys, S.off, j, S.n);
    buf[e] = z;
  }
  __syncthreads();
  lds_fft<T>(buf, S.logN1, logC, 1, C);
  V* W = static_cast<V*>(P->ws) + S.ws + (int64_t)c * ((int64_t)1 << S.logN);
  const int64_t mask = ((int64_t)1 << S.logN) - 1;
  for (int e = threadIdx.x; e < C * N1; e += kIpBlock) {
    const int k1 = e >> logC, col = e & (C - 1);
    const int64_t j2 = c0 + col;
    V z = buf[e];
    if (k1 != 0 && j2 != 0) z = cmul(z, root<T, V>((j2 * k1) & mask, S.logN));
    W[(int64_t)k1 * N2 + j2] = z;
  }
}

__device__ __forceinline__ void block_sum3(double* v, double* red) {
  for (int o = 32; o > 0; o >>= 1) {
    v[0] += __shfl_down(v[0], o, 64);
    v[1] += __shfl_down(v[1], o, 64);
    v[2] += __shfl_down(v[2], o, 64);
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    red[3 * w] = v[0];
    red[3 * w + 1] = v[1];
    red[3 * w + 2] = v[2];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kIpBlock / 64; ++i) {
      v[0] += red[3 * i];
      v[1] += red[3 * i + 1];
      v[2] += red[3 * i + 2];
    }
  }
}

// Pass 2: rows k1 and N1 - k1 of one channel (or the whole series when
// N1 = 1), then the weighted sums over the bins 0 < k < N/2 they hold.
template <typename T>
__global__ void __launch_bounds__(kIpBlock) k_ip_pass2(const IpParams* __restrict__ P) {
  using V = typename Cplx<T>::V;
  __shared__ V buf[elems_of<T>()];
  __shared__ double red[3 * (kIpBlock / 64)];
  const int64_t task = blockIdx.x;
  if (task >= P->n_t2) return;
  const IpSrc* SS = ip_sources(P);
  const IpSrc S = SS[find_task_source<2>(SS, P->n_src, task)];
  const int64_t local = task - S.t2;
  const int c = (int)(local / S.n2);
  const int i = (int)(local - (int64_t)c * S.n2);
  const int N1 = 1 << S.logN1, N2 = 1 << S.logN2;
  const int64_t N = (int64_t)1 << S.logN;
  const int r0 = i, r1 = (N1 - i) & (N1 - 1);
  const int B = r0 == r1 ? 1 : 2;
  if (N1 == 1) {
    const void* xs = P->x[c];
    const void* ys = P->y[c];
    for (int e = threadIdx.x; e < N2; e += kIpBlock) {
      V z;
      z.x = load_or_zero<T>(xs, S.off, e, S.n);
      z.y = load_or_zero<T>(ys, S.off, e, S.n);
      buf[e] = z;
    }
  } else {
    const V* W = static_cast<const V*>(P->ws) + S.ws + (int64_t)c * N;
    for (int e = threadIdx.x; e < B * N2; e += kIpBlock) {
      const int b = e >> S.logN2, k2 = e & (N2 - 1);
      buf[e] = W[(int64_t)(b == 0 ? r0 : r1) * N2 + k2];
    }
  }
  __syncthreads();
  lds_fft<T>(buf, S.logN2, B == 2 ? 1 : 0, N2, 1);
  // bins: row b holds k = k1b + N1 k2; the partner N - k lies in the other row
  // at N2 - 1 - k2 (k1b != 0), or in row 0 itself at (N2 - k2) mod N2 (k1b = 0)
  const double* winv = P->winv + (c < 2 ? 0 : P->kmax + 1);
  const int shift = P->logNmax - S.logN;
  const double Ndt = (double)N * P->dt;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int e = threadIdx.x; e < B * N2; e += kIpBlock) {
    const int b = e >> S.logN2, k2 = e & (N2 - 1);
    const int k1b = b == 0 ? r0 : r1;
    const int64_t k = (int64_t)k1b + (int64_t)N1 * k2;
    if (k < 1 || 2 * k >= N) continue;
    const double f = (double)k / Ndt;
    if (f < P->f_min || f > P->f_max) continue;
    int pb, pk2;
    if (k1b == 0) {
      pb = b;
      pk2 = (N2 - k2) & (N2 - 1);
    } else {
      pb = B == 1 ? b : 1 - b;
      pk2 = N2 - 1 - k2;
    }
    const V z = buf[e];
    const V p = buf[(pb << S.logN2) + pk2];
    const double w = winv[k << shift];
    const double ax = (double)z.x + (double)p.x, ay = (double)z.y - (double)p.y;
    const double bx = (double)z.x - (double)p.x, by = (double)z.y + (double)p.y;
    acc[0] += w * (ax * ax + ay * ay);
    acc[1] += w * ((double)z.x * (double)p.y + (double)z.y * (double)p.x);
    acc[2] += w * (bx * bx + by * by);
  }
  block_sum3(acc, red);
  if (threadIdx.x == 0) {
    double* o = P->part + 3 * (S.part + (int64_t)c * S.n2 + i);
    o[0] = acc[0];
    o[1] = acc[1];
    o[2] = acc[2];
  }
}

// Per source and channel: sum the pass-2 partials in task order and scale,
// <x|x> = dt/N sum w |Z + conj P|^2, <x|y> = 2 dt/N sum w Im(Z P),
// <y|y> = dt/N sum w |Z - conj P|^2.
__global__ void __launch_bounds__(kIpBlock) k_ip_reduce(const IpParams* __restrict__ P) {
  const int64_t id = (int64_t)blockIdx.x * kIpBlock + threadIdx.x;
  if (id >= 9 * P->n_src) return;
  const int64_t s = id / 9;
  const int cq = (int)(id - 9 * s), c = cq / 3, q = cq - 3 * c;
  const IpSrc S = ip_sources(P)[s];
  double sum = 0.0;
  const double* part = P->part + 3 * (S.part + (int64_t)c * S.n2) + q;
  for (int i = 0; i < S.n2; ++i) sum += part[3 * i];
  const double scale = (q == 1 ? 2.0 : 1.0) * P->dt / (double)((int64_t)1 << S.logN);
  P->out[id] = S.n2 > 0 ? sum * scale : 0.0;
}

}  // namespace

int launch_pass1(const IpParams* dp, int fp64, int64_t tasks, void* stream) {
  if (tasks <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  if (fp64) hipLaunchKernelGGL(k_ip_pass1<double>, dim3((unsigned)tasks), dim3(kIpBlock), 0, st, dp);
  else hipLaunchKernelGGL(k_ip_pass1<float>, dim3((unsigned)tasks), dim3(kIpBlock), 0, st, dp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pass2(const IpParams* dp, int fp64, int64_t tasks, void* stream) {
  if (tasks <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  if (fp64) hipLaunchKernelGGL(k_ip_pass2<double>, dim3((unsigned)tasks), dim3(kIpBlock), 0, st, dp);
  else hipLaunchKernelGGL(k_ip_pass2<float>, dim3((unsigned)tasks), dim3(kIpBlock), 0, st, dp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_reduce(const IpParams* dp, int64_t n_src, void* stream) {
  if (n_src <= 0) return 0;
  const int64_t blocks = (9 * n_src + kIpBlock - 1) / kIpBlock;
  hipLaunchKernelGGL(k_ip_reduce, dim3((unsigned)blocks), dim3(kIpBlock), 0, (hipStream_t)stream, dp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tdi_ip
