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
// input (float or double); the weighted sums accumulate in double.  Twiddle
// factors are read from tables computed on the host in FP64 and rounded once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tdi_ip_internal.h"

namespace tdi_ip {
namespace {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using V = float2; };
template <> struct Cplx<double> { using V = double2; };


template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
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
__device__ __forceinline__ void dft4r(V& a0, V& a1, V& a2, V& a3) {
  V a[4] = {a0, a1, a2, a3};
  dft4(a);
  a0 = a[0];
  a1 = a[1];
  a2 = a[2];
  a3 = a[3];
}

// 16-point DFT in registers as 4 x 4: transforms over n1 of a[4 n1 + n2], the
// twiddles e^{-2 pi i n2 k1 / 16}, transforms over n2.  X[k1 + 4 k2] ends in
// a[4 k1 + k2], so output k is read from a[4 (k mod 4) + k / 4].
template <typename T, typename V>
__device__ __forceinline__ void dft16(V* a) {
  const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173, h = (T)0.70710678118654752440;
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4r(a[n2], a[4 + n2], a[8 + n2], a[12 + n2]);
  V w;
  w.x = c1; w.y = -s1; a[5] = cmul(a[5], w);      // W^1
  w.x = h; w.y = -h; a[6] = cmul(a[6], w);        // W^2
  a[9] = cmul(a[9], w);
  w.x = s1; w.y = -c1; a[7] = cmul(a[7], w);      // W^3
  a[13] = cmul(a[13], w);
  {                                               // W^4 = -i
    const V t = a[10];
    a[10].x = t.y;
    a[10].y = -t.x;
  }
  w.x = -h; w.y = -h; a[11] = cmul(a[11], w);     // W^6
  a[14] = cmul(a[14], w);
  w.x = -c1; w.y = s1; a[15] = cmul(a[15], w);    // W^9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4r(a[4 * k1], a[4 * k1 + 1], a[4 * k1 + 2], a[4 * k1 + 3]);
}

template <typename V>
__device__ __forceinline__ void dft2(V* a) {
  V t;
  t.x = a[0].x - a[1].x; t.y = a[0].y - a[1].y;
  a[0].x += a[1].x; a[0].y += a[1].y;
  a[1] = t;
}

// LDS layout: logical element i sits at i + i / 32, one pad element per 32, so
// that the strided accesses of the early stages spread over the banks.
template <int E> constexpr int lds_elems() { return E + E / 32; }
__device__ __forceinline__ int lp(int i) { return i + (i >> 5); }

// One Stockham stage of radix R on B sequences of length L = 2^logL held in
// LDS; element e of sequence b sits at logical index (b << lbs) + (e << les).  Ns is the length
// of the sub-transforms already formed.  Butterfly q maps to sequence
// b = q mod B (B = 2^logB) and index j = q / B, so that neighbouring lanes touch
// neighbouring sequences (interleaved layout) or neighbouring elements.
// Twiddles e^{-2 pi i k r / (Ns R)} come from the table tw of e^{-2 pi i m / 2^log_tw}.
// E: complex elements of the tile, BLK: threads of the workgroup.
template <typename T, int R, int E, int BLK>
__device__ __forceinline__ void fft_stage(typename Cplx<T>::V* buf, const typename Cplx<T>::V* __restrict__ tw,
                                          int logL, int logNs, int logB, int lbs, int les) {
  using V = typename Cplx<T>::V;
  constexpr int kMaxQ = E / (R * BLK) > 0 ? E / (R * BLK) : 1;
  constexpr int kLogR = R == 16 ? 4 : (R == 4 ? 2 : 1);
  const int lnb = logL - kLogR;                // log2 butterflies per sequence
  const int total = 1 << (lnb + logB);
  const int Ns = 1 << logNs;
  V v[kMaxQ][R];
#pragma unroll
  for (int i = 0; i < kMaxQ; ++i) {
    const int q = threadIdx.x + i * BLK;
    if (q < total) {
      const int b = q & ((1 << logB) - 1), j = q >> logB;
      const int base = (b << lbs) + (j << les);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[lp(base + (r << (lnb + les)))];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kMaxQ; ++i) {
    const int q = threadIdx.x + i * BLK;
    if (q < total) {
      const int b = q & ((1 << logB) - 1), j = q >> logB;
      const int k = j & (Ns - 1);
      if (logNs > 0) {
        const int step = k << (log_tw<T>() - logNs - kLogR);
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], tw[r * step]);
      }
      const int base = (b << lbs) + ((((j - k) << kLogR) + k) << les);
      if constexpr (R == 16) {
        dft16<T, V>(v[i]);
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[lp(base + (r << (logNs + les)))] = v[i][4 * (r & 3) + (r >> 2)];
      } else {
        if constexpr (R == 4) dft4(v[i]); else dft2(v[i]);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lp(base + (r << (logNs + les)))] = v[i][r];
      }
    }
  }
  __syncthreads();
}

// Forward DFT (e^{-2 pi i j k / L}) of B sequences in place, natural order out.
// FP32: one radix-2 and one radix-4 stage as log2 L mod 4 requires, then radix
// 16 in registers.  FP64 (twice the registers per element): radix 4 after an
// optional radix-2 stage.
template <typename T, int E, int BLK>
__device__ __forceinline__ void lds_fft(typename Cplx<T>::V* buf, const typename Cplx<T>::V* __restrict__ tw,
                                        int logL, int logB, int lbs, int les) {
  int logNs = 0;
  if (logL & 1) {
    fft_stage<T, 2, E, BLK>(buf, tw, logL, 0, logB, lbs, les);
    logNs = 1;
  }
  if constexpr (sizeof(T) == 4) {
    if (logL & 2) {
      fft_stage<T, 4, E, BLK>(buf, tw, logL, logNs, logB, lbs, les);
      logNs += 2;
    }
    while (logNs < logL) {
      fft_stage<T, 16, E, BLK>(buf, tw, logL, logNs, logB, lbs, les);
      logNs += 4;
    }
  } else {
    while (logNs < logL) {
      fft_stage<T, 4, E, BLK>(buf, tw, logL, logNs, logB, lbs, les);
      logNs += 2;
    }
  }
}

// Persistent workgroups: workgroups are dealt to the eight XCDs in turn, so
// XCD x = blockIdx mod 8 owns the x-th eighth of the tasks, and its workgroups
// walk that range together with a stride of their count.  Neighbouring column
// blocks (which share cache lines) are then in flight at the same time in the
// same L2, and a workgroup's owning source only moves forward.  The grid is a
// multiple of 8.
__device__ __forceinline__ void task_span(int64_t nt, int64_t* b, int64_t* e, int64_t* stride) {
  const int64_t px = (nt + 7) >> 3;
  const int64_t x = blockIdx.x & 7;
  *b = x * px + (blockIdx.x >> 3);
  *e = min((x + 1) * px, nt);
  *stride = gridDim.x >> 3;
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
__device__ __forceinline__ void pass1_task(const IpParams* __restrict__ P, const IpSrc& S, int64_t local,
                                           typename Cplx<T>::V* buf) {
  using V = typename Cplx<T>::V;
  using TL = Tile<T, 1>;
  const int c = (int)(local / S.n1);
  const int blk = (int)(local - (int64_t)c * S.n1);
  const int logC = 31 - __builtin_clz(S.cols);
  const int C = S.cols, N1 = 1 << S.logN1;
  const int64_t N2 = (int64_t)1 << S.logN2;
  const int64_t c0 = (int64_t)blk * C;
  const void* xs = P->x[c];
  const void* ys = P->y[c];
  // element (j1, col) at buf[j1 * C + col]: neighbouring lanes read neighbouring
  // samples.  A first-pass task always fills the LDS (C N1 = E): every load of
  // a thread is issued before the first is consumed.
  constexpr int kIt = TL::kE / TL::kBlock;
  constexpr int kG = 4;
#pragma unroll
  for (int h = 0; h < kIt / kG; ++h) {
    V z[kG];
#pragma unroll
    for (int it = 0; it < kG; ++it) {
      const int e = threadIdx.x + (h * kG + it) * TL::kBlock;
      const int j1 = e >> logC, col = e & (C - 1);
      const int64_t j = ((int64_t)j1 << S.logN2) + c0 + col;
      z[it].x = load_or_zero<T>(xs, S.off, j, S.n);
      z[it].y = load_or_zero<T>(ys, S.off, j, S.n);
    }
#pragma unroll
    for (int it = 0; it < kG; ++it) buf[lp(threadIdx.x + (h * kG + it) * TL::kBlock)] = z[it];
  }
  __syncthreads();
  lds_fft<T, TL::kE, TL::kBlock>(buf, static_cast<const V*>(P->tw), S.logN1, logC, 0, logC);
  V* W = static_cast<V*>(P->ws) + S.ws + (int64_t)c * ((int64_t)1 << S.logN);
  const int64_t mask = ((int64_t)1 << S.logN) - 1;
  const int up = P->logNmax - S.logN, tb = P->tbits;
  const V* th = static_cast<const V*>(P->th);
  const V* tl = static_cast<const V*>(P->tl);
  // twiddle loads in groups of four, each issued together
  constexpr int kGT = 4;
#pragma unroll 1
  for (int h = 0; h < kIt / kGT; ++h) {
    V wh[kGT], wl[kGT];
#pragma unroll
    for (int it = 0; it < kGT; ++it) {
      const int e = threadIdx.x + (h * kGT + it) * TL::kBlock;
      const int k1 = e >> logC, col = e & (C - 1);
      // e^{-2 pi i j2 k1 / N} = e^{-2 pi i m / N_max} with m = (j2 k1 mod N) 2^up;
      // j2 < N2 and k1 < N1 are below 2^13: 24-bit operands, the product fits 32 bits
      const int64_t m = ((int64_t)__umul24((unsigned)(c0 + col), (unsigned)k1) & mask) << up;
      wh[it] = th[m >> tb];
      wl[it] = tl[m & ((1 << tb) - 1)];
    }
#pragma unroll
    for (int it = 0; it < kGT; ++it) {
      const int e = threadIdx.x + (h * kGT + it) * TL::kBlock;
      const int k1 = e >> logC, col = e & (C - 1);
      W[((int64_t)k1 << S.logN2) + c0 + col] = cmul(buf[lp(e)], cmul(wh[it], wl[it]));
    }
  }
}

// persistent driver of a pass: walk the workgroup's task range, advancing the
// owning source along it
template <int Pass>
__device__ __forceinline__ int64_t first_task(const IpSrc& s) { return Pass == 1 ? s.t1 : s.t2; }

template <typename T>
__global__ void __launch_bounds__(kBlock1<T>) __attribute__((amdgpu_waves_per_eu(4)))
k_ip_pass1(const IpParams* __restrict__ P) {
  using V = typename Cplx<T>::V;
  __shared__ V buf[lds_elems<Tile<T, 1>::kE>()];
  int64_t t, te, dt;
  task_span(P->n_t1, &t, &te, &dt);
  if (t >= te) return;
  const IpSrc* SS = ip_sources(P);
  const int64_t ns = P->n_src;
  int64_t s = find_task_source<1>(SS, ns, t);
  IpSrc S = SS[s];
  int64_t next = s + 1 < ns ? SS[s + 1].t1 : INT64_MAX;
  for (; t < te; t += dt) {
    while (t >= next) {
      ++s;
      S = SS[s];
      next = s + 1 < ns ? SS[s + 1].t1 : INT64_MAX;
    }
    pass1_task<T>(P, S, t - S.t1, buf);
    __syncthreads();
  }
}

template <int BLK>
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
    for (int i = 1; i < BLK / 64; ++i) {
      v[0] += red[3 * i];
      v[1] += red[3 * i + 1];
      v[2] += red[3 * i + 2];
    }
  }
}

// Pass 2: rows k1 and N1 - k1 of one channel (or the whole series when
// N1 = 1), then the weighted sums over the bins 0 < k < N/2 they hold.
template <typename T>
__device__ __forceinline__ void pass2_task(const IpParams* __restrict__ P, const IpSrc& S, int64_t local,
                                           typename Cplx<T>::V* buf, double* red) {
  using V = typename Cplx<T>::V;
  using TL = Tile<T, 2>;
  const int c = (int)(local / S.n2);
  const int i = (int)(local - (int64_t)c * S.n2);
  const int N1 = 1 << S.logN1, N2 = 1 << S.logN2;
  const int64_t N = (int64_t)1 << S.logN;
  const int r0 = i, r1 = (N1 - i) & (N1 - 1);
  const int B = r0 == r1 ? 1 : 2;
  // every load of a thread is issued before the first is consumed
  constexpr int kIt = TL::kE / TL::kBlock;
  const int cnt = B << S.logN2;
  {
    V z[kIt];
    // the loads go out ahead of the transform of the other resident workgroup
    __builtin_amdgcn_s_setprio(1);
    if (N1 == 1) {
      const void* xs = P->x[c];
      const void* ys = P->y[c];
#pragma unroll
      for (int it = 0; it < kIt; ++it) {
        const int e = threadIdx.x + it * TL::kBlock;
        z[it].x = load_or_zero<T>(xs, S.off, e, S.n);
        z[it].y = load_or_zero<T>(ys, S.off, e, S.n);
      }
    } else {
      const V* W = static_cast<const V*>(P->ws) + S.ws + (int64_t)c * N;
#pragma unroll
      for (int it = 0; it < kIt; ++it) {
        const int e = threadIdx.x + it * TL::kBlock;
        if (e < cnt) {
          const int b = e >> S.logN2, k2 = e & (N2 - 1);
          z[it] = W[((int64_t)(b == 0 ? r0 : r1) << S.logN2) + k2];
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int e = threadIdx.x + it * TL::kBlock;
      if (e < cnt) buf[lp(e)] = z[it];
    }
  }
  __syncthreads();
  lds_fft<T, TL::kE, TL::kBlock>(buf, static_cast<const V*>(P->tw), S.logN2, B == 2 ? 1 : 0, S.logN2, 0);
  // bins: row b holds k = k1b + N1 k2; the partner N - k lies in the other row
  // at N2 - 1 - k2 (k1b != 0), or in row 0 itself at (N2 - k2) mod N2 (k1b = 0)
  // weight of bin k = k1b + N1 k2 (k < N/2 means k2 < N2/2): wt[k1b N2/2 + k2]
  const T* wt = static_cast<const T*>(P->wt) + S.wofs + (c < 2 ? 0 : N / 2);
  double acc[3] = {0.0, 0.0, 0.0};
  // weights in groups of eight, each group's loads issued together
  constexpr int kG = 8;
#pragma unroll
  for (int g = 0; g < kIt / kG; ++g) {
    T wk[kG];
#pragma unroll
    for (int it = 0; it < kG; ++it) {
      const int e = threadIdx.x + (g * kG + it) * TL::kBlock;
      const int b = e >> S.logN2, k2 = e & (N2 - 1);
      const int k1b = b == 0 ? r0 : r1;
      const int64_t k = (int64_t)k1b + ((int64_t)k2 << S.logN1);
      wk[it] = (e < cnt && k >= 1 && 2 * k < N) ? wt[((int64_t)k1b << (S.logN2 - 1)) + k2] : (T)0;
    }
#pragma unroll
    for (int it = 0; it < kG; ++it) {
      const int e = threadIdx.x + (g * kG + it) * TL::kBlock;
      const double w = (double)wk[it];
      if (w == 0.0) continue;          // outside the band, or not a bin 0 < k < N/2 of this task
      const int b = e >> S.logN2, k2 = e & (N2 - 1);
      const int k1b = b == 0 ? r0 : r1;
      int pb, pk2;
      if (k1b == 0) {
        pb = b;
        pk2 = (N2 - k2) & (N2 - 1);
      } else {
        pb = B == 1 ? b : 1 - b;
        pk2 = N2 - 1 - k2;
      }
      const V z = buf[lp(e)];
      const V p = buf[lp((pb << S.logN2) + pk2)];
      const double ax = (double)z.x + (double)p.x, ay = (double)z.y - (double)p.y;
      const double bx = (double)z.x - (double)p.x, by = (double)z.y + (double)p.y;
      acc[0] += w * (ax * ax + ay * ay);
      acc[1] += w * ((double)z.x * (double)p.y + (double)z.y * (double)p.x);
      acc[2] += w * (bx * bx + by * by);
    }
  }
  block_sum3<TL::kBlock>(acc, red);
  if (threadIdx.x == 0) {
    double* o = P->part + 3 * (S.part + (int64_t)c * S.n2 + i);
    o[0] = acc[0];
    o[1] = acc[1];
    o[2] = acc[2];
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock2<T>) __attribute__((amdgpu_waves_per_eu(4)))
k_ip_pass2(const IpParams* __restrict__ P) {
  using V = typename Cplx<T>::V;
  __shared__ V buf[lds_elems<Tile<T, 2>::kE>()];
  __shared__ double red[3 * (Tile<T, 2>::kBlock / 64)];
  int64_t t, te, dt;
  task_span(P->n_t2, &t, &te, &dt);
  if (t >= te) return;
  const IpSrc* SS = ip_sources(P);
  const int64_t ns = P->n_src;
  int64_t s = find_task_source<2>(SS, ns, t);
  IpSrc S = SS[s];
  int64_t next = s + 1 < ns ? SS[s + 1].t2 : INT64_MAX;
  for (; t < te; t += dt) {
    while (t >= next) {
      ++s;
      S = SS[s];
      next = s + 1 < ns ? SS[s + 1].t2 : INT64_MAX;
    }
    pass2_task<T>(P, S, t - S.t2, buf, red);
    __syncthreads();
  }
}

// Per source and channel: sum the pass-2 partials in task order and scale,
// <x|x> = dt/N sum w |Z + conj P|^2, <x|y> = 2 dt/N sum w Im(Z P),
// <y|y> = dt/N sum w |Z - conj P|^2.
__global__ void __launch_bounds__(kReduceBlock) k_ip_reduce(const IpParams* __restrict__ P) {
  const int64_t id = (int64_t)blockIdx.x * kReduceBlock + threadIdx.x;
  if (id >= 9 * P->n_src) return;
  const int64_t s = id / 9;
  const int cq = (int)(id - 9 * s), c = cq / 3, q = cq - 3 * c;
  const IpSrc S = ip_sources(P)[s];
  double sum = 0.0;
  const double* part = P->part + 3 * (S.part + (int64_t)c * S.n2) + q;
  for (int i = 0; i < S.n2; ++i) sum += part[3 * i];
  const double scale = ldexp((q == 1 ? 2.0 : 1.0) * P->dt / (double)((int64_t)1 << S.logN), P->wexp);
  P->out[id] = S.n2 > 0 ? sum * scale : 0.0;
}

}  // namespace

int launch_pass1(const IpParams* dp, int fp64, int64_t tasks, int grid, void* stream) {
  if (tasks <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  tasks = std::min<int64_t>((tasks + 7) & ~(int64_t)7, grid);
  if (fp64) hipLaunchKernelGGL(k_ip_pass1<double>, dim3((unsigned)tasks), dim3(Tile<double, 1>::kBlock), 0, st, dp);
  else hipLaunchKernelGGL(k_ip_pass1<float>, dim3((unsigned)tasks), dim3(Tile<float, 1>::kBlock), 0, st, dp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pass2(const IpParams* dp, int fp64, int64_t tasks, int grid, void* stream) {
  if (tasks <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  tasks = std::min<int64_t>((tasks + 7) & ~(int64_t)7, grid);
  if (fp64) hipLaunchKernelGGL(k_ip_pass2<double>, dim3((unsigned)tasks), dim3(Tile<double, 2>::kBlock), 0, st, dp);
  else hipLaunchKernelGGL(k_ip_pass2<float>, dim3((unsigned)tasks), dim3(Tile<float, 2>::kBlock), 0, st, dp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_reduce(const IpParams* dp, int64_t n_src, void* stream) {
  if (n_src <= 0) return 0;
  const int64_t blocks = (9 * n_src + kReduceBlock - 1) / kReduceBlock;
  hipLaunchKernelGGL(k_ip_reduce, dim3((unsigned)blocks), dim3(kReduceBlock), 0, (hipStream_t)stream, dp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tdi_ip
