// Radix-2 complex FFT over lines held in LDS, for FP32 and FP64.
//
// The lines are stored contiguously (line l at buf + l*N) in bit-reversed
// order; each stage applies the butterflies x0 +- w x1 with w = exp(-+2 pi i
// k / (2 half)).  The whole workgroup cooperates; the call ends with a barrier.
#pragma once

#include <hip/hip_runtime.h>

namespace ca {

template <typename T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

template <typename C>
__device__ __forceinline__ C cmul_conj(C a, C b) {  // a * conj(b)
  C r;
  r.x = a.x * b.x + a.y * b.y;
  r.y = a.y * b.x - a.x * b.y;
  return r;
}

__device__ __forceinline__ int bitrev(int x, int logn) {
  return (int)(__brev((unsigned)x) >> (32 - logn));
}

// In-place FFT of `lines` lines of length N (bit-reversed input order), with
// twiddles from a table of a larger power-of-two length M = N * tw_scale,
// tw[m] = exp(-2 pi i m / M).  inverse = true uses exp(+2 pi i ...) (no 1/N).
template <typename C>
__device__ void fft_lines(C* buf, int N, int logN, int lines, const C* __restrict__ tw,
                          int tw_scale, bool inverse) {
  const int halfN = N >> 1;
  const int total = lines * halfN;
  for (int s = 0; s < logN; ++s) {
    const int half = 1 << s;
    const int stride = (halfN >> s) * tw_scale;  // M / (2 half)
    for (int b = threadIdx.x; b < total; b += blockDim.x) {
      const int line = b / halfN;
      const int j = b - line * halfN;
      const int k = j & (half - 1);
      const int grp = j >> s;
      const int i0 = line * N + grp * 2 * half + k;
      const int i1 = i0 + half;
      C w = tw[k * stride];
      if (inverse) w.y = -w.y;
      C a = buf[i0];
      C t = cmul(w, buf[i1]);
      C o0, o1;
      o0.x = a.x + t.x; o0.y = a.y + t.y;
      o1.x = a.x - t.x; o1.y = a.y - t.y;
      buf[i0] = o0;
      buf[i1] = o1;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int ilog2(int n) { return 31 - __clz(n); }

}  // namespace ca
