// Per-clip spectra and whitening (paper Sec. 3.2.1(1), Eqs. 3-4).
//
// F = unnormalised forward 2-D DFT of the binary raster, computed in FP64 by
// a row pass (row_fft_kernel: raster rows -> F_row[y][v], v <= N/2) and a
// column pass (col_fft_kernel: F_row[.][v] -> F[u][v]) through a device
// scratch buffer.  Each bin is whitened on its own, W = F/|F| where
// |F| > EPS and 0 elsewhere, so the cross-power spectrum of any pair is
// W_mem * conj(W_rep) -- Eq. 4 wherever both bins are non-zero.  The FP64
// decision |F| > EPS is the same one the FP64 definition takes.  W is stored
// as FP16 (always) and as FP32 / FP64 (on request).
#include "fft_common.h"
#include "kernels.h"

namespace ca {

// grid: (clips in batch, N / rows_per_block), block 256
__global__ void __launch_bounds__(256) row_fft_kernel(ClipsDev cs, const int64_t* __restrict__ ids,
                                                      int N, double2* __restrict__ scratch,
                                                      const double2* __restrict__ tw) {
  extern __shared__ double2 lines[];
  const int b = blockIdx.x;
  const int clip = (int)ids[b];
  const int logN = ilog2(N);
  const int rows = SPEC_LINE_ELEMS / N;
  const int y0 = blockIdx.y * rows;
  const int wpr = N / 64;
  const uint64_t* bits = cs.bits + cs.bits_off[clip];
  for (int t = threadIdx.x; t < rows * N; t += blockDim.x) {
    const int r = t / N, x = t - r * N;
    const int y = y0 + r;
    const double v = (double)((bits[y * wpr + (x >> 6)] >> (x & 63)) & 1ull);
    lines[r * N + bitrev(x, logN)] = make_double2(v, 0.0);
  }
  __syncthreads();
  fft_lines(lines, N, logN, rows, tw, 256 / N, false);
  const int H = N / 2 + 1;
  double2* out = scratch + (int64_t)b * N * H;
  for (int t = threadIdx.x; t < rows * H; t += blockDim.x) {
    const int r = t / H, v = t - r * H;
    out[(int64_t)(y0 + r) * H + v] = lines[r * N + v];
  }
}

// grid: (clips in batch, ceil((N/2+1) / cols_per_block)), block 256
__global__ void __launch_bounds__(256) col_fft_kernel(ClipsDev cs, const int64_t* __restrict__ ids,
                                                      int N, const double2* __restrict__ scratch,
                                                      const double2* __restrict__ tw) {
  extern __shared__ double2 lines[];
  __shared__ int zred[256];
  const int b = blockIdx.x;
  const int clip = (int)ids[b];
  const int logN = ilog2(N);
  const int H = N / 2 + 1;
  const int cols = SPEC_LINE_ELEMS / N;
  const int v0 = blockIdx.y * cols;
  const int ncols = min(cols, H - v0);
  const double2* in = scratch + (int64_t)b * N * H;
  for (int t = threadIdx.x; t < ncols * N; t += blockDim.x) {
    const int c = t / N, y = t - c * N;
    lines[c * N + bitrev(y, logN)] = in[(int64_t)y * H + v0 + c];
  }
  __syncthreads();
  fft_lines(lines, N, logN, ncols, tw, 256 / N, false);
  const int64_t so = cs.spec_off[clip];
  int zeros = 0;
  for (int t = threadIdx.x; t < ncols * N; t += blockDim.x) {
    const int c = t / N, u = t - c * N;
    const int v = v0 + c;
    const double2 F = lines[c * N + u];
    const double mag = sqrt(F.x * F.x + F.y * F.y);
    double2 W = make_double2(0.0, 0.0);
    if (mag > EPS) {
      W.x = F.x / mag;
      W.y = F.y / mag;
    } else {
      zeros += (v == 0 || v == N / 2) ? 1 : 2;  // full-grid bins represented
    }
    const __half2 h = __halves2half2(__float2half_rn((float)W.x), __float2half_rn((float)W.y));
    if (v < N / 2) cs.spec16[so + (int64_t)u * (N / 2) + v] = h;
    else cs.spec16[so + (int64_t)N * (N / 2) + u] = h;
    if (cs.spec32) cs.spec32[so + (int64_t)u * H + v] = make_float2((float)W.x, (float)W.y);
    if (cs.spec64) cs.spec64[so + (int64_t)u * H + v] = W;
  }
  zred[threadIdx.x] = zeros;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) zred[threadIdx.x] += zred[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && zred[0]) atomicAdd(cs.zero_bins + clip, zred[0]);
}

// Whitened image img = (1/N) IFFT2(W) = N w (real; w has unit energy per
// nonzero bin, so the values are O(1) and FP16 keeps them).  Two passes over
// the FP64 half-spectrum: inverse FFTs of its columns along u, then per row
// the Hermitian completion G(y, N - v) = conj(G(y, v)) and the inverse FFT
// along v.  grid: (clips in batch, column / row groups), block 256.
__global__ void __launch_bounds__(256) inv_col_kernel(ClipsDev cs, const int64_t* __restrict__ ids, int N,
                                                      double2* __restrict__ scratch,
                                                      const double2* __restrict__ tw) {
  extern __shared__ double2 lines[];
  const int b = blockIdx.x;
  const int clip = (int)ids[b];
  const int logN = ilog2(N);
  const int H = N / 2 + 1;
  const int cols = SPEC_LINE_ELEMS / N;
  const int v0 = blockIdx.y * cols;
  const int ncols = min(cols, H - v0);
  const double2* W = cs.spec64 + cs.spec_off[clip];
  for (int t = threadIdx.x; t < ncols * N; t += blockDim.x) {
    const int c = t / N, u = t - c * N;
    lines[c * N + bitrev(u, logN)] = W[(int64_t)u * H + v0 + c];
  }
  __syncthreads();
  fft_lines(lines, N, logN, ncols, tw, 256 / N, true);
  double2* out = scratch + (int64_t)b * N * H;
  for (int t = threadIdx.x; t < ncols * N; t += blockDim.x) {
    const int c = t / N, y = t - c * N;
    out[(int64_t)y * H + v0 + c] = lines[c * N + y];
  }
}

__global__ void __launch_bounds__(256) inv_row_kernel(ClipsDev cs, const int64_t* __restrict__ ids, int N,
                                                      const double2* __restrict__ scratch,
                                                      const double2* __restrict__ tw) {
  extern __shared__ double2 lines[];
  const int b = blockIdx.x;
  const int clip = (int)ids[b];
  const int logN = ilog2(N);
  const int H = N / 2 + 1;
  const int rows = SPEC_LINE_ELEMS / N;
  const int y0 = blockIdx.y * rows;
  const double2* in = scratch + (int64_t)b * N * H;
  for (int t = threadIdx.x; t < rows * N; t += blockDim.x) {
    const int r = t / N, v = t - r * N;
    const int64_t row = (int64_t)(y0 + r) * H;
    const double2 G = v <= N / 2 ? in[row + v] : make_double2(in[row + N - v].x, -in[row + N - v].y);
    lines[r * N + bitrev(v, logN)] = G;
  }
  __syncthreads();
  fft_lines(lines, N, logN, rows, tw, 256 / N, true);
  __half* img = cs.img16 + cs.img_off[clip];
  const double inv_n = 1.0 / (double)N;
  for (int t = threadIdx.x; t < rows * N; t += blockDim.x) {
    const int r = t / N, x = t - r * N;
    img[(int64_t)(y0 + r) * N + x] = __float2half_rn((float)(lines[r * N + x].x * inv_n));
  }
}

// ---------------------------------------------------------------------------
// 128 x 128 rasters: the whole transform in one workgroup per clip.
//
// Each 128-point line DFT is split as 128 = 8 x 16 (x = r + 16 j, f = k + 8 s):
//   X[k + 8 s] = sum_r w16^{r s} w128^{r k} sum_j x[r + 16 j] w8^{j k},
// an 8-point DFT per r (stage A), the twiddle w128^{r k}, and a 16-point DFT
// per k (stage B), both in registers, in place in LDS.  A line's point q lives
// at slot q + q/16 (one pad slot per 16) so that both stages read LDS without
// bank conflicts; after stage B frequency f sits at slot 17 (f % 8) + f / 8.
// Rows: two real rows p and p + 64 form one complex line z = a_p + i a_{p+64},
// split after the transform by Z(v) and conj Z(-v).  Columns: the 65 columns
// v <= 64 of the row transform.  FP64 throughout, whitening and all stores
// fused; the half-spectrum (65 lines x 136 slots x 16 B) fills 138 KB of LDS.

constexpr int S128_THREADS = 1024;
constexpr int S128_LINE = 136;  // slots per line: 128 points + 8 pad

__device__ __forceinline__ int s128_pt(int q) { return q + (q >> 4); }      // slot of point q
__device__ __forceinline__ int s128_freq(int f) { return 17 * (f & 7) + (f >> 3); }  // slot of frequency f

// twiddles exp(-2 pi i m / 16), m < 8 (cos and sin of multiples of pi/8)
constexpr double C1_16 = 0.92387953251128675613;  // cos(pi/8)
constexpr double S1_16 = 0.38268343236508977173;  // sin(pi/8)
constexpr double R2_2 = 0.70710678118654752440;   // sqrt(2)/2

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// a * exp(-2 pi i m / 16) for a compile-time m < 8
template <int M>
__device__ __forceinline__ double2 ctw16(double2 a) {
  if constexpr (M == 0) return a;
  else if constexpr (M == 4) return make_double2(a.y, -a.x);  // * (-i)
  else {
    constexpr double c = M == 1 ? C1_16 : M == 2 ? R2_2 : M == 3 ? S1_16 : M == 5 ? -S1_16 : M == 6 ? -R2_2 : -C1_16;
    constexpr double sn = M == 1 ? S1_16 : M == 2 ? R2_2 : M == 3 ? C1_16 : M == 5 ? C1_16 : M == 6 ? R2_2 : S1_16;
    // (a.x + i a.y)(c - i sn)
    return make_double2(fma(a.x, c, a.y * sn), fma(a.y, c, -(a.x * sn)));
  }
}

// In-register radix-2 DIF DFT of length L (8 or 16): x in natural order,
// result in bit-reversed order (X[k] at x[bitrev_L(k)]).
template <int L, int LEN = L>
__device__ __forceinline__ void dif_pass(double2 (&x)[L]) {
  if constexpr (LEN >= 2) {
#pragma unroll
    for (int b = 0; b < L; b += LEN) {
#pragma unroll
      for (int i = 0; i < LEN / 2; ++i) {
        const double2 u = x[b + i], t = x[b + i + LEN / 2];
        x[b + i] = cadd(u, t);
        const double2 d = csub(u, t);
        // exp(-2 pi i i / LEN) = exp(-2 pi i (i 16 / LEN) / 16)
        switch (i * (16 / LEN)) {
          case 0: x[b + i + LEN / 2] = ctw16<0>(d); break;
          case 1: x[b + i + LEN / 2] = ctw16<1>(d); break;
          case 2: x[b + i + LEN / 2] = ctw16<2>(d); break;
          case 3: x[b + i + LEN / 2] = ctw16<3>(d); break;
          case 4: x[b + i + LEN / 2] = ctw16<4>(d); break;
          case 5: x[b + i + LEN / 2] = ctw16<5>(d); break;
          case 6: x[b + i + LEN / 2] = ctw16<6>(d); break;
          default: x[b + i + LEN / 2] = ctw16<7>(d); break;
        }
      }
    }
    dif_pass<L, LEN / 2>(x);
  }
}
template <int L>
constexpr int brev_small(int k) {
  int r = 0;
  for (int b = 1; b < L; b <<= 1) r = (r << 1) | ((k & b) ? 1 : 0);
  return r;
}

// Stage A of one line: 8-point DFTs over j of x[r + 16 j], times w128^{r k},
// written back to the same slots (point r + 16 k).
__device__ __forceinline__ void s128_stage_a(double2* line, int r, const double2* w128, const double2 (&in)[8]) {
  double2 x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = in[j];
  dif_pass<8>(x);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double2 X = x[brev_small<8>(k)];
    const double2 w = w128[r * k];
    line[s128_pt(r + 16 * k)] = make_double2(X.x * w.x - X.y * w.y, X.x * w.y + X.y * w.x);
  }
}
// Stage B of one line: the 16-point DFT over r of point r + 16 k; frequency
// k + 8 s is written to point 16 k + s.
__device__ __forceinline__ void s128_stage_b(double2* line, int k) {
  double2 x[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = line[s128_pt(r + 16 * k)];
  dif_pass<16>(x);
#pragma unroll
  for (int t = 0; t < 16; ++t) line[s128_pt(16 * k + t)] = x[brev_small<16>(t)];
}

// grid: one workgroup per clip
__global__ void __launch_bounds__(S128_THREADS) spectrum128_kernel(ClipsDev cs,
                                                                   const int64_t* __restrict__ ids,
                                                                   const double2* __restrict__ tw256) {
  __shared__ double2 buf[65 * S128_LINE];
  __shared__ double2 w128[128];
  __shared__ uint64_t sbits[256];
  __shared__ int zred[S128_THREADS / 64];
  const int tid = threadIdx.x;
  {
    const int clip = (int)ids[blockIdx.x];
    if (tid < 128) {
      // exp(-2 pi i m / 128) from exp(-2 pi i e / 256), e < 128
      const double2 b = tw256[(2 * tid) & 127];
      w128[tid] = tid >= 64 ? make_double2(-b.x, -b.y) : b;
    } else if (tid < 128 + 256) {
      sbits[tid - 128] = cs.bits[cs.bits_off[clip] + (tid - 128)];
    }
    __syncthreads();
    // rows, stage A: line p = rows p (real) and p + 64 (imaginary), task (p, r)
    {
      const int p = tid >> 4, r = tid & 15;
      double2 in[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int x = r + 16 * j;
        in[j] = make_double2((double)((sbits[2 * p + (x >> 6)] >> (x & 63)) & 1ull),
                             (double)((sbits[2 * (p + 64) + (x >> 6)] >> (x & 63)) & 1ull));
      }
      s128_stage_a(buf + p * S128_LINE, r, w128, in);
    }
    __syncthreads();
    if (tid < 64 * 8) s128_stage_b(buf + (tid >> 3) * S128_LINE, tid & 7);
    __syncthreads();
    // split the complex lines into rows p and p + 64 (v <= 64), then store them
    // as the 65 column lines: F_row(y, v) at column v, point y
    constexpr int NSPLIT = (64 * 65 + S128_THREADS - 1) / S128_THREADS;
    double2 ra[NSPLIT], rb[NSPLIT];
#pragma unroll
    for (int t = 0; t < NSPLIT; ++t) {
      const int task = tid + t * S128_THREADS;
      if (task < 64 * 65) {
        const int p = task / 65, v = task - p * 65;
        const double2 zv = buf[p * S128_LINE + s128_freq(v)];
        const double2 zm = buf[p * S128_LINE + s128_freq((128 - v) & 127)];
        ra[t] = make_double2(0.5 * (zv.x + zm.x), 0.5 * (zv.y - zm.y));   // (Z(v) + conj Z(-v)) / 2
        rb[t] = make_double2(0.5 * (zv.y + zm.y), -0.5 * (zv.x - zm.x));  // (Z(v) - conj Z(-v)) / 2i
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NSPLIT; ++t) {
      const int task = tid + t * S128_THREADS;
      if (task < 64 * 65) {
        const int p = task / 65, v = task - p * 65;
        buf[v * S128_LINE + s128_pt(p)] = ra[t];
        buf[v * S128_LINE + s128_pt(p + 64)] = rb[t];
      }
    }
    __syncthreads();
    // columns, stage A: task (v, r), 65 x 16
    for (int task = tid; task < 65 * 16; task += S128_THREADS) {
      const int v = task >> 4, r = task & 15;
      double2* line = buf + v * S128_LINE;
      double2 in[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) in[j] = line[s128_pt(r + 16 * j)];
      s128_stage_a(line, r, w128, in);
    }
    __syncthreads();
    if (tid < 65 * 8) s128_stage_b(buf + (tid >> 3) * S128_LINE, tid & 7);
    __syncthreads();
    // whitening and stores, v fastest: W = F / |F| where |F| > EPS, else 0
    const int64_t so = cs.spec_off[clip];
    int zeros = 0;
    for (int task = tid; task < 128 * 65; task += S128_THREADS) {
      const int u = task / 65, v = task - u * 65;
      const double2 F = buf[v * S128_LINE + s128_freq(u)];
      const double mag = sqrt(F.x * F.x + F.y * F.y);
      double2 W = make_double2(0.0, 0.0);
      if (mag > EPS) {
        W.x = F.x / mag;
        W.y = F.y / mag;
      } else {
        zeros += (v == 0 || v == 64) ? 1 : 2;  // full-grid bins represented
      }
      const __half2 h = __halves2half2(__float2half_rn((float)W.x), __float2half_rn((float)W.y));
      if (cs.spec16) {
        if (v < 64) cs.spec16[so + (int64_t)u * 64 + v] = h;
        else cs.spec16[so + 128 * 64 + u] = h;
      }
      if (cs.spec32) cs.spec32[so + (int64_t)u * 65 + v] = make_float2((float)W.x, (float)W.y);
      if (cs.spec64) cs.spec64[so + (int64_t)u * 65 + v] = W;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) zeros += __shfl_xor(zeros, o);
    if ((tid & 63) == 0) zred[tid >> 6] = zeros;
    __syncthreads();
    if (tid == 0) {
      int z = 0;
      for (int w = 0; w < S128_THREADS / 64; ++w) z += zred[w];
      if (cs.zero_bins) cs.zero_bins[clip] = z;
    }
  }
}

}  // namespace ca

namespace ca {

hipError_t launch_image(const ClipsDev& cs, const int64_t* ids, int64_t n_ids, int N, double2* scratch,
                        const double2* tw256, hipStream_t s) {
  if (n_ids == 0) return hipSuccess;
  const size_t smem = (size_t)SPEC_LINE_ELEMS * sizeof(double2);
  const int lines = SPEC_LINE_ELEMS / N;
  const int H = N / 2 + 1;
  hipLaunchKernelGGL(inv_col_kernel, dim3((unsigned)n_ids, (unsigned)((H + lines - 1) / lines)), dim3(256), smem, s,
                     cs, ids, N, scratch, tw256);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(inv_row_kernel, dim3((unsigned)n_ids, (unsigned)(N / lines)), dim3(256), smem, s, cs, ids, N,
                     (const double2*)scratch, tw256);
  return hipGetLastError();
}

hipError_t launch_spectrum128(const ClipsDev& cs, const int64_t* ids, int64_t n_ids, const double2* tw256,
                              hipStream_t s) {
  if (n_ids == 0) return hipSuccess;
  // one workgroup per clip; 142 KB of LDS each, so one per compute unit at a time
  for (int64_t c0 = 0; c0 < n_ids; c0 += 1ll << 30) {
    const unsigned grid = (unsigned)std::min<int64_t>(n_ids - c0, 1ll << 30);
    hipLaunchKernelGGL(spectrum128_kernel, dim3(grid), dim3(S128_THREADS), 0, s, cs, ids + c0, tw256);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_spectrum(const ClipsDev& cs, const int64_t* ids, int64_t n_ids, int N,
                           double2* scratch, const double2* tw256, hipStream_t s) {
  if (n_ids == 0) return hipSuccess;
  const size_t smem = (size_t)SPEC_LINE_ELEMS * sizeof(double2);
  const int rows = SPEC_LINE_ELEMS / N;
  const int H = N / 2 + 1;
  hipLaunchKernelGGL(row_fft_kernel, dim3((unsigned)n_ids, (unsigned)(N / rows)), dim3(256), smem, s,
                     cs, ids, N, scratch, tw256);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(col_fft_kernel, dim3((unsigned)n_ids, (unsigned)((H + rows - 1) / rows)), dim3(256),
                     smem, s, cs, ids, N, scratch, tw256);
  return hipGetLastError();
}

}  // namespace ca
