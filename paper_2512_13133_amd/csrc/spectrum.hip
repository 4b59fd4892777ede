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

hipError_t launch_spectrum(const ClipsDev& cs, const int64_t* ids, int64_t n_ids, int N,
                           double2* scratch, const double2* tw256, hipStream_t s) {
  if (n_ids == 0) return hipSuccess;
  (void)tw256;
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
