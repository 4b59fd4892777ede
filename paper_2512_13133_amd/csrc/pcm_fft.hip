// Per-pair phase-correlation surface by FFT (paper Sec. 3.2.1(1), Eqs. 3-5),
// one workgroup per unordered pair, FP32 or FP64.
//
// K r(s) = Re sum_u sum_{v <= N/2} h(v) R(u, v) exp(2 pi i (u dy + v dx)/N),
// R = W_mem conj(W_rep), h = 1 on the v = 0 and v = N/2 columns and 2
// elsewhere (R is Hermitian, so the other half-plane is the conjugate).  The
// inverse transform is pruned to the window: a length-N inverse FFT along v
// for every row u keeps only the window columns dx (T(u, dx) in LDS), then a
// length-N inverse FFT along u for every kept column keeps only the window
// rows.  The surface covers the union of both directions' windows, so one
// surface serves both directions: the reverse pair sees r_rev(s) = r(-s).
//
// Modes
//   MODE_LOW     (FP32): per direction, the window maximum and the runner-up;
//                a direction whose gap is below `band` (normalised units) is
//                queued for the FP64 re-decision, the others are final.
//   MODE_EXACT   (FP64): the exact tie rule for both directions.
//   MODE_RESCORE (FP64): the exact tie rule for the queued directions only.
#include "fft_common.h"
#include "kernels.h"
#include "pair_common.h"

namespace ca {

template <typename T>
__global__ void __launch_bounds__(256)
pcm_fft_kernel(ClipsDev cr, ClipsDev cm, PairIO io, const int64_t* __restrict__ list, int mode, Threshold thr,
               double band, const typename cplx<T>::type* __restrict__ tw256, int CH, int LINES,
               int Lmax, RescoreQueue q, int64_t n_blocks, const unsigned long long* __restrict__ n_dev) {
  using C = typename cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int ired[256];
  __shared__ T vred1[256];
  __shared__ T vred2[256];
  __shared__ int idxred[256];
  __shared__ uint64_t keyred[256];

  // grid-stride over the pairs (or listed pairs); the count comes from the
  // host, or from device memory (capped by n_blocks) when n_dev is given
  const int64_t nb_eff = n_dev ? min((int64_t)*n_dev, n_blocks) : n_blocks;
  for (int64_t b = blockIdx.x; b < nb_eff; b += gridDim.x) {
  const int64_t k = list ? list[b] : b;
  const int tid = threadIdx.x;
  const int j = io.rep[k], i = io.mem[k];
  const int N = cm.N[i];
  const int logN = ilog2(N);
  const int H = N / 2;
  const int wf = cm.w[i], wr = cr.w[j];
  const int n_i = cm.npix[i], n_j = cr.npix[j];
  const int dirs = (mode == MODE_RESCORE) ? (int)q.need[k] : 3;

  if (mode != MODE_RESCORE && tid == 0) {
    io.bits[k] = 0;
    io.flags[k] = 0;
    if (q.need) q.need[k] = 0;
  }
  if (n_i == 0 || n_j == 0) {
    if (tid == 0) {
      write_direction(io, k, 0, 0, 0, 0, 0.0, false);
      write_direction(io, k, 1, 0, 0, 0, 0.0, false);
      io.flags[k] |= CA_FLAG_EMPTY;
    }
    continue;
  }

  C* Tbuf = reinterpret_cast<C*>(smem);
  C* lines = Tbuf + (size_t)N * CH;
  T* surf = reinterpret_cast<T*>(lines + (size_t)LINES * N);

  const Axis ax = make_axis(max(wf, wr), N);
  const int L = ax.L;
  const int tws = 256 / N;
  const C* Wi;
  const C* Wj;
  if constexpr (sizeof(T) == 4) {
    Wi = reinterpret_cast<const C*>(cm.spec32 + cm.spec_off[i]);
    Wj = reinterpret_cast<const C*>(cr.spec32 + cr.spec_off[j]);
  } else {
    Wi = reinterpret_cast<const C*>(cm.spec64 + cm.spec_off[i]);
    Wj = reinterpret_cast<const C*>(cr.spec64 + cr.spec_off[j]);
  }
  const int Hs = H + 1;  // stored half-spectrum columns

  int kcount = 0;
  for (int c0 = 0; c0 < L; c0 += CH) {
    const int ncol = min(CH, L - c0);
    // step 1: rows u -> T(u, dx) for the chunk's window columns
    for (int u0 = 0; u0 < N; u0 += LINES) {
      const int nl = min(LINES, N - u0);
      for (int t = tid; t < nl * N; t += blockDim.x) {
        const int r = t >> logN, v = t & (N - 1);
        const int u = u0 + r;
        C z;
        z.x = 0; z.y = 0;
        if (v <= H) {
          const C a = Wi[(size_t)u * Hs + v];
          const C b = Wj[(size_t)u * Hs + v];
          const bool nz = (a.x != 0 || a.y != 0) && (b.x != 0 || b.y != 0);
          const T h = (v == 0 || v == H) ? T(1) : T(2);
          z = cmul_conj(a, b);
          z.x *= h;
          z.y *= h;
          if (c0 == 0 && nz) kcount += (v == 0 || v == H) ? 1 : 2;
        }
        lines[r * N + bitrev(v, logN)] = z;
      }
      __syncthreads();
      // inverse FFT along v (twiddles from the N = 256 table at stride 256/N)
      {
        const int total = nl * (N >> 1);
        for (int s = 0; s < logN; ++s) {
          const int half = 1 << s;
          const int stride = ((N >> 1) >> s) * tws;
          for (int b = tid; b < total; b += blockDim.x) {
            const int line = b / (N >> 1);
            const int jj = b - line * (N >> 1);
            const int kk = jj & (half - 1);
            const int i0 = line * N + (jj >> s) * 2 * half + kk;
            const int i1 = i0 + half;
            C w = tw256[kk * stride];
            w.y = -w.y;
            const C a = lines[i0];
            const C tt = cmul(w, lines[i1]);
            lines[i0].x = a.x + tt.x; lines[i0].y = a.y + tt.y;
            lines[i1].x = a.x - tt.x; lines[i1].y = a.y - tt.y;
          }
          __syncthreads();
        }
      }
      for (int t = tid; t < nl * ncol; t += blockDim.x) {
        const int r = t / ncol, l = t - r * ncol;
        int x = (c0 + l - ax.base) % N;
        if (x < 0) x += N;
        Tbuf[(size_t)(u0 + r) * CH + l] = lines[r * N + x];
      }
      __syncthreads();
    }
    // step 2: columns of the chunk -> surface rows of the window
    for (int l0 = 0; l0 < ncol; l0 += LINES) {
      const int nl = min(LINES, ncol - l0);
      for (int t = tid; t < nl * N; t += blockDim.x) {
        const int c = t >> logN, u = t & (N - 1);
        lines[c * N + bitrev(u, logN)] = Tbuf[(size_t)u * CH + l0 + c];
      }
      __syncthreads();
      {
        const int total = nl * (N >> 1);
        for (int s = 0; s < logN; ++s) {
          const int half = 1 << s;
          const int stride = ((N >> 1) >> s) * tws;
          for (int b = tid; b < total; b += blockDim.x) {
            const int line = b / (N >> 1);
            const int jj = b - line * (N >> 1);
            const int kk = jj & (half - 1);
            const int i0 = line * N + (jj >> s) * 2 * half + kk;
            const int i1 = i0 + half;
            C w = tw256[kk * stride];
            w.y = -w.y;
            const C a = lines[i0];
            const C tt = cmul(w, lines[i1]);
            lines[i0].x = a.x + tt.x; lines[i0].y = a.y + tt.y;
            lines[i1].x = a.x - tt.x; lines[i1].y = a.y - tt.y;
          }
          __syncthreads();
        }
      }
      for (int t = tid; t < nl * L; t += blockDim.x) {
        const int c = t / L, ly = t - c * L;
        int y = (ly - ax.base) % N;
        if (y < 0) y += N;
        surf[ly * L + c0 + l0 + c] = lines[c * N + y].x;
      }
      __syncthreads();
    }
  }
  ired[tid] = kcount;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) ired[tid] += ired[tid + s];
    __syncthreads();
  }
  const int K = ired[0];
  __syncthreads();
  // peak values are recorded and compared normalised by the same K_hi as the
  // batched path uses, so the reported error compares like with like
  const double K_hi = (double)(N * N - max(cm.zero_bins[i], cr.zero_bins[j]));

  const uint64_t* bits_i = cm.bits + cm.bits_off[i];
  const uint64_t* bits_j = cr.bits + cr.bits_off[j];

  for (int d = 0; d < 2; ++d) {
    if (!(dirs & (1 << d))) continue;
    const int wd = d == 0 ? wf : wr;
    const Axis ad = make_axis(wd, N);
    const int P = ad.L * ad.L;
    const uint64_t* brep = d == 0 ? bits_j : bits_i;
    const uint64_t* bmem = d == 0 ? bits_i : bits_j;
    const int nm = d == 0 ? n_i : n_j, nr = d == 0 ? n_j : n_i;
    // value of direction-d shift at window position p
    auto value = [&](int p, int& dy, int& dx) -> T {
      const int ly = p / ad.L, lx = p - ly * ad.L;
      dy = ly - ad.base;
      dx = lx - ad.base;
      int fy = dy, fx = dx;
      if (d == 1) { fy = neg_rep(dy, N); fx = neg_rep(dx, N); }
      return surf[(fy + ax.base) * L + (fx + ax.base)];
    };
    // window maximum (and runner-up for the low-precision decision)
    T v1 = -1e30, v2 = -1e30;
    int i1 = 0x7fffffff;
    for (int p = tid; p < P; p += blockDim.x) {
      int dy, dx;
      const T v = value(p, dy, dx);
      if (v > v1) { v2 = v1; v1 = v; i1 = p; }
      else if (v > v2) v2 = v;
    }
    vred1[tid] = v1; vred2[tid] = v2; idxred[tid] = i1;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        const T a1 = vred1[tid], a2 = vred2[tid], b1 = vred1[tid + s], b2 = vred2[tid + s];
        const int ai = idxred[tid], bi = idxred[tid + s];
        if (a1 > b1 || (a1 == b1 && ai < bi)) {
          vred2[tid] = a2 > b1 ? a2 : b1;
        } else {
          vred1[tid] = b1; idxred[tid] = bi;
          vred2[tid] = b2 > a1 ? b2 : a1;
        }
      }
      __syncthreads();
    }
    const T top = vred1[0], second = vred2[0];
    const int topi = idxred[0];
    __syncthreads();

    if (mode == MODE_LOW) {
      int dy, dx;
      (void)value(topi, dy, dx);
      const int c = block_overlap(brep, bmem, N, dy, dx, ired);
      const bool decided = (double)(top - second) >= band * (double)K;
      if (tid == 0) {
        write_direction(io, k, d, dy, dx, c, cosine_score(c, nm, nr), cosine_bit(c, nm, nr, thr));
        if (!decided && q.need) {
          const uint8_t old = q.need[k];
          q.need[k] = (uint8_t)(old | (1u << d));
          q.r1_low[k * 2 + d] = (float)((double)top / K_hi);
          if (old == 0) {
            const unsigned long long pos = atomicAdd(q.len, 1ull);
            q.list[pos] = k;
          }
        }
      }
      __syncthreads();
      continue;
    }

    // exact tie rule: every shift within TAU of the maximum, then larger c,
    // smaller |dy|+|dx|, lexicographically smaller (dy, dx) -- one integer key
    // per candidate whose maximum is the winner (a running comparison with
    // nested branches is a pattern the compiler has mistranslated here).
    // Each thread counts the overlap of its own window positions, so pairs
    // with many near-tied shifts (periodic patterns) evaluate them in parallel.
    const T cut = top - (T)(TAU * (double)K);
    uint64_t best_key = 0;
    for (int p = tid; p < P; p += blockDim.x) {
      int dy, dx;
      if (value(p, dy, dx) >= cut) best_key = max(best_key, tie_key(thread_overlap(brep, bmem, N, dy, dx), dy, dx));
    }
    keyred[tid] = best_key;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) keyred[tid] = max(keyred[tid], keyred[tid + s]);
      __syncthreads();
    }
    best_key = keyred[0];
    __syncthreads();
    int best_c, best_dy, best_dx;
    tie_decode(best_key, best_c, best_dy, best_dx);
    if (tid == 0) {
      write_direction(io, k, d, best_dy, best_dx, best_c, cosine_score(best_c, nm, nr),
                      cosine_bit(best_c, nm, nr, thr));
      if (mode == MODE_RESCORE) {
        io.flags[k] |= (d == 0) ? CA_FLAG_RESCORED_FWD : CA_FLAG_RESCORED_REV;
        const double err = fabs((double)top / K_hi - (double)q.r1_low[k * 2 + d]);
        atomicMax(q.peak_err_bits, (unsigned long long)__double_as_longlong(err));
        if (q.peak_ratio_bits)
          atomicMax(q.peak_ratio_bits, (unsigned long long)__double_as_longlong(err * sqrt(K_hi)));
      }
    }
    __syncthreads();
  }
  }
}

size_t pcm_fft_smem(int scalar_bytes, int N, int CH, int LINES, int Lmax) {
  const size_t c = 2 * (size_t)scalar_bytes;
  return (size_t)N * CH * c + (size_t)LINES * N * c + (size_t)Lmax * Lmax * scalar_bytes;
}

template <typename T>
static hipError_t launch_pcm_fft_t(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, const int64_t* list,
                                   int64_t n_blocks, int mode, Threshold thr, double band,
                                   const typename cplx<T>::type* tw256, int CH, int LINES, int Lmax,
                                   int maxN, const RescoreQueue& q, const unsigned long long* n_dev,
                                   hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  const size_t smem = pcm_fft_smem((int)sizeof(T), maxN, CH, LINES, Lmax);
  // the dynamic LDS limit is raised once to the largest size seen (not a
  // stream operation, so it stays out of captured sequences once set)
  static size_t smem_set = 0;
  if (smem > smem_set) {
    const hipError_t e = hipFuncSetAttribute((const void*)pcm_fft_kernel<T>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    smem_set = smem;
  }
  // a device-side count is a rare queue: a small grid strides over it
  const unsigned grid = (unsigned)std::min<int64_t>(n_blocks, n_dev ? 2048 : LAUNCH_CHUNK);
  hipLaunchKernelGGL(pcm_fft_kernel<T>, dim3(grid), dim3(256), smem, s, cr, cm, io, list, mode, thr, band, tw256,
                     CH, LINES, Lmax, q, n_blocks, n_dev);
  return hipGetLastError();
}

hipError_t launch_pcm_fft32(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, const int64_t* list, int64_t n_blocks,
                            int mode, Threshold thr, double band, const float2* tw256, int CH,
                            int LINES, int Lmax, int maxN, const RescoreQueue& q, hipStream_t s,
                            const unsigned long long* n_dev) {
  return launch_pcm_fft_t<float>(cr, cm, io, list, n_blocks, mode, thr, band, tw256, CH, LINES, Lmax, maxN, q, n_dev, s);
}

hipError_t launch_pcm_fft64(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, const int64_t* list, int64_t n_blocks,
                            int mode, Threshold thr, double band, const double2* tw256, int CH,
                            int LINES, int Lmax, int maxN, const RescoreQueue& q, hipStream_t s,
                            const unsigned long long* n_dev) {
  return launch_pcm_fft_t<double>(cr, cm, io, list, n_blocks, mode, thr, band, tw256, CH, LINES, Lmax, maxN, q, n_dev, s);
}

}  // namespace ca
