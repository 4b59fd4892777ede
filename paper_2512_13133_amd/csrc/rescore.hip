// FP64 re-decision of near-tied window peaks (paper Eq. 5 evaluated term by
// term; tie rule of the library documentation).
//
// The low-precision kernel queues a direction whose top-2 gap is below the
// band (2 e + TAU, e the low-precision surface error) together with every
// window shift whose low-precision value lies within the band of its maximum.
// Those candidates contain the true maximum and every shift tied with it, so
// the exact decision only needs r(s) at them:
//   K r(s) = Re sum_u sum_{v <= N/2} h(v) W_mem(u, v) conj(W_rep(u, v)) e^{2 pi i (u dy + v dx)/N},
// summed in FP64 from the FP64 whitened spectra, K = the number of full-grid
// bins where both spectra are non-zero.  Shifts within TAU of the best are
// tied; the larger overlap count c wins, then the smaller |dy|+|dx|, then the
// lexicographically smaller (dy, dx).
//
// A group of both directions (equal windows) holds forward shifts.  The
// reverse direction's value and overlap count at -s equal the forward ones at
// s, so the sums and counts serve both; only the lexicographic tie-break is
// taken in each direction's own coordinates.
#include "kernels.h"
#include "pair_common.h"

namespace ca {

constexpr int RS_THREADS = 256;


// Sum over the wave, by a butterfly whose partial sums are the same in every
// lane (fixed order, so the result is deterministic).
__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ int wave_sum_i32(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// One workgroup per candidate group (grid-stride over the groups, whose count
// is read on the device).  Every thread accumulates all candidates over its
// share of the bins; the sums, the bin count K and the overlap counts of the
// candidates are reduced per wave and then over the four waves in a fixed
// order, with three workgroup barriers per group.
__global__ void __launch_bounds__(RS_THREADS)
rescore_candidates_kernel(ClipsDev cr, ClipsDev cm, PairIO io, Threshold thr, CandQueue cq,
                          const double2* __restrict__ tw256, unsigned long long* peak_err_bits,
                          unsigned long long* peak_ratio_bits, const float* __restrict__ r1_low) {
  constexpr int WAVES = RS_THREADS / 64;
  __shared__ double s_part[WAVES][MAX_CAND];
  __shared__ int s_kpart[WAVES];
  __shared__ int s_cpart[WAVES][MAX_CAND];
  __shared__ double2 tw[256];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int twN = 0;  // raster size the twiddle table holds (workgroup-uniform)
  const int64_t n_groups = min((int64_t)*cq.n_groups, cq.cap_groups);
  for (int64_t gi = blockIdx.x; gi < n_groups; gi += gridDim.x) {
    const CandGroup gr = cq.groups[gi];
    const int m = gr.count;
    if (m == 0) continue;
    const int64_t k = gr.pair;
    const int d = gr.dir;
    const int j = io.rep[k], i = io.mem[k];
    const int N = cm.N[i];
    const int H = N / 2;
    __syncthreads();  // the previous group's reads of the shared arrays are done
    if (N != twN) {
      // tw[t] = exp(-2 pi i t / N) from the half-circle table exp(-2 pi i m / 256), m < 128
      const int tws = 256 / N;
      for (int t = tid; t < N; t += RS_THREADS) {
        const double2 base = tw256[(t * tws) & 127];
        tw[t] = (t * tws) >= 128 ? make_double2(-base.x, -base.y) : base;
      }
      twN = N;
      __syncthreads();
    }
    const double2* Wi = cm.spec64 + cm.spec_off[i];
    const double2* Wj = cr.spec64 + cr.spec_off[j];
    // forward shifts of the candidates (direction 1 reads the mirrored surface)
    int fy[MAX_CAND], fx[MAX_CAND];
    double acc[MAX_CAND];
#pragma unroll
    for (int c = 0; c < MAX_CAND; ++c) {
      const int16_t sh = c < m ? cq.shifts[gr.offset + c] : (int16_t)0;
      const int sy = (int8_t)(sh >> 8), sx = (int8_t)(sh & 0xff);
      fy[c] = d == 1 ? -sy : sy;
      fx[c] = d == 1 ? -sx : sx;
      acc[c] = 0.0;
    }
    int kc = 0;
    const int bins = N * (H + 1);
    for (int b = tid; b < bins; b += RS_THREADS) {
      const int u = b / (H + 1), v = b - u * (H + 1);
      const double2 a = Wi[b], w = Wj[b];
      if ((a.x == 0.0 && a.y == 0.0) || (w.x == 0.0 && w.y == 0.0)) continue;
      const double h = (v == 0 || v == H) ? 1.0 : 2.0;
      kc += (v == 0 || v == H) ? 1 : 2;
      const double rr = h * (a.x * w.x + a.y * w.y);
      const double ri = h * (a.y * w.x - a.x * w.y);
#pragma unroll
      for (int c = 0; c < MAX_CAND; ++c) {
        if (c >= m) break;  // m is workgroup-uniform
        // e^{+2 pi i (u dy + v dx)/N} = conj(tw[(u dy + v dx) mod N])
        const double2 t = tw[(u * fy[c] + v * fx[c]) & (N - 1)];  // N is a power of two
        acc[c] += rr * t.x + ri * t.y;  // Re((rr + i ri)(t.x - i t.y))
      }
    }
#pragma unroll
    for (int c = 0; c < MAX_CAND; ++c) {
      if (c < m) {
        const double v = wave_sum_f64(acc[c]);
        if (lane == 0) s_part[wave][c] = v;
      }
    }
    {
      const int v = wave_sum_i32(kc);
      if (lane == 0) s_kpart[wave] = v;
    }
    __syncthreads();
    double val[MAX_CAND];
    double best = -1e300;
#pragma unroll
    for (int c = 0; c < MAX_CAND; ++c) {
      val[c] = ((s_part[0][c] + s_part[1][c]) + s_part[2][c]) + s_part[3][c];
      if (c < m) best = fmax(best, val[c]);
    }
    const int K = ((s_kpart[0] + s_kpart[1]) + s_kpart[2]) + s_kpart[3];
    const double cut = best - TAU * (double)K;
    // overlap counts of the candidates within TAU of the best, rows spread over the threads
    const uint64_t* bits_i = cm.bits + cm.bits_off[i];
    const uint64_t* bits_j = cr.bits + cr.bits_off[j];
    // candidate shifts are in the group's coordinates: forward for d = 0 and 2
    const uint64_t* brep = d == 1 ? bits_i : bits_j;
    const uint64_t* bmem = d == 1 ? bits_j : bits_i;
    int cpart[MAX_CAND];
#pragma unroll
    for (int c = 0; c < MAX_CAND; ++c) {
      cpart[c] = 0;
      if (c < m && val[c] >= cut) {
        const int16_t sh = cq.shifts[gr.offset + c];
        const int dy = (int8_t)(sh >> 8), dx = (int8_t)(sh & 0xff);
        for (int y = tid; y < N; y += RS_THREADS) cpart[c] += row_overlap(brep, bmem, N, y, dy, dx);
      }
    }
#pragma unroll
    for (int c = 0; c < MAX_CAND; ++c) {
      if (c < m) {
        const int v = wave_sum_i32(cpart[c]);
        if (lane == 0) s_cpart[wave][c] = v;
      }
    }
    __syncthreads();
    if (tid == 0) {
      // best per direction of the group: [0] in the stored coordinates, [1]
      // mirrored (d == 2).  The tie rule is one total order, encoded in a key
      // whose maximum is the winner: larger c, then smaller |dy|+|dx|, then
      // smaller dy, then smaller dx.
      uint64_t best_key[2] = {0, 0};
      for (int c = 0; c < m; ++c) {
        if (val[c] < cut) continue;
        const int16_t sh = cq.shifts[gr.offset + c];
        const int dy = (int8_t)(sh >> 8), dx = (int8_t)(sh & 0xff);
        const int cnt = ((s_cpart[0][c] + s_cpart[1][c]) + s_cpart[2][c]) + s_cpart[3][c];
        best_key[0] = max(best_key[0], tie_key(cnt, dy, dx));
        best_key[1] = max(best_key[1], tie_key(cnt, -dy, -dx));
      }
      const int n_i = cm.npix[i], n_j = cr.npix[j];
      const double K_hi = (double)(N * N - max(cm.zero_bins[i], cr.zero_bins[j]));
      for (int h = 0; h < (d == 2 ? 2 : 1); ++h) {
        int bc, bdy, bdx;
        tie_decode(best_key[h], bc, bdy, bdx);
        const int dd = d == 2 ? h : d;  // the pair direction written
        const int nm = dd == 0 ? n_i : n_j, nr = dd == 0 ? n_j : n_i;
        // the other direction of the pair may be decided concurrently by another
        // workgroup, so the shared byte of cover bits is updated atomically
        write_direction_atomic(io, k, dd, bdy, bdx, bc, cosine_score(bc, nm, nr), cosine_bit(bc, nm, nr, thr));
        atomicOr(io.flags + k, dd == 0 ? (uint32_t)CA_FLAG_RESCORED_FWD : (uint32_t)CA_FLAG_RESCORED_REV);
        if (peak_err_bits) {
          // compare like with like: both sides normalised by K_hi
          const double err = fabs(best / K_hi - (double)r1_low[k * 2 + dd]);
          atomicMax(peak_err_bits, (unsigned long long)__double_as_longlong(err));
          if (peak_ratio_bits)
            atomicMax(peak_ratio_bits, (unsigned long long)__double_as_longlong(err * sqrt(K_hi)));
        }
      }
    }
  }
}

hipError_t launch_rescore_candidates(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr,
                                     const CandQueue& cq, const double2* tw256,
                                     unsigned long long* peak_err_bits, unsigned long long* peak_ratio_bits,
                                     const float* r1_low, hipStream_t s) {
  if (cq.cap_groups <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(cq.cap_groups, 8192);
  hipLaunchKernelGGL(rescore_candidates_kernel, dim3(grid), dim3(RS_THREADS), 0, s, cr, cm, io, thr, cq, tw256,
                     peak_err_bits, peak_ratio_bits, r1_low);
  return hipGetLastError();
}

}  // namespace ca
