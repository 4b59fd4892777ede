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

__global__ void __launch_bounds__(RS_THREADS)
rescore_candidates_kernel(ClipsDev cr, ClipsDev cm, PairIO io, Threshold thr, CandQueue cq,
                          const double2* __restrict__ tw256, unsigned long long* peak_err_bits,
                          const float* __restrict__ r1_low) {
  __shared__ double red[RS_THREADS];
  __shared__ double s_acc[MAX_CAND];
  __shared__ int ired[RS_THREADS];
  __shared__ double2 tw[256];
  const int tid = threadIdx.x;
  // grid-stride over the queued groups (count read on the device)
  const int64_t n_groups = min((int64_t)*cq.n_groups, cq.cap_groups);
  for (int64_t gi = blockIdx.x; gi < n_groups; gi += gridDim.x) {
  const CandGroup gr = cq.groups[gi];
  const int64_t k = gr.pair;
  const int d = gr.dir;
  const int m = gr.count;
  const int j = io.rep[k], i = io.mem[k];
  const int N = cm.N[i];
  const int H = N / 2;
  const int tws = 256 / N;
  if (m == 0) continue;
  __syncthreads();  // the previous group's last reads of tw / ired are done
  // tw[t] = exp(-2 pi i t / N) from the half-circle table exp(-2 pi i m / 256), m < 128
  for (int t = tid; t < N; t += RS_THREADS) {
    const double2 base = tw256[((t * tws) & 127)];
    const bool second_half = (t * tws) >= 128;
    tw[t] = second_half ? make_double2(-base.x, -base.y) : base;
  }
  __syncthreads();
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
      if (c >= m) break;
      // e^{+2 pi i (u dy + v dx)/N} = conj(tw[(u dy + v dx) mod N])
      const int e = (u * fy[c] + v * fx[c]) & (N - 1);  // N is a power of two
      const double2 t = tw[e];
      acc[c] += rr * t.x + ri * t.y;  // Re((rr + i ri)(t.x - i t.y))
    }
  }
  // deterministic block reductions (fixed tree)
  ired[tid] = kc;
  __syncthreads();
  for (int s = RS_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s) ired[tid] += ired[tid + s];
    __syncthreads();
  }
  const int K = ired[0];
  for (int c = 0; c < m; ++c) {
    red[tid] = acc[c];
    __syncthreads();
    for (int s = RS_THREADS / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) s_acc[c] = red[0];
    __syncthreads();
  }
  double best = -1e300;
  for (int c = 0; c < m; ++c) best = fmax(best, s_acc[c]);
  const double cut = best - TAU * (double)K;
  const uint64_t* bits_i = cm.bits + cm.bits_off[i];
  const uint64_t* bits_j = cr.bits + cr.bits_off[j];
  // candidate shifts are in the group's coordinates: forward for d = 0 and 2
  const uint64_t* brep = d == 1 ? bits_i : bits_j;
  const uint64_t* bmem = d == 1 ? bits_j : bits_i;
  // best per direction of the group: [0] in the stored coordinates, [1] mirrored (d == 2)
  int best_c[2] = {-1, -1}, best_l1[2] = {0, 0}, best_dy[2] = {0, 0}, best_dx[2] = {0, 0};
  for (int c = 0; c < m; ++c) {
    if (s_acc[c] < cut) continue;
    const int16_t sh = cq.shifts[gr.offset + c];
    const int dy = (int8_t)(sh >> 8), dx = (int8_t)(sh & 0xff);
    const int cnt = block_overlap(brep, bmem, N, dy, dx, ired);
    const int l1 = abs(dy) + abs(dx);
    for (int h = 0; h < (d == 2 ? 2 : 1); ++h) {
      const int ey = h == 0 ? dy : -dy, ex = h == 0 ? dx : -dx;
      bool better = false;
      if (best_c[h] < 0 || cnt > best_c[h]) better = true;
      else if (cnt == best_c[h]) {
        if (l1 < best_l1[h]) better = true;
        else if (l1 == best_l1[h] && (ey < best_dy[h] || (ey == best_dy[h] && ex < best_dx[h]))) better = true;
      }
      if (better) { best_c[h] = cnt; best_l1[h] = l1; best_dy[h] = ey; best_dx[h] = ex; }
    }
  }
  if (tid == 0) {
    const int n_i = cm.npix[i], n_j = cr.npix[j];
    const double K_hi = (double)(N * N - max(cm.zero_bins[i], cr.zero_bins[j]));
    for (int h = 0; h < (d == 2 ? 2 : 1); ++h) {
      const int dd = d == 2 ? h : d;  // the pair direction written
      const int nm = dd == 0 ? n_i : n_j, nr = dd == 0 ? n_j : n_i;
      // the other direction of the pair may be decided concurrently by another
      // workgroup, so the shared byte of cover bits is updated atomically
      write_direction_atomic(io, k, dd, best_dy[h], best_dx[h], best_c[h], cosine_score(best_c[h], nm, nr),
                             cosine_bit(best_c[h], nm, nr, thr));
      atomicOr(io.flags + k, dd == 0 ? (uint32_t)CA_FLAG_RESCORED_FWD : (uint32_t)CA_FLAG_RESCORED_REV);
      if (peak_err_bits) {
        // compare like with like: both sides normalised by K_hi
        const double err = fabs(best / K_hi - (double)r1_low[k * 2 + dd]);
        atomicMax(peak_err_bits, (unsigned long long)__double_as_longlong(err));
      }
    }
  }
  }
}

hipError_t launch_rescore_candidates(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr,
                                     const CandQueue& cq, const double2* tw256,
                                     unsigned long long* peak_err_bits, const float* r1_low, hipStream_t s) {
  if (cq.cap_groups <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(cq.cap_groups, 8192);
  hipLaunchKernelGGL(rescore_candidates_kernel, dim3(grid), dim3(RS_THREADS), 0, s, cr, cm, io, thr, cq, tw256,
                     peak_err_bits, r1_low);
  return hipGetLastError();
}

}  // namespace ca
