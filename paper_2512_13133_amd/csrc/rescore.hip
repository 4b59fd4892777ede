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
//
// When both clip sets hold FP32 spectra, a screening pass first evaluates the
// same sums from them (FP64 arithmetic on the FP32-rounded spectra).  Each
// bin's product then moves by at most 2 * 2^-24 (|W| = 1), so every sum is
// within SCREEN_ERR * K of its FP64 value.  A group is settled by the screen
// when exactly one candidate lies within 2 SCREEN_ERR K + TAU K of the
// screened maximum: every other candidate is then certainly more than TAU
// below the true maximum, so the exact rule has a single tied shift and needs
// no overlap count but the winner's.  The other groups go to the FP64 pass.
// The screen reads half the bytes of the FP64 pass.
//
// Raster sizes are 64, 128 or 256 (the clip-set constructor admits no other).
#include <type_traits>

#include "kernels.h"
#include "pair_common.h"

namespace ca {

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int CAND_PASS = 8;  // candidates summed per pass over the spectra
typedef short short2_t __attribute__((ext_vector_type(2)));

// |K r_screen(s) - K r(s)| / K for FP32-rounded unit spectra: 2 * 2^-24 per
// bin product (+ 2^-48), plus FP64 rounding of the sums below 1e-11.
constexpr double SCREEN_ERR = 1.25e-7;

// Twiddles exp(-2 pi i t / N) for N = 64, 128 and 256, back to back in LDS.
constexpr int TW_TOTAL = 64 + 128 + 256;
template <int N>
constexpr int tw_offset() {
  return N == 64 ? 0 : N == 128 ? 64 : 192;
}

template <typename V>
__device__ __forceinline__ const V* spec_of(const ClipsDev& c, int i);
template <>
__device__ __forceinline__ const double2* spec_of<double2>(const ClipsDev& c, int i) {
  return c.spec64 + c.spec_off[i];
}
template <>
__device__ __forceinline__ const float2* spec_of<float2>(const ClipsDev& c, int i) {
  return c.spec32 + c.spec_off[i];
}

// Sum over the wave, by a butterfly whose partial sums are the same in every
// lane (fixed order, so the result is deterministic and wave-uniform).
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

// One lane's share of the group sums: bins b = lane, lane + 64, ... of the
// half-spectrum (b = u (N/2 + 1) + v), U bins per step with the next step's
// loads in flight while this step computes.  acc[c] for the 4 NCH candidates
// f[c] = 16 (dy, dx) (forward shifts of the group's direction); kc counts the
// full-grid bins where both spectra are non-zero.
template <int N, int NCH, int U, typename V>
__device__ __forceinline__ void lane_sums(const V* __restrict__ Wi, const V* __restrict__ Wj,
                                          const short2_t* f, const double2* tw_all, double* acc, int& kc) {
  constexpr int H = N / 2, H1 = H + 1, BINS = N * H1;
  constexpr int QS = 64 / H1, RS = 64 - QS * H1;  // a step of 64 bins in (u, v), RS < H1
  constexpr int STEP = QS | (RS << 16), CARRY = 1 - (H1 << 16);
  constexpr int MASK16 = 16 * (N - 1);              // byte offset of a twiddle, mod N
  const char* tw = reinterpret_cast<const char*>(tw_all + tw_offset<N>());
  const int lane = threadIdx.x & 63;
  int uv = (lane / H1) | ((lane % H1) << 16);       // (u, v) packed as two 16-bit halves
  V ca[U], cw[U];
#pragma unroll
  for (int t = 0; t < U; ++t) {
    const int b = min(lane + 64 * t, BINS - 1);
    ca[t] = Wi[b];
    cw[t] = Wj[b];
  }
  for (int b0 = lane; b0 < BINS; b0 += 64 * U) {
    V na[U], nw[U];
#pragma unroll
    for (int t = 0; t < U; ++t) {  // next step (clamped: the last step re-reads the last bin)
      const int b = min(b0 + 64 * (U + t), BINS - 1);
      na[t] = Wi[b];
      nw[t] = Wj[b];
    }
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const double ax = ca[t].x, ay = ca[t].y, wx = cw[t].x, wy = cw[t].y;
      const int v = uv >> 16;
      // branch-free: a bin past the end or with a zero spectrum adds 0
      const bool live = (b0 + 64 * t < BINS) & ((ax != 0.0) | (ay != 0.0)) & ((wx != 0.0) | (wy != 0.0));
      const bool edge = (v == 0) | (v == H);
      kc += live ? (edge ? 1 : 2) : 0;
      const double h = live ? (edge ? 1.0 : 2.0) : 0.0;
      const double rr = h * fma(ax, wx, ay * wy);
      const double ri = h * fma(ay, wx, -(ax * wy));
#pragma unroll
      for (int c0 = 0; c0 < 4 * NCH; c0 += 4) {
        double2 t2[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          // e^{+2 pi i (u dy + v dx)/N} = conj(tw[(u dy + v dx) mod N]); N is a power of two
          const int off = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, uv), f[c0 + e], 0, false) & MASK16;
          t2[e] = *reinterpret_cast<const double2*>(tw + off);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {  // Re((rr + i ri)(t.x - i t.y))
          acc[c0 + e] = fma(rr, t2[e].x, acc[c0 + e]);
          acc[c0 + e] = fma(ri, t2[e].y, acc[c0 + e]);
        }
      }
      uv += STEP;
      if ((uv >> 16) >= H1) uv += CARRY;
    }
#pragma unroll
    for (int t = 0; t < U; ++t) {
      ca[t] = na[t];
      cw[t] = nw[t];
    }
  }
}

template <int N, int U, typename V>
__device__ __forceinline__ void lane_sums_m(int m, const V* Wi, const V* Wj, const short2_t* f,
                                            const double2* tw_all, double* acc, int& kc) {
  if (m > 4) lane_sums<N, 2, U>(Wi, Wj, f, tw_all, acc, kc);
  else lane_sums<N, 1, U>(Wi, Wj, f, tw_all, acc, kc);
}

// One wave per candidate group (grid-stride over the groups, whose count is
// read on the device); the waves of a workgroup share only the twiddle
// tables.  The lanes' partial sums and bin counts are reduced by a butterfly,
// so every lane holds the group's values.  SCREEN: FP32 spectra, and the
// groups it cannot settle are appended to `exact`.
template <bool SCREEN>
__global__ void __launch_bounds__(RS_THREADS)
rescore_candidates_kernel(ClipsDev cr, ClipsDev cm, PairIO io, Threshold thr, CandQueue cq, CandQueue exact,
                          const double2* __restrict__ tw256, unsigned long long* peak_err_bits,
                          unsigned long long* peak_ratio_bits, const float* __restrict__ r1_low) {
  using V = typename std::conditional<SCREEN, float2, double2>::type;
  constexpr int U = 2;
  __shared__ double2 tw_all[TW_TOTAL];
  __shared__ double s_val[RS_WAVES][MAX_CAND];  // per wave: the group's candidate sums
  __shared__ int s_cnt[RS_WAVES][MAX_CAND];     // per wave: overlap counts of the tied candidates
  for (int t = threadIdx.x; t < TW_TOTAL; t += RS_THREADS) {
    // table of size N at offset o: entry t - o is exp(-2 pi i e / 256), e = (t - o) 256 / N
    const int e = t < 64 ? 4 * t : t < 192 ? 2 * (t - 64) : t - 192;
    const double2 base = tw256[e & 127];  // exp(-2 pi i m / 256), m < 128
    tw_all[t] = e >= 128 ? make_double2(-base.x, -base.y) : base;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wslot = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wave = (int64_t)blockIdx.x * RS_WAVES + wslot;
  const int64_t n_waves = (int64_t)gridDim.x * RS_WAVES;
  const int64_t n_groups = min((int64_t)*cq.n_groups, cq.cap_groups);
  double err_max = -1.0, ratio_max = -1.0;  // lane 0: largest peak errors of the wave's groups
  for (int64_t gi = wave; gi < n_groups; gi += n_waves) {
    const CandGroup gr = cq.groups[gi];
    const int m = __builtin_amdgcn_readfirstlane(gr.count);
    if (m == 0) continue;
    const int64_t k = __builtin_amdgcn_readfirstlane((int)gr.pair);  // pair ids are below 2^31
    const int d = __builtin_amdgcn_readfirstlane(gr.dir);
    const int j = __builtin_amdgcn_readfirstlane(io.rep[k]), i = __builtin_amdgcn_readfirstlane(io.mem[k]);
    const int N = __builtin_amdgcn_readfirstlane(cm.N[i]);
    const V* Wi = spec_of<V>(cm, i);
    const V* Wj = spec_of<V>(cr, j);
    // candidates eight at a time, one pass over the spectra each (few groups
    // have more than eight); the wave's sums go to its row of s_val
    int kc = 0;
    for (int c0 = 0; c0 < m; c0 += CAND_PASS) {
      // forward shifts of the candidates (direction 1 reads the mirrored
      // surface), times 16 so that u dy + v dx comes out as a twiddle's byte
      // offset from one dot2
      short2_t f[CAND_PASS];
      double acc[CAND_PASS];
#pragma unroll
      for (int c = 0; c < CAND_PASS; ++c) {
        const int sh = __builtin_amdgcn_readfirstlane(c0 + c < m ? (int)cq.shifts[gr.offset + c0 + c] : 0);
        const int sy = (int8_t)(sh >> 8), sx = (int8_t)(sh & 0xff);
        f[c] = short2_t{(short)(16 * (d == 1 ? -sy : sy)), (short)(16 * (d == 1 ? -sx : sx))};
        acc[c] = 0.0;
      }
      int kp = 0;
      const int mp = min(m - c0, CAND_PASS);
      if (N == 128) lane_sums_m<128, U>(mp, Wi, Wj, f, tw_all, acc, kp);
      else if (N == 64) lane_sums_m<64, U>(mp, Wi, Wj, f, tw_all, acc, kp);
      else lane_sums_m<256, U>(mp, Wi, Wj, f, tw_all, acc, kp);
      if (c0 == 0) kc = kp;
#pragma unroll
      for (int c = 0; c < CAND_PASS; ++c) {
        if (c < mp) {
          const double sv = wave_sum_f64(acc[c]);
          if (lane == 0) s_val[wslot][c0 + c] = sv;
        }
      }
    }
    const double* val = s_val[wslot];  // read from LDS where needed
    double best = -1e300;
    for (int c = 0; c < m; ++c) best = fmax(best, val[c]);
    const int K = wave_sum_i32(kc);
    const double cut = best - (SCREEN ? 2.0 * SCREEN_ERR + TAU : TAU) * (double)K;
    if constexpr (SCREEN) {
      // settled only if a single candidate can be tied with the true maximum
      int n_in = 0;
      for (int c = 0; c < m; ++c) n_in += val[c] >= cut ? 1 : 0;
      if (n_in != 1) {
        if (lane == 0) {
          const unsigned long long slot = atomicAdd(exact.n_groups, 1ull);
          if ((int64_t)slot < exact.cap_groups) exact.groups[slot] = gr;
        }
        continue;  // wave-uniform: every lane holds the same sums
      }
    }
    // overlap counts of the candidates within the cut, rows spread over the lanes
    const uint64_t* bits_i = cm.bits + cm.bits_off[i];
    const uint64_t* bits_j = cr.bits + cr.bits_off[j];
    // candidate shifts are in the group's coordinates: forward for d = 0 and 2
    const uint64_t* brep = d == 1 ? bits_i : bits_j;
    const uint64_t* bmem = d == 1 ? bits_j : bits_i;
    int* cnt = s_cnt[wslot];
    for (int c = 0; c < m; ++c) {
      if (val[c] >= cut) {
        const int16_t sh = cq.shifts[gr.offset + c];
        const int dy = (int8_t)(sh >> 8), dx = (int8_t)(sh & 0xff);
        int part = 0;
        for (int y = lane; y < N; y += 64) part += row_overlap(brep, bmem, N, y, dy, dx);
        part = wave_sum_i32(part);
        if (lane == 0) cnt[c] = part;
      }
    }
    if (lane == 0) {
      // best per direction of the group: [0] in the stored coordinates, [1]
      // mirrored (d == 2).  The tie rule is one total order, encoded in a key
      // whose maximum is the winner: larger c, then smaller |dy|+|dx|, then
      // smaller dy, then smaller dx.
      uint64_t best_key[2] = {0, 0};
      for (int c = 0; c < m; ++c) {
        if (val[c] < cut) continue;
        const int16_t sh = cq.shifts[gr.offset + c];
        const int dy = (int8_t)(sh >> 8), dx = (int8_t)(sh & 0xff);
        best_key[0] = max(best_key[0], tie_key(cnt[c], dy, dx));
        best_key[1] = max(best_key[1], tie_key(cnt[c], -dy, -dx));
      }
      const int n_i = cm.npix[i], n_j = cr.npix[j];
      const double K_hi = (double)(N * N - max(cm.zero_bins[i], cr.zero_bins[j]));
      for (int h = 0; h < (d == 2 ? 2 : 1); ++h) {
        int bc, bdy, bdx;
        tie_decode(best_key[h], bc, bdy, bdx);
        const int dd = d == 2 ? h : d;  // the pair direction written
        const int nm = dd == 0 ? n_i : n_j, nr = dd == 0 ? n_j : n_i;
        // the other direction of the pair may be decided concurrently by another
        // wave, so the shared byte of cover bits is updated atomically
        write_direction_atomic(io, k, dd, bdy, bdx, bc, cosine_score(bc, nm, nr), cosine_bit(bc, nm, nr, thr));
        atomicOr(io.flags + k, dd == 0 ? (uint32_t)CA_FLAG_RESCORED_FWD : (uint32_t)CA_FLAG_RESCORED_REV);
        // compare like with like: both sides normalised by K_hi
        const double err = fabs(best / K_hi - (double)r1_low[k * 2 + dd]);
        err_max = fmax(err_max, err);
        ratio_max = fmax(ratio_max, err * sqrt(K_hi));
      }
    }
  }
  // one atomic per wave: thousands of groups updating one word would
  // serialise on it
  if (lane == 0 && peak_err_bits && err_max >= 0.0) {
    atomicMax(peak_err_bits, (unsigned long long)__double_as_longlong(err_max));
    if (peak_ratio_bits) atomicMax(peak_ratio_bits, (unsigned long long)__double_as_longlong(ratio_max));
  }
}

hipError_t launch_rescore_screen(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr,
                                 const CandQueue& cq, const CandQueue& exact, const double2* tw256,
                                 unsigned long long* peak_err_bits, unsigned long long* peak_ratio_bits,
                                 const float* r1_low, hipStream_t s) {
  if (cq.cap_groups <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((cq.cap_groups + RS_WAVES - 1) / RS_WAVES, 2048);
  hipLaunchKernelGGL(rescore_candidates_kernel<true>, dim3(grid), dim3(RS_THREADS), 0, s, cr, cm, io, thr, cq, exact,
                     tw256, peak_err_bits, peak_ratio_bits, r1_low);
  return hipGetLastError();
}

hipError_t launch_rescore_exact(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr,
                                const CandQueue& groups, const double2* tw256, unsigned long long* peak_err_bits,
                                unsigned long long* peak_ratio_bits, const float* r1_low, hipStream_t s) {
  if (groups.cap_groups <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((groups.cap_groups + RS_WAVES - 1) / RS_WAVES, 2048);
  hipLaunchKernelGGL(rescore_candidates_kernel<false>, dim3(grid), dim3(RS_THREADS), 0, s, cr, cm, io, thr, groups,
                     groups, tw256, peak_err_bits, peak_ratio_bits, r1_low);
  return hipGetLastError();
}

// Claim clip c in a set's table: the first claimant takes the next slot and
// records the clip's FP64 spectrum offset (slot * per); later ones see it taken.
__device__ __forceinline__ void claim_clip(int c, int64_t* remap, int64_t* ids, unsigned long long* cnt, int64_t per) {
  unsigned long long* r = reinterpret_cast<unsigned long long*>(remap + c);
  if (atomicCAS(r, ~0ull, ~1ull) == ~0ull) {
    const unsigned long long slot = atomicAdd(cnt, 1ull);
    ids[slot] = c;
    atomicExch(r, (unsigned long long)((int64_t)slot * per));
  }
}

// The clips of the queued groups and of the pairs queued for the full FP64
// surface (representatives in table r, members in table m).
__global__ void mark_fp64_kernel(PairIO io, const CandGroup* __restrict__ groups, int64_t n_groups,
                                 const int64_t* __restrict__ list, int64_t n_list, int64_t* remap_r, int64_t* ids_r,
                                 unsigned long long* cnt_r, int64_t* remap_m, int64_t* ids_m,
                                 unsigned long long* cnt_m, int64_t per) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_groups + n_list) return;
  const int64_t k = t < n_groups ? groups[t].pair : list[t - n_groups];
  claim_clip(io.rep[k], remap_r, ids_r, cnt_r, per);
  claim_clip(io.mem[k], remap_m, ids_m, cnt_m, per);
}

hipError_t launch_mark_fp64(const PairIO& io, const CandGroup* groups, int64_t n_groups, const int64_t* list,
                            int64_t n_list, int64_t* remap_r, int64_t* ids_r, unsigned long long* cnt_r,
                            int64_t* remap_m, int64_t* ids_m, unsigned long long* cnt_m, int64_t per, hipStream_t s) {
  const int64_t n = n_groups + n_list;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(mark_fp64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, io, groups, n_groups, list,
                     n_list, remap_r, ids_r, cnt_r, remap_m, ids_m, cnt_m, per);
  return hipGetLastError();
}

hipError_t launch_rescore_candidates(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr,
                                     const CandQueue& cq, const CandQueue& exact, const double2* tw256,
                                     unsigned long long* peak_err_bits, unsigned long long* peak_ratio_bits,
                                     const float* r1_low, hipStream_t s) {
  if (cq.cap_groups <= 0) return hipSuccess;
  // enough waves to fill the chip several times over; each loops over groups
  const unsigned grid = (unsigned)std::min<int64_t>((cq.cap_groups + RS_WAVES - 1) / RS_WAVES, 2048);
  if (cr.spec32 && cm.spec32 && exact.groups) {
    hipLaunchKernelGGL(rescore_candidates_kernel<true>, dim3(grid), dim3(RS_THREADS), 0, s, cr, cm, io, thr, cq,
                       exact, tw256, peak_err_bits, peak_ratio_bits, r1_low);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rescore_candidates_kernel<false>, dim3(grid), dim3(RS_THREADS), 0, s, cr, cm, io, thr, exact,
                       exact, tw256, peak_err_bits, peak_ratio_bits, r1_low);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(rescore_candidates_kernel<false>, dim3(grid), dim3(RS_THREADS), 0, s, cr, cm, io, thr, cq, cq,
                     tw256, peak_err_bits, peak_ratio_bits, r1_low);
  return hipGetLastError();
}

// ---- FP64 check of decided pairs ------------------------------------------
//
// A deterministic sample of the pairs that the low-precision pass decided in
// both directions (no FP64 re-decision, no empty clip) goes through the full
// FP64 surface as well: their results are saved, they are queued for both
// directions, the FP64 pass rewrites them with the exact answer and records
// |low - FP64| of the peak value, and the compare step counts the pairs whose
// answer changed (a decision the band should have caught; the FP64 answer is
// kept for them) and restores the flags of the others.

__global__ void sample_pick_kernel(int64_t n, int64_t stride, int64_t offset, int64_t count, PairIO io, uint8_t* need,
                                   int64_t* list, unsigned long long* len, SampleSave* saved) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t k = (offset + i * stride) % n;
  const uint32_t f = io.flags[k];
  if (need[k] != 0 || (f & (CA_FLAG_RESCORED_FWD | CA_FLAG_RESCORED_REV | CA_FLAG_EMPTY)) != 0) return;
  const unsigned long long slot = atomicAdd(len, 1ull);
  SampleSave v;
  for (int e = 0; e < 4; ++e) v.shift[e] = io.shift[4 * k + e];
  v.count[0] = io.count[2 * k];
  v.count[1] = io.count[2 * k + 1];
  v.flags = f;
  v.bits = io.bits[k];
  saved[slot] = v;
  list[slot] = k;
  need[k] = 3;
}

__global__ void sample_compare_kernel(const int64_t* list, const unsigned long long* len, const SampleSave* saved,
                                      PairIO io, uint8_t* need, unsigned long long* mismatches) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)*len) return;
  const int64_t k = list[t];
  const SampleSave v = saved[t];
  bool same = io.bits[k] == v.bits && io.count[2 * k] == v.count[0] && io.count[2 * k + 1] == v.count[1];
  for (int e = 0; e < 4; ++e) same = same && io.shift[4 * k + e] == v.shift[e];
  if (same) io.flags[k] = v.flags;
  else atomicAdd(mismatches, 1ull);
  need[k] = 0;
}

hipError_t launch_sample_pick(int64_t n, int64_t count, const PairIO& io, uint8_t* need, int64_t* list,
                              unsigned long long* len, SampleSave* saved, hipStream_t s) {
  if (n <= 0 || count <= 0) return hipSuccess;
  count = std::min(count, n);
  const int64_t stride = n / count;          // count * stride <= n: distinct pairs
  const int64_t offset = (n * 7919) % stride;  // a fixed function of n: repeated calls check the same pairs
  hipLaunchKernelGGL(sample_pick_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, n, stride, offset,
                     count, io, need, list, len, saved);
  return hipGetLastError();
}

hipError_t launch_sample_compare(int64_t cap, const int64_t* list, const unsigned long long* len,
                                 const SampleSave* saved, const PairIO& io, uint8_t* need,
                                 unsigned long long* mismatches, hipStream_t s) {
  if (cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(sample_compare_kernel, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, list, len, saved,
                     io, need, mismatches);
  return hipGetLastError();
}

}  // namespace ca
