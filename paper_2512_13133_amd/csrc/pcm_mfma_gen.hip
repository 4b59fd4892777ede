// Batched mixed-precision phase-correlation surface on MFMA for raster sizes
// 64, 128 and 256 and half-windows up to 32 (paper Sec. 3.2.1(1), Eqs. 3-5).
//
// The surface of a pair (member i, representative j) on the window is
//   K r(dy, dx) = Re sum_u sum_{v<=N/2} h(v) R(u, v) e^{2 pi i (u dy + v dx)/N},
// R = W_i conj(W_j), h = 1 at v = 0, N/2 and 2 elsewhere, computed as the two
// dense contractions of the 128 x 128 kernel, generalised:
//   stage 1  T(u, dx) = sum_{v<N/2} R(u, v) h(v) e^{2 pi i v dx/N} (+ the Nyquist
//            column on the VALU): N/32 K chunks of 16 columns (re, im);
//   stage 2  K r(dy, dx) = sum_u Tr(u, dx) cos(2 pi u dy/N) - Ti(u, dx) sin(...):
//            N/16 row blocks, T entering as its FP16 rounding plus remainder.
// The window is tiled by NB x NB blocks of 16 x 16 shifts: shift = 16 b + l - 8 NB
// for block b and in-block index l, so a tile covers [-8 NB, 8 NB - 1]^2
// (NB = 5 covers half-windows up to 32; NB = 4 on 64 x 64 rasters covers every
// residue, named in [-32, 31]).
//
// Unlike the 128 x 128 kernel, the waves of a workgroup are independent: a
// wave takes every fourth pair of a 64-pair tile and streams both the
// member's and the representative's FP16 spectra through buffer loads,
// double-buffered in registers, block by block.  Consecutive pairs of a
// candidate list share their representative, so its blocks come from the
// caches; candidate lists of any length keep all four waves busy, and no
// workgroup barrier separates pairs.  The stage-1 and stage-2 twiddle
// fragments (built on the host in FP64, rounded to FP16) are read from LDS.
//
// The window peak, runner-up, decision band, overlap count, FP64 score, exact
// bit and the FP64 candidate queue follow the 128 x 128 kernel; the candidate
// shifts of an undecided direction are collected straight from the result
// registers with wave ballots.
#include "kernels.h"
#include "mfma_common.h"
#include "pair_common.h"

namespace ca {

namespace {

template <int N, int NB>
struct GenShape {
  static constexpr int H = N / 2;    // stored columns v < H, then the Nyquist column v = H
  static constexpr int KB = H / 16;  // stage-1 K chunks of 16 columns (re, im)
  static constexpr int MB = N / 16;  // 16-row blocks of the half-spectrum
  static constexpr int C = 8 * NB;   // tile offset: shift = 16 b + l - C
  static constexpr int W = 16 * NB;  // tile width (positions per axis)
  static constexpr int SPEC_BYTES = (N * H + N) * 4;
};

constexpr int GEN_TILE = 64;
constexpr int GEN_THREADS = 256;

// The lane's share of a spectrum's 16-row block mb: KB 16-byte K chunks of
// row 16 mb + col and the Nyquist column at rows 16 mb + 4 g .. + 3.
template <int N>
__device__ __forceinline__ void load_block(__amdgpu_buffer_rsrc_t rs, int mb, int col, int g, uint4* out) {
  constexpr int H = N / 2, KB = H / 16;
  const int u = mb * 16 + col;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (u * H + kb * 16 + g * 4) * 4, 0, 0);
    out[kb] = uint4{v[0], v[1], v[2], v[3]};
  }
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (N * H + mb * 16 + g * 4) * 4, 0, 0);
  out[KB] = uint4{v[0], v[1], v[2], v[3]};
}

// Window membership of a shift component on an N-grid (every residue once,
// named in [-N/2, N/2 - 1], when 2 w + 1 > N).
template <int N>
__device__ __forceinline__ bool in_win(int s, int w) {
  return (2 * w + 1 > N) ? (s >= -N / 2 && s < N / 2) : (s >= -w && s <= w);
}

template <int N>
__device__ __forceinline__ int wave_overlap_n(const uint64_t* rep, const uint64_t* mem, int dy, int dx, int lane) {
  int c = 0;
#pragma unroll
  for (int y = lane; y < N; y += 64) c += row_overlap(rep, mem, N, y, dy, dx);
  return wave_sum(c);
}

// Waves per SIMD the register allocation is held to: two where that fits
// without spilling (measured on the compiler's resource report), else one.
// Without the candidate queue (QUEUE false) the 64 x 64 kernel of four
// blocks fits two waves as well.
template <int N, int NB, bool QUEUE = true>
constexpr int gen_min_waves() {
  return (N == 64 && NB <= 3) || (N == 128 && NB == 3) || (N == 64 && NB == 4 && !QUEUE) ? 2 : 1;
}

// QUEUE true: every pair (sel null), or the pairs listed in sel[0, *n_sel),
// with the candidate queue of undecided directions.  QUEUE false: every pair,
// results as above, and each pair with an undecided direction appended to
// sel (count in *n_sel) for a QUEUE pass over just those pairs.
template <int N, int NB, bool QUEUE = true>
__global__ void __launch_bounds__(GEN_THREADS, (gen_min_waves<N, NB, QUEUE>()))
pcm_mfma_gen_kernel(MfView cr, MfView cm, PairIO io, Threshold thr, float band, RescoreQueue q, CandQueue cq,
                    const h8_t* b1frag, const h8_t* a2frag, unsigned long long* tiles, int64_t n_tiles,
                    int32_t* sel, unsigned long long* n_sel) {
  using S = GenShape<N, NB>;
  constexpr int KB = S::KB, MB = S::MB, C = S::C, W = S::W;
  // only the instance that runs two passes reads a pair list
  constexpr bool LIST = QUEUE && gen_min_waves<N, NB, false>() > gen_min_waves<N, NB, true>();
  __shared__ h8_t s_b1[KB * NB * 64];  // stage-1 twiddles
  __shared__ h8_t s_a2[MB * NB * 64];  // stage-2 twiddles
  __shared__ int64_t s_tile;
  // per wave: the pair's two bit rasters (member, then representative) for
  // the overlap counts, at rasters up to 128 x 128
  constexpr int BW = N <= 128 ? N * N / 64 : 1;  // 64-bit words of one raster
  __shared__ uint64_t s_pbits[4][2 * BW];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4;    // k-group of the lane
  const int col = lane & 15;  // row (A) / column (B, C) of the lane in a 16x16 block
  for (int t = tid; t < KB * NB * 64; t += GEN_THREADS) s_b1[t] = b1frag[t];
  for (int t = tid; t < MB * NB * 64; t += GEN_THREADS) s_a2[t] = a2frag[t];

  // over a list, its length (written by the pass before this launch) sets the tiles
  const int64_t n_pairs = (LIST && sel) ? (int64_t)*n_sel : io.n_pairs;
  const int64_t tiles_end = (LIST && sel) ? (n_pairs + GEN_TILE - 1) / GEN_TILE : n_tiles;
  for (;;) {
    __syncthreads();  // every wave has read the previous tile number (and the tables are in place)
    if (tid == 0) {
      const int64_t got = (int64_t)atomicAdd(tiles, 1ull);
      s_tile = got < tiles_end ? got : -1;
    }
    __syncthreads();
    const int64_t tile = s_tile;
    if (tile < 0) break;
    const int64_t base = tile * GEN_TILE;
    const int cnt = (int)min((int64_t)GEN_TILE, n_pairs - base);

    // Metadata of the tile's pairs, pair base + l on lane l (read per pair
    // with readlane): member and representative ids, spectrum and bit
    // offsets, pixel counts, half-window | zero bins << 16.
    int t_i = 0, t_j = 0, t_ni = 0, t_nj = 0, t_wzi = 0, t_wzj = 0;
    int64_t t_soi = 0, t_soj = 0, t_boi = 0, t_boj = 0;
    // the lane's pair: the tile's base + lane, or (list pass) the listed one
    int64_t t_k = 0;
    if constexpr (LIST) t_k = sel ? (lane < cnt ? (int64_t)sel[base + lane] : 0) : base + lane;
    if (lane < cnt) {
      const int64_t kk = LIST ? t_k : base + lane;
      t_i = io.mem[kk];
      t_j = io.rep[kk];
      t_soi = cm.spec_off[t_i];
      t_soj = cr.spec_off[t_j];
      t_boi = cm.bits_off[t_i];
      t_boj = cr.bits_off[t_j];
      t_ni = cm.npix[t_i];
      t_nj = cr.npix[t_j];
      t_wzi = ((int)cm.w[t_i] & 0xffff) | (cm.zero_bins[t_i] << 16);
      t_wzj = ((int)cr.w[t_j] & 0xffff) | (cr.zero_bins[t_j] << 16);
    }

    uint4 m_cur[KB + 1], r_cur[KB + 1];
    bool have0 = false;
    for (int p = wave; p < cnt; p += 4) {
      const int64_t k = LIST ? readlane64(t_k, p) : base + p;
      const int n_i = __builtin_amdgcn_readlane(t_ni, p);
      const int n_j = __builtin_amdgcn_readlane(t_nj, p);
      const int wzi = __builtin_amdgcn_readlane(t_wzi, p);
      const int wzj = __builtin_amdgcn_readlane(t_wzj, p);
      const int w_i = (int)(int16_t)(wzi & 0xffff), z_i = wzi >> 16;
      const int w_j = (int)(int16_t)(wzj & 0xffff), z_j = wzj >> 16;
      if (n_i == 0 || n_j == 0) {
        have0 = false;
        if (lane == 0) {
          io.bits[k] = 0;
          io.flags[k] = CA_FLAG_EMPTY;
          if (q.need) q.need[k] = 0;
          write_direction(io, k, 0, 0, 0, 0, 0.0, false);
          write_direction(io, k, 1, 0, 0, 0, 0.0, false);
        }
        continue;
      }
      // this pair's spectra, and the next pair's (or empty ranges: their loads
      // read nothing) for the prefetch of block 0 during the last block
      const bool has_next = p + 4 < cnt;
      const int pn = has_next ? p + 4 : p;
      const __half2* mptr = cm.spec16 + readlane64(t_soi, p);
      const __half2* rptr = cr.spec16 + readlane64(t_soj, p);
      const __half2* mnext = cm.spec16 + readlane64(t_soi, pn);
      const __half2* rnext = cr.spec16 + readlane64(t_soj, pn);
      const int nbytes = has_next ? S::SPEC_BYTES : 0;
      const __amdgpu_buffer_rsrc_t mrs =
          __builtin_amdgcn_make_buffer_rsrc((void*)mptr, (short)0, S::SPEC_BYTES, MF_RSRC_WORD3);
      const __amdgpu_buffer_rsrc_t rrs =
          __builtin_amdgcn_make_buffer_rsrc((void*)rptr, (short)0, S::SPEC_BYTES, MF_RSRC_WORD3);

      f4_t D2[NB][NB];
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) D2[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};

      // stage 1 of block mb: T(u, dx) for the block's 16 rows into D1
      f4_t D1[2 * NB];  // D1[2 nb] = Tr, D1[2 nb + 1] = Ti at dx = 16 nb + col - C
      auto stage1 = [&](const uint4* mv, const uint4* rv) {
        // Nyquist column v = N/2 for the lane's rows 16 mb + 4 g + t: R(u, N/2)
        // (-1)^dx starts the accumulation; dx has the parity of col in every block
        f4_t N_re, N_im;
        {
          const h2_t n0 = cmulc_h2(as_h2(mv[KB].x), as_h2(rv[KB].x));
          const h2_t n1 = cmulc_h2(as_h2(mv[KB].y), as_h2(rv[KB].y));
          const h2_t n2 = cmulc_h2(as_h2(mv[KB].z), as_h2(rv[KB].z));
          const h2_t n3 = cmulc_h2(as_h2(mv[KB].w), as_h2(rv[KB].w));
          const float sg = (col & 1) ? -1.f : 1.f;
          N_re = f4_t{sgn_lo(n0, sg), sgn_lo(n1, sg), sgn_lo(n2, sg), sgn_lo(n3, sg)};
          N_im = f4_t{sgn_hi(n0, sg), sgn_hi(n1, sg), sgn_hi(n2, sg), sgn_hi(n3, sg)};
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          D1[2 * nb] = N_re;
          D1[2 * nb + 1] = N_im;
        }
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const h2_t r0 = cmulc_h2(as_h2(mv[kb].x), as_h2(rv[kb].x));
          const h2_t r1 = cmulc_h2(as_h2(mv[kb].y), as_h2(rv[kb].y));
          const h2_t r2 = cmulc_h2(as_h2(mv[kb].z), as_h2(rv[kb].z));
          const h2_t r3 = cmulc_h2(as_h2(mv[kb].w), as_h2(rv[kb].w));
          const h8_t A1 = h8_t{r0.x, r0.y, r1.x, r1.y, r2.x, r2.y, r3.x, r3.y};
          const h2_t q0 = mul_neg_i(r0), q1 = mul_neg_i(r1), q2 = mul_neg_i(r2), q3 = mul_neg_i(r3);
          const h8_t A1n = h8_t{q0.x, q0.y, q1.x, q1.y, q2.x, q2.y, q3.x, q3.y};
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const h8_t B1 = s_b1[(kb * NB + nb) * 64 + lane];
            D1[2 * nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, B1, D1[2 * nb], 0, 0, 0);
            D1[2 * nb + 1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1n, B1, D1[2 * nb + 1], 0, 0, 0);
          }
        }
      };
      // stage 2 of block mb: the B operand (u, re/im) x dx straight from D1
      auto stage2 = [&](int mb) {
#pragma unroll
        for (int db = 0; db < NB; ++db) {
          h2_t hi[4], lo[4];
          split_f16(D1[2 * db][0], D1[2 * db][1], hi[0], lo[0]);
          split_f16(D1[2 * db][2], D1[2 * db][3], hi[1], lo[1]);
          split_f16(D1[2 * db + 1][0], D1[2 * db + 1][1], hi[2], lo[2]);
          split_f16(D1[2 * db + 1][2], D1[2 * db + 1][3], hi[3], lo[3]);
          const h8_t B2 = h8_t{hi[0].x, hi[0].y, hi[1].x, hi[1].y, hi[2].x, hi[2].y, hi[3].x, hi[3].y};
          const h8_t B2lo = h8_t{lo[0].x, lo[0].y, lo[1].x, lo[1].y, lo[2].x, lo[2].y, lo[3].x, lo[3].y};
#pragma unroll
          for (int yb = 0; yb < NB; ++yb) {
            const h8_t A2 = s_a2[(mb * NB + yb) * 64 + lane];
            D2[yb][db] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A2, B2, D2[yb][db], 0, 0, 0);
            D2[yb][db] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A2, B2lo, D2[yb][db], 0, 0, 0);
          }
        }
      };
      // The member's blocks are double-buffered in registers (block mb + 1, or
      // the next pair's block 0, loads while block mb computes).  The
      // representative's block, mostly a cache hit (consecutive pairs share it),
      // has one buffer: the next block loads into it as soon as stage 1 has
      // consumed it, and arrives during stage 2.
      if (!have0) {
        load_block<N>(mrs, 0, col, g, m_cur);
        load_block<N>(rrs, 0, col, g, r_cur);
      }
      const __amdgpu_buffer_rsrc_t mrs_next =
          __builtin_amdgcn_make_buffer_rsrc((void*)mnext, (short)0, nbytes, MF_RSRC_WORD3);
      const __amdgpu_buffer_rsrc_t rrs_next =
          __builtin_amdgcn_make_buffer_rsrc((void*)rnext, (short)0, nbytes, MF_RSRC_WORD3);
#pragma unroll 1
      for (int mb = 0; mb < MB; mb += 2) {
        uint4 m_odd[KB + 1];
        load_block<N>(mrs, mb + 1, col, g, m_odd);
        __builtin_amdgcn_sched_barrier(0);
        stage1(m_cur, r_cur);
        load_block<N>(rrs, mb + 1, col, g, r_cur);
        __builtin_amdgcn_sched_barrier(0);
        stage2(mb);
        const bool last = mb == MB - 2;
        load_block<N>(last ? mrs_next : mrs, last ? 0 : mb + 2, col, g, m_cur);
        __builtin_amdgcn_sched_barrier(0);
        stage1(m_odd, r_cur);
        load_block<N>(last ? rrs_next : rrs, last ? 0 : mb + 2, col, g, r_cur);
        __builtin_amdgcn_sched_barrier(0);
        stage2(mb + 1);
      }
      have0 = has_next;
      // the two bit rasters go to the wave's LDS tile by direct global-to-LDS
      // loads issued after the matrix loop (inside it they would make each
      // block wait for every outstanding load); they land during the peak search
      if constexpr (N <= 128) {
        const uint64_t* src_i = cm.bits + readlane64(t_boi, p);
        const uint64_t* src_j = cr.bits + readlane64(t_boj, p);
        if constexpr (N == 64) {
          // 16 bytes a lane: lanes 0-31 the member's 512 bytes, 32-63 the representative's
          const uint64_t* src = lane < 32 ? src_i + 2 * lane : src_j + 2 * (lane - 32);
          __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)s_pbits[wave],
                                           16, 0, 0);
        } else {
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            const uint64_t* src = (h < 2 ? src_i : src_j) + 128 * (h & 1) + 2 * lane;
            __builtin_amdgcn_global_load_lds((const void*)src,
                                             (__attribute__((address_space(3))) void*)(s_pbits[wave] + 128 * h), 16, 0,
                                             0);
          }
        }
      }

      // D2[yb][db][t] = K r(dy, dx) at dy = 16 yb + 4 g + t - C, dx = 16 db + col - C;
      // tile position (dy + C) W + (dx + C) breaks value ties low.
      const int K_hi = N * N - max(z_i, z_j);
      int gl = g, cl = col;
      asm volatile("" : "+v"(gl), "+v"(cl));
      auto top2 = [&](int wd, float& v1, int& i1, float& v2) {
        v1 = -3.0e38f;
        v2 = -3.0e38f;
        i1 = 0x7fffffff;
#pragma unroll
        for (int yb = 0; yb < NB; ++yb)
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int db = 0; db < NB; ++db) {
              const int dy = 16 * yb + 4 * gl + t - C, dx = 16 * db + cl - C;
              const bool ok = in_win<N>(dy, wd) && in_win<N>(dx, wd);
              const float v = ok ? D2[yb][db][t] : -3.0e38f;
              v2 = fmaxf(v2, fminf(v, v1));
              if (v > v1) {
                v1 = v;
                i1 = (dy + C) * W + dx + C;
              }
            }
        wave_top2(v1, i1, v2);
      };
      float v1f, v2f, v1r, v2r;
      int i1f, i1r;
      top2(w_i, v1f, i1f, v2f);
      if (w_j == w_i) {
        v1r = v1f;
        v2r = v2f;
        i1r = i1f;
      } else {
        top2(w_j, v1r, i1r, v2r);
      }
      // the reverse direction's value at shift s is the forward value at -s
      const int sy0 = i1f / W - C, sx0 = i1f % W - C;
      const int sy1 = neg_rep(i1r / W - C, N), sx1 = neg_rep(i1r % W - C, N);
      const uint64_t* bits_i = N <= 128 ? s_pbits[wave] : cm.bits + readlane64(t_boi, p);
      const uint64_t* bits_j = N <= 128 ? s_pbits[wave] + BW : cr.bits + readlane64(t_boj, p);
      // The compiler's own wait for the direct loads is not placed before every
      // read of the tile (at 128 it let the first read of the representative's
      // half go ahead of it), so the wait is explicit; the memory clobber keeps
      // every tile read after it.  The direct loads were the last vector loads
      // issued, so this waits for nothing else.
      if constexpr (N <= 128) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      const int c0 = wave_overlap_n<N>(bits_j, bits_i, sy0, sx0, lane);
      const int c1 = i1r == i1f ? c0 : wave_overlap_n<N>(bits_i, bits_j, sy1, sx1, lane);
      const float band_k = band * sqrtf((float)K_hi);  // in units of K r
      const bool dec0 = (v1f - v2f) >= band_k;
      const bool dec1 = (v1r - v2r) >= band_k;
      if (lane == 0) {
        const bool b0 = cosine_bit(c0, n_i, n_j, thr), b1 = cosine_bit(c1, n_j, n_i, thr);
        io.shift[k * 4 + 0] = (int16_t)sy0;
        io.shift[k * 4 + 1] = (int16_t)sx0;
        io.shift[k * 4 + 2] = (int16_t)sy1;
        io.shift[k * 4 + 3] = (int16_t)sx1;
        io.count[k * 2 + 0] = c0;
        io.count[k * 2 + 1] = c1;
        io.score[k * 2 + 0] = cosine_score(c0, n_i, n_j);
        io.score[k * 2 + 1] = cosine_score(c1, n_j, n_i);
        io.bits[k] = (uint8_t)((b0 ? 1u : 0u) | (b1 ? 2u : 0u));
        io.flags[k] = 0;
        if (q.need) q.need[k] = 0;
        if (q.r1_low) {  // the low-precision peaks, read by the FP64 passes' error statistics
          q.r1_low[k * 2 + 0] = v1f / (float)K_hi;
          q.r1_low[k * 2 + 1] = v1r / (float)K_hi;
        }
      }
      // An undecided direction queues every window shift whose value is within
      // the band of its maximum (d == 2: both directions of equal windows, in
      // forward shifts; d == 1: reverse shifts, mirrors of forward positions),
      // or falls back to the full FP64 surface when there are more than
      // MAX_CAND of them or no room.
      auto queue = [&](int d, int wd, float cutv, float r1) {
        int m = 0;
#pragma unroll
        for (int yb = 0; yb < NB; ++yb)
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int db = 0; db < NB; ++db) {
              const int dy = 16 * yb + 4 * gl + t - C, dx = 16 * db + cl - C;
              const bool ok = in_win<N>(dy, wd) && in_win<N>(dx, wd) && D2[yb][db][t] >= cutv;
              m += __popcll(__ballot(ok));
            }
        unsigned long long slot = 0, off = 0;
        if (lane == 0) {
          slot = atomicAdd(cq.n_groups, 1ull);
          off = m <= MAX_CAND ? atomicAdd(cq.n_shifts, (unsigned long long)m) : 0ull;
        }
        slot = (unsigned long long)readlane64((int64_t)slot, 0);
        off = (unsigned long long)readlane64((int64_t)off, 0);
        const bool fits = m <= MAX_CAND && (int64_t)slot < cq.cap_groups && (int64_t)(off + m) <= cq.cap_shifts;
        if (fits) {
          int written = 0;
#pragma unroll
          for (int yb = 0; yb < NB; ++yb)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
              for (int db = 0; db < NB; ++db) {
                const int dy = 16 * yb + 4 * gl + t - C, dx = 16 * db + cl - C;
                const bool ok = in_win<N>(dy, wd) && in_win<N>(dx, wd) && D2[yb][db][t] >= cutv;
                const unsigned long long bm = __ballot(ok);
                if (ok) {
                  const int idx = written + __popcll(bm & ((1ull << lane) - 1ull));
                  const int ty = d == 1 ? neg_rep(dy, N) : dy, tx = d == 1 ? neg_rep(dx, N) : dx;
                  cq.shifts[off + idx] = (int16_t)((ty << 8) | (tx & 0xff));
                }
                written += __popcll(bm);
              }
        }
        if (lane == 0) {
          if ((int64_t)slot < cq.cap_groups) {
            CandGroup gr;
            gr.pair = k;
            gr.offset = (int64_t)off;
            gr.dir = d;
            gr.count = fits ? m : 0;
            cq.groups[slot] = gr;
          }
          const uint8_t dirs = d == 2 ? 3u : (uint8_t)(1u << d);
          if (dirs & 1u) q.r1_low[k * 2 + 0] = r1;
          if (dirs & 2u) q.r1_low[k * 2 + 1] = r1;
          if (!fits) {
            const uint8_t old = q.need[k];
            q.need[k] = (uint8_t)(old | dirs);
            if (old == 0) {
              const unsigned long long qs = atomicAdd(q.len, 1ull);
              q.list[qs] = k;
            }
          }
        }
      };
      if constexpr (QUEUE) {
        if (w_i == w_j) {
          if (!dec0) queue(2, w_i, v1f - band_k, v1f / (float)K_hi);
        } else {
          if (!dec0) queue(0, w_i, v1f - band_k, v1f / (float)K_hi);
          if (!dec1) queue(1, w_j, v1r - band_k, v1r / (float)K_hi);
        }
      } else {
        if ((!dec0 || (w_i != w_j && !dec1)) && lane == 0) sel[atomicAdd(n_sel, 1ull)] = (int32_t)k;
      }
    }
  }
}

// Workgroups of one kernel instance resident on the device at once.
template <int N, int NB, bool QUEUE>
int resident_groups() {
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pcm_mfma_gen_kernel<N, NB, QUEUE>, GEN_THREADS, 0) !=
            hipSuccess ||
        per <= 0)
      per = 1;
    resident = cus * per;
  }
  return resident;
}

// Where the queue-free kernel runs more waves than the queue kernel, the call
// runs it over every pair and then the queue kernel over the pairs it left
// undecided (their number stays on the device); elsewhere one queue pass.
template <int N, int NB>
hipError_t launch_nb(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr, float band,
                     const RescoreQueue& q, const CandQueue& cq, const void* b1, const void* a2,
                     unsigned long long* tiles, int32_t* sel, unsigned long long* n_sel, hipStream_t s) {
  const int64_t n_tiles = (io.n_pairs + GEN_TILE - 1) / GEN_TILE;
  hipError_t e = launch_zero_u64(tiles, 1, s);
  if (e != hipSuccess) return e;
  if constexpr (gen_min_waves<N, NB, false>() > gen_min_waves<N, NB, true>()) {
    if (sel && n_sel) {
      if ((e = launch_zero_u64(n_sel, 1, s)) != hipSuccess) return e;
      const unsigned g1 = (unsigned)std::min<int64_t>(n_tiles, (int64_t)resident_groups<N, NB, false>());
      hipLaunchKernelGGL((pcm_mfma_gen_kernel<N, NB, false>), dim3(g1), dim3(GEN_THREADS), 0, s, mf_view(cr),
                         mf_view(cm), io, thr, band, q, cq, (const h8_t*)b1, (const h8_t*)a2, tiles, n_tiles, sel,
                         n_sel);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if ((e = launch_zero_u64(tiles, 1, s)) != hipSuccess) return e;
      // the list is at most the whole call; groups without a tile exit at once
      const unsigned g2 = (unsigned)std::min<int64_t>(n_tiles, (int64_t)resident_groups<N, NB, true>());
      hipLaunchKernelGGL((pcm_mfma_gen_kernel<N, NB, true>), dim3(g2), dim3(GEN_THREADS), 0, s, mf_view(cr),
                         mf_view(cm), io, thr, band, q, cq, (const h8_t*)b1, (const h8_t*)a2, tiles, n_tiles, sel,
                         n_sel);
      return hipGetLastError();
    }
  }
  const unsigned grid = (unsigned)std::min<int64_t>(n_tiles, (int64_t)resident_groups<N, NB, true>());
  hipLaunchKernelGGL((pcm_mfma_gen_kernel<N, NB, true>), dim3(grid), dim3(GEN_THREADS), 0, s, mf_view(cr),
                     mf_view(cm), io, thr, band, q, cq, (const h8_t*)b1, (const h8_t*)a2, tiles, n_tiles,
                     (int32_t*)nullptr, (unsigned long long*)nullptr);
  return hipGetLastError();
}

}  // namespace

// Rasters of 128 with half-windows <= 16 run the 128 x 128 kernel, so blocks
// 1 and 2 are not built for them.
int mfma_gen_blocks(int N, int half_window) {
  if (N == 64 && 2 * half_window + 1 > 64) return 4;  // every residue, [-32, 31]
  if (half_window > 32) return 0;
  const int nb = (half_window + 8) / 8;               // [-8 NB, 8 NB - 1] covers [-w, w]
  return N == 128 ? std::max(nb, 3) : nb;
}

size_t mfma_gen_table_halves(int N, int NB) { return (size_t)(N / 32 + N / 16) * NB * 64 * 8; }

void build_mfma_gen_tables(int N, int NB, _Float16* b1, _Float16* a2) {
  const double tau = 2.0 * M_PI / N;
  const int C = 8 * NB, KB = N / 32, MB = N / 16;
  for (int kb = 0; kb < KB; ++kb)
    for (int nb = 0; nb < NB; ++nb)
      for (int lane = 0; lane < 64; ++lane) {
        const int gg = lane >> 4, cc = lane & 15;
        const int dx = 16 * nb + cc - C;
        for (int t = 0; t < 8; ++t) {
          const int v = 16 * kb + 4 * gg + t / 2;
          const double h = v == 0 ? 1.0 : 2.0;
          const double th = tau * (double)((int64_t)v * dx);
          b1[((kb * NB + nb) * 64 + lane) * 8 + t] = (_Float16)((t % 2) ? -h * std::sin(th) : h * std::cos(th));
        }
      }
  for (int mb = 0; mb < MB; ++mb)
    for (int yb = 0; yb < NB; ++yb)
      for (int lane = 0; lane < 64; ++lane) {
        const int gg = lane >> 4, cc = lane & 15;
        const int dy = 16 * yb + cc - C;
        for (int t = 0; t < 8; ++t) {
          const int u = 16 * mb + 4 * gg + t % 4;
          const double th = tau * (double)((int64_t)u * dy);
          a2[((mb * NB + yb) * 64 + lane) * 8 + t] = (_Float16)((t / 4 == 0) ? std::cos(th) : -std::sin(th));
        }
      }
}

hipError_t launch_pcm_mfma_gen(int N, int NB, const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr,
                               float band, const RescoreQueue& q, const CandQueue& cq, const void* b1, const void* a2,
                               unsigned long long* tiles, int32_t* sel, unsigned long long* n_sel, hipStream_t s) {
  if (io.n_pairs == 0) return hipSuccess;
  switch (N * 8 + NB) {
    case 64 * 8 + 1: return launch_nb<64, 1>(cr, cm, io, thr, band, q, cq, b1, a2, tiles, sel, n_sel, s);
    case 64 * 8 + 2: return launch_nb<64, 2>(cr, cm, io, thr, band, q, cq, b1, a2, tiles, sel, n_sel, s);
    case 64 * 8 + 3: return launch_nb<64, 3>(cr, cm, io, thr, band, q, cq, b1, a2, tiles, sel, n_sel, s);
    case 64 * 8 + 4: return launch_nb<64, 4>(cr, cm, io, thr, band, q, cq, b1, a2, tiles, sel, n_sel, s);
    case 128 * 8 + 3: return launch_nb<128, 3>(cr, cm, io, thr, band, q, cq, b1, a2, tiles, sel, n_sel, s);
    case 128 * 8 + 4: return launch_nb<128, 4>(cr, cm, io, thr, band, q, cq, b1, a2, tiles, sel, n_sel, s);
    case 128 * 8 + 5: return launch_nb<128, 5>(cr, cm, io, thr, band, q, cq, b1, a2, tiles, sel, n_sel, s);
    case 256 * 8 + 1: return launch_nb<256, 1>(cr, cm, io, thr, band, q, cq, b1, a2, tiles, sel, n_sel, s);
    case 256 * 8 + 2: return launch_nb<256, 2>(cr, cm, io, thr, band, q, cq, b1, a2, tiles, sel, n_sel, s);
    case 256 * 8 + 3: return launch_nb<256, 3>(cr, cm, io, thr, band, q, cq, b1, a2, tiles, sel, n_sel, s);
    case 256 * 8 + 4: return launch_nb<256, 4>(cr, cm, io, thr, band, q, cq, b1, a2, tiles, sel, n_sel, s);
    case 256 * 8 + 5: return launch_nb<256, 5>(cr, cm, io, thr, band, q, cq, b1, a2, tiles, sel, n_sel, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ca
