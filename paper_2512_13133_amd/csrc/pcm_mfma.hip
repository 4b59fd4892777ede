// Batched mixed-precision phase-correlation surface on MFMA, raster 128,
// half-windows up to 16 (paper Sec. 3.2.1(1), Eqs. 3-5).
//
// For a pair (member i, representative j) the window surface is
//   K r(dy, dx) = Re sum_u sum_{v<=64} h(v) R(u, v) e^{2 pi i (u dy + v dx)/128},
// R = W_i conj(W_j), h = 1 at v = 0, 64 and 2 elsewhere.  Restricted to the
// 33 x 33 window it is two dense contractions, run on 16x16x32 FP16 MFMA with
// FP32 accumulation:
//   stage 1  T(u, dx)  = sum_{v<64} R(u, v) h(v) e^{2 pi i v dx/128}   (+ the v = 64
//            term on the VALU): rows u, K = (v, re/im) = 128, columns dx; the
//            real part uses the operand R, the imaginary part the operand -i R
//            against the same twiddles (Im T = Re(-i T));
//   stage 2  K r(dy, dx) = sum_u Tr(u, dx) cos(2 pi u dy/128) - Ti(u, dx) sin(...):
//            rows dy, K = (u, re/im) = 256, columns dx.  T enters as two FP16
//            operands, its rounding and the remainder (T - fp16(T)), so that
//            its conversion adds no error of FP16 size.
// R is formed with packed FP16 complex multiplies directly in the stage-1 A
// operand layout; each 16-row stage-1 result block converts in registers into
// the matching stage-2 B operand, so the intermediate never leaves the wave.
//
// Representatives come from the clip set `cr` and members from `cm` (the same
// set for pairs within one set, a device-resident library and a request batch
// when serving).
//
// Batching: a workgroup owns TILE consecutive pairs.  Consecutive pairs with
// the same representative form a run; the run's representative spectrum and
// bits are staged once in LDS and the four waves take its members.  The
// stage-1 twiddles are held in registers through a pair's contractions, the
// stage-2 twiddles in LDS.
//
// Each direction's peak is taken over its window with a wavefront shuffle
// reduction that keeps the maximum and the runner-up.  A peak whose gap (in
// units of K r) is below band * sqrt(K_hi), K_hi = N^2 - max(zero bins), is
// queued for the FP64 re-decision together with its candidate shifts (all
// within that band of the maximum); the others are final here, with the
// overlap count c, the FP64 score and the exact-rational bit.  The error of
// the surface grows like the square root of the number of non-zero bins, so
// the band scales with it.
#include "kernels.h"
#include "mfma_common.h"
#include "pair_common.h"

namespace ca {

constexpr int MF_N = 128;
constexpr int MF_TILE = 64;
constexpr int MF_ROW_H2 = 68;           // LDS row stride of the staged spectrum (half2), padded
constexpr int MF_SPEC_H2 = MF_N * MF_ROW_H2 + MF_N;
constexpr int MF_SPEC_BYTES = (MF_N * 64 + MF_N) * 4;  // one clip's FP16 half-spectrum

// The lane's share of the member's 16-row block mb: four 16-byte K chunks of
// row 16 mb + col, and the Nyquist column at rows 16 mb + 4 g .. + 3.  Buffer
// loads (bounded by the spectrum's size) through a wave-uniform descriptor.
__device__ __forceinline__ void load_member_block(__amdgpu_buffer_rsrc_t rs, int mb, int col, int g, uint4* out) {
  const int u = mb * 16 + col;
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (u * 64 + kb * 16 + g * 4) * 4, 0, 0);
    out[kb] = uint4{v[0], v[1], v[2], v[3]};
  }
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (MF_N * 64 + mb * 16 + g * 4) * 4, 0, 0);
  out[4] = uint4{v[0], v[1], v[2], v[3]};
}

// Overlap count c(s) = sum_x rep(x) mem((x + s) mod 128) on one wave.
__device__ __forceinline__ int wave_overlap128(const uint64_t* rep, const uint64_t* mem, int dy, int dx) {
  const int c = row_overlap(rep, mem, MF_N, threadIdx.x & 63, dy, dx) +
                row_overlap(rep, mem, MF_N, (threadIdx.x & 63) + 64, dy, dx);
  return wave_sum(c);
}

// Queue an undecided direction: every window shift whose low-precision value
// is at least `cutv` becomes a candidate of the FP64 re-decision; when there
// are more than MAX_CAND of them (or no room) the direction falls back to the
// full FP64 surface.  d == 2 queues both directions of a pair with equal
// windows at once (candidates in forward shifts; the reverse ones mirror).
// Wave-wide; kept out of line to spare the caller's registers.
__device__ __noinline__ void queue_candidates(const float* sw, int d, int wd, float cutv, float r1, int64_t k,
                                              int lane, RescoreQueue q, CandQueue cq) {
  int m = 0;
  for (int t0 = 0; t0 < 33 * 33; t0 += 64) {
    const int t = t0 + lane;
    bool ok = false;
    if (t < 33 * 33) {
      const int ty = t / 33 - 16, tx = t - (t / 33) * 33 - 16;
      ok = ty >= -wd && ty <= wd && tx >= -wd && tx <= wd && sw[d == 1 ? 33 * 33 - 1 - t : t] >= cutv;
    }
    m += __popcll(__ballot(ok));
  }
  unsigned long long slot = 0, off = 0;
  if (lane == 0) {
    slot = atomicAdd(cq.n_groups, 1ull);
    off = m <= MAX_CAND ? atomicAdd(cq.n_shifts, (unsigned long long)m) : 0ull;
  }
  slot = __shfl(slot, 0);
  off = __shfl(off, 0);
  const bool fits = m <= MAX_CAND && (int64_t)slot < cq.cap_groups && (int64_t)(off + m) <= cq.cap_shifts;
  if (fits) {
    int written = 0;
    for (int t0 = 0; t0 < 33 * 33; t0 += 64) {
      const int t = t0 + lane;
      bool ok = false;
      int ty = 0, tx = 0;
      if (t < 33 * 33) {
        ty = t / 33 - 16;
        tx = t - (t / 33) * 33 - 16;
        ok = ty >= -wd && ty <= wd && tx >= -wd && tx <= wd && sw[d == 1 ? 33 * 33 - 1 - t : t] >= cutv;
      }
      const unsigned long long bm = __ballot(ok);
      if (ok) {
        const int idx = written + __popcll(bm & ((1ull << lane) - 1ull));
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
}

__global__ void __launch_bounds__(256, 2)
pcm_mfma128_kernel(MfView cr, MfView cm, PairIO io, Threshold thr, float band, RescoreQueue q, CandQueue cq,
                   const h8_t* b1frag, const h8_t* a2frag, float* surf_out, unsigned long long* tiles,
                   int64_t n_tiles) {
  __shared__ __align__(16) uint32_t s_spec[MF_SPEC_H2];   // representative W (half2)
  __shared__ __align__(16) h8_t s_a2[8 * 3 * 64];          // stage-2 twiddles
  __shared__ uint64_t s_bits[MF_N * 2];                   // representative bits
  __shared__ int s_rep[MF_TILE];
  __shared__ int s_seg_end;
  __shared__ float s_surf[4][33 * 33];                    // per-wave window surface
  __shared__ int64_t s_tile;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform (scalar) pair indices
  const int g = lane >> 4;      // k-group of the lane
  const int col = lane & 15;    // row (A) / column (B, C) of the lane in a 16x16 block

  // stage-1 twiddles (4 K-blocks x 3 dx-blocks) of this lane, held for the
  // workgroup's lifetime, and the stage-2 twiddles in LDS
  h8_t B1[4][3];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
#pragma unroll
    for (int nb = 0; nb < 3; ++nb) B1[kb][nb] = b1frag[(kb * 3 + nb) * 64 + lane];
  for (int t = tid; t < 8 * 3 * 64; t += 256) s_a2[t] = a2frag[t];

  // Persistent workgroups pull 64-pair tiles, in list order, from one
  // counter; a workgroup leaves when the list is exhausted.  (Giving each XCD
  // a contiguous eighth of the list measured slower than this interleaving.)
  for (;;) {
    if (tid == 0) {
      const int64_t got = (int64_t)atomicAdd(tiles, 1ull);
      s_tile = got < n_tiles ? got : -1;
    }
    __syncthreads();
    const int64_t tile = s_tile;
    if (tile < 0) break;
    const int64_t base = tile * MF_TILE;
    const int cnt = (int)min((int64_t)MF_TILE, io.n_pairs - base);

    // Member metadata of the tile, pair base + l on lane l of every wave (read
    // per pair with readlane), loaded once so no pair waits on a chain of
    // dependent loads.  w in the low and the zero-bin count in the high half.
    int t_i = 0, t_n = 0, t_wz = 0;
    int64_t t_so = 0, t_bo = 0;
    if (lane < cnt) {
      t_i = io.mem[base + lane];
      t_so = cm.spec_off[t_i];
      t_bo = cm.bits_off[t_i];
      t_n = cm.npix[t_i];
      t_wz = ((int)cm.w[t_i] & 0xffff) | (cm.zero_bins[t_i] << 16);
    }
    if (tid < cnt) s_rep[tid] = io.rep[base + tid];
    __syncthreads();

    int seg = 0;
    while (seg < cnt) {
      if (tid == 0) {
        int e = seg + 1;
        while (e < cnt && s_rep[e] == s_rep[seg]) ++e;
        s_seg_end = e;
      }
      const int j = s_rep[seg];
      // stage the representative's spectrum (rows padded) and bits
      {
        const uint4* src = reinterpret_cast<const uint4*>(cr.spec16 + cr.spec_off[j]);
        for (int t = tid; t < MF_N * 16; t += 256) {  // 16 x 16 B per row
          const int u = t >> 4, c4 = t & 15;
          *reinterpret_cast<uint4*>(&s_spec[u * MF_ROW_H2 + c4 * 4]) = src[t];
        }
        const uint4* nyq = reinterpret_cast<const uint4*>(cr.spec16 + cr.spec_off[j] + MF_N * 64);
        if (tid < 32) *reinterpret_cast<uint4*>(&s_spec[MF_N * MF_ROW_H2 + tid * 4]) = nyq[tid];
        const uint64_t* bj = cr.bits + cr.bits_off[j];
        s_bits[tid] = bj[tid];
      }
      __syncthreads();
      const int seg_end = s_seg_end;
      const int n_j = cr.npix[j], w_j = cr.w[j], z_j = cr.zero_bins[j];

      // block 0 of the wave's next pair in the segment is loaded during the
      // current pair's last block; m_cur holds it when have0 is set
      uint4 m_cur[5];
      bool have0 = false;
      for (int p = seg + wave; p < seg_end; p += 4) {
        const int64_t k = base + p;
        const int n_i = __builtin_amdgcn_readlane(t_n, p);
        const int wz = __builtin_amdgcn_readlane(t_wz, p);
        const int w_i = (int)(int16_t)(wz & 0xffff), z_i = wz >> 16;
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
        // this pair's spectrum, and the next pair's or an empty range (its loads
        // read nothing) at the segment's end; wave-uniform, so the buffer
        // descriptors are scalar
        const __half2* mptr = cm.spec16 + readlane64(t_so, p);
        const bool has_next = p + 4 < seg_end;
        const __half2* nptr = cm.spec16 + readlane64(t_so, has_next ? p + 4 : p);
        const int nbytes = has_next ? MF_SPEC_BYTES : 0;
        const __amdgpu_buffer_rsrc_t mrs =
            __builtin_amdgcn_make_buffer_rsrc((void*)mptr, (short)0, MF_SPEC_BYTES, MF_RSRC_WORD3);
        // the member's bit raster, staged in LDS after the matrix loop
        const uint64_t* mbits = cm.bits + readlane64(t_bo, p);
        f4_t D2[3][3];
  #pragma unroll
        for (int a = 0; a < 3; ++a)
  #pragma unroll
          for (int b = 0; b < 3; ++b) D2[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};

        // One 16-row block of both stages from the member data mv[0..4] of block mb.
        auto block = [&](int mb, const uint4* mv5) {
          const int u = mb * 16 + col;  // A-operand row of this lane
          // Nyquist column v = 64: T(u, dx) gets R(u, 64) (-1)^dx for the lane's
          // 4 rows; the parity of dx (-16 + col, col, 16 + col) is that of col,
          // so one pair of vectors starts the accumulation of all three blocks.
          f4_t N_re, N_im;
          {
            const int u0 = mb * 16 + g * 4;
            const uint4 mv = mv5[4];
            const uint4 rv = *reinterpret_cast<const uint4*>(&s_spec[MF_N * MF_ROW_H2 + u0]);
            const h2_t n0 = cmulc_h2(as_h2(mv.x), as_h2(rv.x));
            const h2_t n1 = cmulc_h2(as_h2(mv.y), as_h2(rv.y));
            const h2_t n2 = cmulc_h2(as_h2(mv.z), as_h2(rv.z));
            const h2_t n3 = cmulc_h2(as_h2(mv.w), as_h2(rv.w));
            const float sg = (col & 1) ? -1.f : 1.f;
            N_re = f4_t{sgn_lo(n0, sg), sgn_lo(n1, sg), sgn_lo(n2, sg), sgn_lo(n3, sg)};
            N_im = f4_t{sgn_hi(n0, sg), sgn_hi(n1, sg), sgn_hi(n2, sg), sgn_hi(n3, sg)};
          }
          // D1[2 db] = Tr, D1[2 db + 1] = Ti for dx = 16 db - 16 + col
          f4_t D1[6];
  #pragma unroll
          for (int nb = 0; nb < 3; ++nb) {
            D1[2 * nb] = N_re;
            D1[2 * nb + 1] = N_im;
          }
  #pragma unroll
          for (int kb = 0; kb < 4; ++kb) {
            const uint4 mv = mv5[kb];
            const uint4 rv = *reinterpret_cast<const uint4*>(&s_spec[u * MF_ROW_H2 + kb * 16 + g * 4]);
            const h2_t r0 = cmulc_h2(as_h2(mv.x), as_h2(rv.x));
            const h2_t r1 = cmulc_h2(as_h2(mv.y), as_h2(rv.y));
            const h2_t r2 = cmulc_h2(as_h2(mv.z), as_h2(rv.z));
            const h2_t r3 = cmulc_h2(as_h2(mv.w), as_h2(rv.w));
            const h8_t A1 = h8_t{r0.x, r0.y, r1.x, r1.y, r2.x, r2.y, r3.x, r3.y};
            const h2_t q0 = mul_neg_i(r0), q1 = mul_neg_i(r1), q2 = mul_neg_i(r2), q3 = mul_neg_i(r3);
            const h8_t A1n = h8_t{q0.x, q0.y, q1.x, q1.y, q2.x, q2.y, q3.x, q3.y};
  #pragma unroll
            for (int nb = 0; nb < 3; ++nb) {
              D1[2 * nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, B1[kb][nb], D1[2 * nb], 0, 0, 0);
              D1[2 * nb + 1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1n, B1[kb][nb], D1[2 * nb + 1], 0, 0, 0);
            }
          }
          // stage 2: B operand (u, re/im) x dx straight from the stage-1 block
  #pragma unroll
          for (int db = 0; db < 3; ++db) {
            h2_t hi[4], lo[4];
            split_f16(D1[2 * db][0], D1[2 * db][1], hi[0], lo[0]);
            split_f16(D1[2 * db][2], D1[2 * db][3], hi[1], lo[1]);
            split_f16(D1[2 * db + 1][0], D1[2 * db + 1][1], hi[2], lo[2]);
            split_f16(D1[2 * db + 1][2], D1[2 * db + 1][3], hi[3], lo[3]);
            const h8_t B2 = h8_t{hi[0].x, hi[0].y, hi[1].x, hi[1].y, hi[2].x, hi[2].y, hi[3].x, hi[3].y};
            const h8_t B2lo = h8_t{lo[0].x, lo[0].y, lo[1].x, lo[1].y, lo[2].x, lo[2].y, lo[3].x, lo[3].y};
  #pragma unroll
            for (int yb = 0; yb < 3; ++yb) {
              const h8_t A2 = s_a2[(mb * 3 + yb) * 64 + lane];
              D2[yb][db] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A2, B2, D2[yb][db], 0, 0, 0);
              D2[yb][db] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A2, B2lo, D2[yb][db], 0, 0, 0);
            }
          }
        };
        // The member's blocks are double-buffered in registers: block mb+1 (or
        // the next pair's block 0) loads while block mb computes, so the HBM
        // latency hides behind the previous block's matrix work.
        // Two buffers alternate (blocks mb and mb+1), so no registers are
        // copied between blocks; the next pair's block 0 ends in m_cur.
        if (!have0) load_member_block(mrs, 0, col, g, m_cur);
  #pragma unroll 1
        for (int mb = 0; mb < 8; mb += 2) {
          uint4 m_odd[5];
          load_member_block(mrs, mb + 1, col, g, m_odd);
          // keep the loads at the top: sunk to where registers free up, their
          // latency would surface at the next block
          __builtin_amdgcn_sched_barrier(0);
          block(mb, m_cur);
          const bool last = mb == 6;
          load_member_block(__builtin_amdgcn_make_buffer_rsrc((void*)(last ? nptr : mptr), (short)0,
                                                              last ? nbytes : MF_SPEC_BYTES, MF_RSRC_WORD3),
                            last ? 0 : mb + 2, col, g, m_cur);
          __builtin_amdgcn_sched_barrier(0);
          block(mb + 1, m_odd);
        }
        have0 = has_next;
        // the member's bit raster goes to the wave's LDS tile by direct
        // global-to-LDS loads now, after the matrix loop (issued inside it they
        // would make every block wait for all outstanding loads); they land
        // while the peak search runs from the registers
        uint64_t* mtile = reinterpret_cast<uint64_t*>(s_surf[wave]);
        {
          const uint64_t* mb_src = mbits + 2 * lane;
          __builtin_amdgcn_global_load_lds((const void*)mb_src, (__attribute__((address_space(3))) void*)mtile, 16, 0, 0);
          __builtin_amdgcn_global_load_lds((const void*)(mb_src + 128),
                                           (__attribute__((address_space(3))) void*)(mtile + 128), 16, 0, 0);
        }

        // D2[yb][db][t] holds K r(dy, dx) at dy = 16 yb - 16 + 4 g + t,
        // dx = 16 db - 16 + col (rows and columns valid up to 16).  Window
        // position of a shift: (dy + 16) * 33 + (dx + 16).
        const int K_hi = MF_N * MF_N - max(z_i, z_j);
        // The lane coordinates pass through an empty asm statement so that the
        // positions and window tests derived from them are formed here, per
        // pair, and are not hoisted to live across the matrix loop.
        int gl = g, cl = col;
        asm volatile("" : "+v"(gl), "+v"(cl));
        // Top two values over the window |dy|, |dx| <= wd and the lowest position
        // of the top one, straight from the registers (a lane visits its
        // positions in increasing order).  The reverse direction's value at
        // shift s is the forward value at -s and the window is symmetric, so the
        // same search over the reverse window gives the reverse top two; its
        // position mirrors.
        auto top2 = [&](int wd, float& v1, int& i1, float& v2) {
          v1 = -3.0e38f;
          v2 = -3.0e38f;
          i1 = 0x7fffffff;
  #pragma unroll
          for (int yb = 0; yb < 3; ++yb)
  #pragma unroll
            for (int t = 0; t < 4; ++t)
  #pragma unroll
              for (int db = 0; db < 3; ++db) {
                const int dy = 16 * yb - 16 + 4 * gl + t, dx = 16 * db - 16 + cl;
                const bool ok = dy >= -wd && dy <= wd && dx >= -wd && dx <= wd;
                const float v = ok ? D2[yb][db][t] : -3.0e38f;
                v2 = fmaxf(v2, fminf(v, v1));
                if (v > v1) {
                  v1 = v;
                  i1 = (dy + 16) * 33 + dx + 16;
                }
              }
          wave_top2(v1, i1, v2);
        };
        // Both windows cover the whole tile (half-window 16): no window tests,
        // only the tile's partial row dy = 16 (lanes g == 0, t == 0) and
        // column dx = 16 (lanes col == 0).  Four operations a value: the
        // runner-up is the median of (value, top, runner-up).  The top one is
        // tracked by its element number e (small integers are free operands)
        // and turned into a position once: e = 3 (4 yb + t) + db for yb < 2,
        // 24 + db for the row dy = 16.
        auto top2_full = [&](float& v1, int& i1, float& v2) {
          v1 = -3.0e38f;
          v2 = -3.0e38f;
          int e1 = 0;
          const bool row16 = gl == 0, col16 = cl == 0;
          auto upd = [&](float v, int e) {
            const bool gt = v > v1;
            v2 = __builtin_amdgcn_fmed3f(v, v1, v2);
            v1 = gt ? v : v1;
            e1 = gt ? e : e1;
          };
  #pragma unroll
          for (int yb = 0; yb < 2; ++yb)
  #pragma unroll
            for (int t = 0; t < 4; ++t) {
              const int r = 4 * yb + t;
              upd(D2[yb][0][t], 3 * r);
              upd(D2[yb][1][t], 3 * r + 1);
              upd(col16 ? D2[yb][2][t] : -3.0e38f, 3 * r + 2);
            }
          upd(row16 ? D2[2][0][0] : -3.0e38f, 24);
          upd(row16 ? D2[2][1][0] : -3.0e38f, 25);
          upd(row16 && col16 ? D2[2][2][0] : -3.0e38f, 26);
          // every lane holds valid values (yb, db < 2), so v1 is a real value
          const int r = e1 / 3, db = e1 - 3 * r;
          const int dy16 = r < 8 ? 16 * (r >> 2) + (r & 3) + 4 * gl : 32;  // dy + 16
          i1 = dy16 * 33 + 16 * db + cl;
          wave_top2(v1, i1, v2);
        };
        float v1f, v2f, v1r, v2r;
        int i1f, i1r;
        const bool full = w_i >= 16 && w_j >= 16;
        if (full) top2_full(v1f, i1f, v2f);
        else top2(w_i, v1f, i1f, v2f);
        if (full || w_j == w_i) {
          v1r = v1f;
          v2r = v2f;
          i1r = i1f;
        } else {
          top2(w_j, v1r, i1r, v2r);
        }
        // forward shift and the reverse one (mirror of the reverse top position)
        const int sy0 = i1f / 33 - 16, sx0 = i1f % 33 - 16;
        const int sy1 = 16 - i1r / 33, sx1 = 16 - i1r % 33;
        // The wait for the direct loads is explicit: the compiler places its
        // own from alias information, which has been seen to let a read of such
        // a tile go ahead of it; the memory clobber keeps every tile read after
        // it.  The direct loads were the last vector loads issued.
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        // c(s) of the reverse direction at -s equals the forward c(s)
        const int c0 = wave_overlap128(s_bits, mtile, sy0, sx0);
        const int c1 = i1r == i1f ? c0 : wave_overlap128(mtile, s_bits, sy1, sx1);
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
        if (!dec0 || !dec1 || surf_out) {
          // the window surface goes to the wave's LDS tile (over the member
          // bits, no longer needed) for the candidate queue and the surface output
          float* sw = s_surf[wave];
  #pragma unroll
          for (int yb = 0; yb < 3; ++yb)
  #pragma unroll
            for (int db = 0; db < 3; ++db)
  #pragma unroll
              for (int t = 0; t < 4; ++t) {
                const bool ok = (yb < 2 || (gl == 0 && t == 0)) && (db < 2 || cl == 0);
                if (ok) sw[(4 * gl + t) * 33 + cl + (16 * yb * 33 + 16 * db)] = D2[yb][db][t];
              }
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (surf_out) {
            float* so = surf_out + k * 33 * 33;
            for (int t = lane; t < 33 * 33; t += 64) so[t] = sw[t] / (float)K_hi;
          }
          if (w_i == w_j) {  // one group settles both (mirrored) directions
            if (!dec0) queue_candidates(sw, 2, w_i, v1f - band_k, v1f / (float)K_hi, k, lane, q, cq);
          } else {
            if (!dec0) queue_candidates(sw, 0, w_i, v1f - band_k, v1f / (float)K_hi, k, lane, q, cq);
            if (!dec1) queue_candidates(sw, 1, w_j, v1r - band_k, v1r / (float)K_hi, k, lane, q, cq);
          }
          // the tile is rewritten by the wave's next pair only after every lane is done reading
          __builtin_amdgcn_wave_barrier();
        }
      }
      __syncthreads();
      seg = seg_end;
    }
    __syncthreads();
  }
}

// Fragment tables, built on the host in double precision and rounded to FP16.
//   b1[(kb * 3 + nb) * 64 + lane][t]: K index kk = 32 kb + 8 g + t <-> (v = 16 kb + 4 g + t/2,
//     re/im = t % 2); column col of block nb <-> dx = 16 nb - 16 + col; entries
//     h(v) cos(theta) for re, -h(v) sin(theta) for im, theta = 2 pi v dx / 128.
//   a2[(mb * 3 + yb) * 64 + lane][t]: row col <-> dy = 16 yb - 16 + col; K index <->
//     (u = 16 mb + 4 g + t % 4, re/im = t / 4): cos(2 pi u dy/128) or -sin(2 pi u dy/128).
void build_mfma128_tables(_Float16* b1, _Float16* a2) {
  const double tau = 2.0 * M_PI / 128.0;
  for (int kb = 0; kb < 4; ++kb)
    for (int nb = 0; nb < 3; ++nb)
      for (int lane = 0; lane < 64; ++lane) {
        const int gg = lane >> 4, cc = lane & 15;
        const int dx = 16 * nb - 16 + cc;
        for (int t = 0; t < 8; ++t) {
          const int v = 16 * kb + 4 * gg + t / 2;
          const int im = t % 2;
          const double h = v == 0 ? 1.0 : 2.0;
          double val = 0.0;
          if (dx <= 16) {
            const double th = tau * v * dx;
            val = im ? -h * std::sin(th) : h * std::cos(th);
          }
          b1[((kb * 3 + nb) * 64 + lane) * 8 + t] = (_Float16)val;
        }
      }
  for (int mb = 0; mb < 8; ++mb)
    for (int yb = 0; yb < 3; ++yb)
      for (int lane = 0; lane < 64; ++lane) {
        const int gg = lane >> 4, cc = lane & 15;
        const int dy = 16 * yb - 16 + cc;
        for (int t = 0; t < 8; ++t) {
          const int u = 16 * mb + 4 * gg + t % 4;
          double val = 0.0;
          if (dy <= 16) {
            const double th = tau * u * dy;
            val = (t / 4 == 0) ? std::cos(th) : -std::sin(th);
          }
          a2[((mb * 3 + yb) * 64 + lane) * 8 + t] = (_Float16)val;
        }
      }
}

hipError_t launch_pcm_mfma128(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr, float band,
                              const RescoreQueue& q, const CandQueue& cq, const void* b1frag,
                              const void* a2frag, float* surf_out, unsigned long long* tiles, hipStream_t s) {
  if (io.n_pairs == 0) return hipSuccess;
  const int64_t n_tiles = (io.n_pairs + MF_TILE - 1) / MF_TILE;
  // resident workgroups: two per compute unit
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
    else
      cus = 256;
  }
  const unsigned grid = (unsigned)std::min<int64_t>(n_tiles, 2 * (int64_t)cus);
  hipError_t e = launch_zero_u64(tiles, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pcm_mfma128_kernel, dim3(grid), dim3(256), 0, s, mf_view(cr), mf_view(cm), io, thr, band, q, cq,
                     (const h8_t*)b1frag, (const h8_t*)a2frag, surf_out, tiles, n_tiles);
  return hipGetLastError();
}

}  // namespace ca
