// Direct shift-window phase correlation on MFMA for small windows (paper
// Sec. 3.2.1(1), Eqs. 3-5 evaluated in the spatial domain).
//
// With img = N w the whitened image of a clip (w the inverse DFT of its
// whitened spectrum W), Parseval turns the window surface of Eq. 5 into a
// circular cross-correlation of two real images:
//   K r(dy, dx) = sum_{y,x} img_mem(y, x) img_rep(y - dy, x - dx).
// For a batch of 16 members of one representative and one dy this is the
// product D_dy[m][dx] = sum_k A[m][k] B_dy[k][dx], with k over the member's
// pixels: A[m][k] = img_m(pixel k) (the members' rows, streamed from HBM) and
// B_dy[k][dx] = img_rep(y_k - dy, x_k - dx) (the representative's shifted
// rows, read from LDS).  16x16x32 FP16 MFMA with FP32 accumulation; the 16
// columns carry dx = -7 .. 8 (8 is never in a window) and 15 accumulators
// carry dy = -7 .. 7, so half-windows up to 7 are covered.
//
// Schedule: the members' pixels go 64 columns x one row per step (two
// 32-pixel K chunks), row after row.  B_dy for member row y is the
// representative's row y - dy, so the shifted representative rows rotate
// through 16 register slots: one new row per step and chunk, read from LDS
// (aligned dword reads and a funnel shift for the odd half offsets), where
// the representative image lies with 8 wrapped columns on either side.
// Member rows are prefetched seven steps ahead.  One workgroup of four
// waves per compute unit: a wave holds 32 shifted rows, 15 accumulators and
// the prefetch ring (about 300 registers).
//
// The peak search, the overlap count at the peak, the decision band and the
// FP64 candidate queue follow the FFT paths: each direction's top two
// values come from a 16-lane DPP reduction per member, and a direction whose
// gap is below the band queues its candidate shifts for the FP64 re-decision.
#include "kernels.h"
#include "pair_common.h"

namespace ca {

namespace {

typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// The arrays of a clip set the kernel reads.
struct DView {
  const __half* img16;
  const int64_t* img_off;
  const uint64_t* bits;
  const int64_t* bits_off;
  const int32_t* npix;
  const int16_t* w;
  const int32_t* zero_bins;
};

__host__ inline DView d_view(const ClipsDev& c) {
  return DView{c.img16, c.img_off, c.bits, c.bits_off, c.npix, c.w, c.zero_bins};
}

constexpr int DR_TILE = 64;   // pairs per tile pulled from the queue
constexpr int DR_WMAX = 7;    // largest half-window
constexpr int DR_POS = 33;    // positions are numbered (dy + 16) * 33 + dx + 16

template <int CTRL>
__device__ __forceinline__ int dpp_row(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, true);
}

// Larger value wins, ties to the lower position; commutative.
__device__ __forceinline__ void merge2(float& v1, int& i1, float& v2, float o1, int oi, float o2) {
  const bool take = o1 > v1 || (o1 == v1 && oi < i1);
  const float a = take ? v1 : o1;
  const float b = take ? o2 : v2;
  v2 = a > b ? a : b;
  v1 = take ? o1 : v1;
  i1 = take ? oi : i1;
}

template <int CTRL>
__device__ __forceinline__ void merge_step(float& v1, int& i1, float& v2) {
  merge2(v1, i1, v2, __builtin_bit_cast(float, dpp_row<CTRL>(__builtin_bit_cast(int, v1))), dpp_row<CTRL>(i1),
         __builtin_bit_cast(float, dpp_row<CTRL>(__builtin_bit_cast(int, v2))));
}

// Top two over the 16 lanes of each row; every lane of the row ends with it.
__device__ __forceinline__ void row_top2(float& v1, int& i1, float& v2) {
  merge_step<0xB1>(v1, i1, v2);   // quad_perm [1,0,3,2]
  merge_step<0x4E>(v1, i1, v2);   // quad_perm [2,3,0,1]
  merge_step<0x141>(v1, i1, v2);  // row_half_mirror
  merge_step<0x140>(v1, i1, v2);  // row_mirror
}

__device__ __forceinline__ int wave_total(int c) {
  c += dpp_row<0xB1>(c);
  c += dpp_row<0x4E>(c);
  c += dpp_row<0x141>(c);
  c += dpp_row<0x140>(c);
  return __builtin_amdgcn_readlane(c, 0) + __builtin_amdgcn_readlane(c, 16) + __builtin_amdgcn_readlane(c, 32) +
         __builtin_amdgcn_readlane(c, 48);
}

// c(s) = sum_x rep(x) mem((x + s) mod N) on one wave.
template <int N>
__device__ __forceinline__ int wave_overlap(const uint64_t* rep, const uint64_t* mem, int dy, int dx, int lane) {
  int c = 0;
#pragma unroll
  for (int y = lane; y < N; y += 64) c += row_overlap(rep, mem, N, y, dy, dx);
  return wave_total(c);
}

// Queue an undecided direction of the wave's member whose window surface is
// in `sw` ([dy + 7][dx + 7], 16 floats a row): the shifts whose value is at
// least `cutv` become FP64 candidates, or the whole direction goes to the
// FP64 surface when there are more than MAX_CAND of them or no room.  d == 2
// covers both directions of a pair with equal windows (forward shifts).
__device__ __noinline__ void queue_direct(const float* sw, int d, int wd, float cutv, float r1, int64_t k, int lane,
                                          RescoreQueue q, CandQueue cq) {
  constexpr int P = 15 * 15;
  int m = 0;
  for (int t0 = 0; t0 < P; t0 += 64) {
    const int t = t0 + lane;
    bool ok = false;
    if (t < P) {
      const int ty = t / 15 - 7, tx = t - (t / 15) * 15 - 7;
      const int fy = d == 1 ? -ty : ty, fx = d == 1 ? -tx : tx;
      ok = ty >= -wd && ty <= wd && tx >= -wd && tx <= wd && sw[(fy + 7) * 16 + fx + 7] >= cutv;
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
    for (int t0 = 0; t0 < P; t0 += 64) {
      const int t = t0 + lane;
      bool ok = false;
      int ty = 0, tx = 0;
      if (t < P) {
        ty = t / 15 - 7;
        tx = t - (t / 15) * 15 - 7;
        const int fy = d == 1 ? -ty : ty, fx = d == 1 ? -tx : tx;
        ok = ty >= -wd && ty <= wd && tx >= -wd && tx <= wd && sw[(fy + 7) * 16 + fx + 7] >= cutv;
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

// 8 halves of a shifted representative row from 5 dwords: the lane's
// window starts at half offset 2 q + (sh / 16).
__device__ __forceinline__ h8_t funnel8(const uint32_t* d, int sh) {
  uint4 o;
  o.x = __builtin_amdgcn_alignbit(d[1], d[0], sh);
  o.y = __builtin_amdgcn_alignbit(d[2], d[1], sh);
  o.z = __builtin_amdgcn_alignbit(d[3], d[2], sh);
  o.w = __builtin_amdgcn_alignbit(d[4], d[3], sh);
  return __builtin_bit_cast(h8_t, o);
}

template <int N>
__global__ void __launch_bounds__(256, 1)
pcm_direct_kernel(DView cr, DView cm, PairIO io, Threshold thr, float band, RescoreQueue q, CandQueue cq,
                  float* surf_out, unsigned long long* tiles, int64_t n_tiles) {
  constexpr int RSW = N / 2 + 8;        // LDS row stride of the representative (dwords): N + 16 halves
  constexpr int STEPS = (N / 64) * N;   // member steps of a batch: 64 columns x one row each
  extern __shared__ __align__(16) uint32_t s_img[];  // N rows of RSW dwords
  __shared__ float s_surf[4][16 * 16];              // per-wave window surface of one member
  __shared__ int s_rep[DR_TILE];
  __shared__ int s_seg_end;
  __shared__ int64_t s_tile;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4;     // K group of the lane
  const int col = lane & 15;   // A row (member) / B, D column (dx = col - 7)
  // the lane's window of a representative row, relative to a K chunk: halves
  // 8 g + 15 - col .. + 7 of the padded row, read as 5 dwords from qd
  const int lane_p = 8 * g + 15 - col;
  const int lane_qd = lane_p >> 1;
  const int sh = (lane_p & 1) * 16;

  for (;;) {
    if (tid == 0) {
      const int64_t got = (int64_t)atomicAdd(tiles, 1ull);
      s_tile = got < n_tiles ? got : -1;
    }
    __syncthreads();
    const int64_t tile = s_tile;
    if (tile < 0) break;
    const int64_t base = tile * DR_TILE;
    const int cnt = (int)min((int64_t)DR_TILE, io.n_pairs - base);
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
      // the representative image with 8 wrapped columns either side: padded
      // 8-half chunk pc of row r holds chunk (pc - 1) mod (N / 8)
      {
        const uint4* src = reinterpret_cast<const uint4*>(cr.img16 + cr.img_off[j]);
        constexpr int CPR = N / 8 + 2;
        for (int t = tid; t < N * CPR; t += 256) {
          const int r = t / CPR, pc = t - r * CPR;
          const int sc = pc == 0 ? N / 8 - 1 : (pc == CPR - 1 ? 0 : pc - 1);
          *reinterpret_cast<uint4*>(&s_img[r * RSW + 4 * pc]) = src[r * (N / 8) + sc];
        }
      }
      __syncthreads();
      const int seg_end = s_seg_end;
      const int n_j = cr.npix[j], w_j = cr.w[j], z_j = cr.zero_bins[j];
      const uint64_t* bits_j = cr.bits + cr.bits_off[j];

      for (int p0 = seg + 16 * wave; p0 < seg_end; p0 += 64) {
        const int nb = min(16, seg_end - p0);
        // member of this lane's A row (absent rows repeat the first member)
        const int i_a = io.mem[base + p0 + (col < nb ? col : 0)];
        const __half* mrow = cm.img16 + cm.img_off[i_a] + 8 * g;

        f4_t D[15];
#pragma unroll
        for (int a = 0; a < 15; ++a) D[a] = f4_t{0.f, 0.f, 0.f, 0.f};
        h8_t Ba[16], Bb[16];
        uint4 Aring[8][2];
        auto load_a = [&](int s, uint4* out) {
          const int ss = s < STEPS ? s : STEPS - 1;
          const int xp = ss / N, y = ss - xp * N;
          const __half* p = mrow + y * N + 64 * xp;
          out[0] = *reinterpret_cast<const uint4*>(p);
          out[1] = *reinterpret_cast<const uint4*>(p + 32);
        };
#pragma unroll
        for (int a = 0; a < 7; ++a) load_a(a, Aring[a]);

#pragma unroll 1
        for (int xp = 0; xp < N / 64; ++xp) {
          const int qa = 32 * xp + lane_qd, qb = qa + 16;
          // representative rows -7 .. 7 for the first member row
#pragma unroll
          for (int r = -7; r <= 7; ++r) {
            const uint32_t* ra = &s_img[(r & (N - 1)) * RSW + qa];
            const uint32_t* rb = &s_img[(r & (N - 1)) * RSW + qb];
            uint32_t da[5], db[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) {
              da[i] = ra[i];
              db[i] = rb[i];
            }
            Ba[r & 15] = funnel8(da, sh);
            Bb[r & 15] = funnel8(db, sh);
          }
#pragma unroll 1
          for (int yb = 0; yb < N; yb += 16) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
              const int y = yb + u;
              const int s = xp * N + y;
              // the representative row y + 8 for the next step, the member
              // rows seven steps ahead
              uint32_t da[5], db[5];
              {
                const uint32_t* ra = &s_img[((y + 8) & (N - 1)) * RSW + qa];
                const uint32_t* rb = &s_img[((y + 8) & (N - 1)) * RSW + qb];
#pragma unroll
                for (int i = 0; i < 5; ++i) {
                  da[i] = ra[i];
                  db[i] = rb[i];
                }
              }
              load_a(s + 7, Aring[(u + 7) & 7]);
              const h8_t A0 = __builtin_bit_cast(h8_t, Aring[u & 7][0]);
              const h8_t A1 = __builtin_bit_cast(h8_t, Aring[u & 7][1]);
#pragma unroll
              for (int a = 14; a >= 0; --a)
                D[a] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A0, Ba[(u - (a - 7)) & 15], D[a], 0, 0, 0);
#pragma unroll
              for (int a = 14; a >= 0; --a)
                D[a] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, Bb[(u - (a - 7)) & 15], D[a], 0, 0, 0);
              Ba[(u + 8) & 15] = funnel8(da, sh);
              Bb[(u + 8) & 15] = funnel8(db, sh);
            }
          }
        }

        // D[a][t] = K r(dy, dx) of member 4 g + t at dy = a - 7, dx = col - 7.
        int gl = g, cl = col;
        asm volatile("" : "+v"(gl), "+v"(cl));
        const int dx = cl - 7;
        int mi[4], wi[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int mm = 4 * gl + t;
          mi[t] = io.mem[base + p0 + (mm < nb ? mm : 0)];
          wi[t] = cm.w[mi[t]];
        }
        float v1f[4], v2f[4], v1r[4], v2r[4];
        int i1f[4], i1r[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          float a1 = -3.0e38f, a2 = -3.0e38f, b1 = -3.0e38f, b2 = -3.0e38f;
          int ai = 0x7fffffff, bi = 0x7fffffff;
#pragma unroll
          for (int a = 0; a < 15; ++a) {
            const int dy = a - 7;
            const int pos = (dy + 16) * DR_POS + dx + 16;
            const float v = D[a][t];
            const bool okf = dy >= -wi[t] && dy <= wi[t] && dx >= -wi[t] && dx <= wi[t];
            const bool okr = dy >= -w_j && dy <= w_j && dx >= -w_j && dx <= w_j;
            const float vf = okf ? v : -3.0e38f, vr = okr ? v : -3.0e38f;
            a2 = fmaxf(a2, fminf(vf, a1));
            if (vf > a1) { a1 = vf; ai = pos; }
            b2 = fmaxf(b2, fminf(vr, b1));
            if (vr > b1) { b1 = vr; bi = pos; }
          }
          row_top2(a1, ai, a2);
          row_top2(b1, bi, b2);
          v1f[t] = a1; i1f[t] = ai; v2f[t] = a2;
          v1r[t] = b1; i1r[t] = bi; v2r[t] = b2;
        }

        float* sw = s_surf[wave];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll 1
          for (int gg = 0; gg < 4; ++gg) {
            const int mm = 4 * gg + t;
            if (mm >= nb) continue;
            const int64_t k = base + p0 + mm;
            const int src = 16 * gg;
            const int i = __builtin_amdgcn_readlane(mi[t], src);
            const int w_i = __builtin_amdgcn_readlane(wi[t], src);
            const int n_i = cm.npix[i], z_i = cm.zero_bins[i];
            if (n_i == 0 || n_j == 0) {
              if (lane == 0) {
                io.bits[k] = 0;
                io.flags[k] = CA_FLAG_EMPTY;
                if (q.need) q.need[k] = 0;
                write_direction(io, k, 0, 0, 0, 0, 0.0, false);
                write_direction(io, k, 1, 0, 0, 0, 0.0, false);
              }
              continue;
            }
            const float f1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v1f[t]), src));
            const float f2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v2f[t]), src));
            const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v1r[t]), src));
            const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v2r[t]), src));
            const int pf = __builtin_amdgcn_readlane(i1f[t], src);
            const int pr = __builtin_amdgcn_readlane(i1r[t], src);
            const int sy0 = pf / DR_POS - 16, sx0 = pf % DR_POS - 16;
            const int sy1 = 16 - pr / DR_POS, sx1 = 16 - pr % DR_POS;
            const uint64_t* bits_i = cm.bits + cm.bits_off[i];
            const int c0 = wave_overlap<N>(bits_j, bits_i, sy0, sx0, lane);
            const int c1 = pr == pf ? c0 : wave_overlap<N>(bits_i, bits_j, sy1, sx1, lane);
            const int K_hi = N * N - max(z_i, z_j);
            const float band_k = band * sqrtf((float)K_hi);  // in units of K r
            const bool dec0 = (f1 - f2) >= band_k;
            const bool dec1 = (r1 - r2) >= band_k;
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
            }
            if (!dec0 || !dec1 || surf_out) {
              // the member's window surface to the wave's LDS tile
              if (gl == gg) {
#pragma unroll
                for (int a = 0; a < 15; ++a) sw[a * 16 + cl] = D[a][t];
              }
              __builtin_amdgcn_wave_barrier();
              __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
              __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
              if (surf_out) {
                float* so = surf_out + k * 33 * 33;
                for (int t2 = lane; t2 < 15 * 15; t2 += 64) {
                  const int ty = t2 / 15, tx = t2 - ty * 15;
                  so[(ty + 9) * 33 + tx + 9] = sw[ty * 16 + tx] / (float)K_hi;
                }
              }
              if (w_i == w_j) {
                if (!dec0) queue_direct(sw, 2, w_i, f1 - band_k, f1 / (float)K_hi, k, lane, q, cq);
              } else {
                if (!dec0) queue_direct(sw, 0, w_i, f1 - band_k, f1 / (float)K_hi, k, lane, q, cq);
                if (!dec1) queue_direct(sw, 1, w_j, r1 - band_k, r1 / (float)K_hi, k, lane, q, cq);
              }
              __builtin_amdgcn_wave_barrier();
            }
          }
        }
      }
      __syncthreads();
      seg = seg_end;
    }
    __syncthreads();
  }
}

template <int N>
hipError_t launch_n(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr, float band,
                    const RescoreQueue& q, const CandQueue& cq, float* surf_out, unsigned long long* tiles,
                    hipStream_t s) {
  const size_t smem = (size_t)N * (N / 2 + 8) * 4;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)pcm_direct_kernel<N>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    attr = true;
  }
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
    else
      cus = 256;
  }
  const int64_t n_tiles = (io.n_pairs + DR_TILE - 1) / DR_TILE;
  const unsigned grid = (unsigned)std::min<int64_t>(n_tiles, (int64_t)cus);
  hipError_t e = launch_zero_u64(tiles, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pcm_direct_kernel<N>, dim3(grid), dim3(256), smem, s, d_view(cr), d_view(cm), io, thr, band, q,
                     cq, surf_out, tiles, n_tiles);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pcm_direct(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, int N, Threshold thr,
                             float band, const RescoreQueue& q, const CandQueue& cq, float* surf_out,
                             unsigned long long* tiles, hipStream_t s) {
  if (io.n_pairs == 0) return hipSuccess;
  switch (N) {
    case 64: return launch_n<64>(cr, cm, io, thr, band, q, cq, surf_out, tiles, s);
    case 128: return launch_n<128>(cr, cm, io, thr, band, q, cq, surf_out, tiles, s);
    case 256: return launch_n<256>(cr, cm, io, thr, band, q, cq, surf_out, tiles, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ca
