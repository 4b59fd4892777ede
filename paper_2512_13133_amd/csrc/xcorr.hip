// Exact-objective alignment (paper Sec. 3.2: the shift of the member's window
// that maximises the similarity to the fixed representative).
//
// For a pair (member i, representative j) every shift s = (dy, dx) of the
// window gets its overlap count
//   c(s) = sum_x a_j(x) a_i((x + s) mod N),
// the chosen shift is the largest c, ties to the smaller |dy| + |dx|, then to
// the smaller (dy, dx) (one integer key, as in the FP64 re-decision), and the
// score and bit are those of Eq. 2 there.  Maximising c maximises the cosine,
// whose denominator does not depend on s.  The reverse direction (j aligned
// to i) reads the same counts at -s, over j's window.  Integer work only, so
// the result is exact.
//
// One workgroup per 16 consecutive pairs (pairs grouped by representative
// reuse its copies).  The representative's bit rows are staged in LDS in 33
// rotated copies, copy dx holding bit (x - dx) mod N at x, so that
//   c(dy, dx) = sum_y popcount(rot_dx(a_j)[y] & a_i[(y + dy) mod N])
// is an AND and a bit count per 32-bit word.  Thread t takes one dx and five
// consecutive dy (33 x 7 = 231 threads): per row y it reads its rotated
// representative row once and one new member row (the same row for all
// threads of a dy block, broadcast by LDS) into a ring of five rows in
// registers.  Rows are N / 32 words; rasters of
// 64 and 128, half-windows up to 16.
#include "kernels.h"
#include "pair_common.h"

namespace ca {

namespace {

constexpr int XC_THREADS = 256;
constexpr int XC_W = 16;               // largest half-window
constexpr int XC_NDX = 2 * XC_W + 1;   // dx values
constexpr int XC_R = 5;                // dy values per thread
constexpr int XC_NBY = 7;              // dy blocks (7 x 5 = 35 >= 33)
static_assert(XC_NDX * XC_NBY <= XC_THREADS, "one task per thread");
constexpr int XC_TILE = 16;            // consecutive pairs per workgroup

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o);
    const uint64_t u = ((uint64_t)hi << 32) | lo;
    v = u > v ? u : v;
  }
  return v;
}

// grid: one workgroup per XC_TILE consecutive pairs from k0 on; pairs of
// another raster size are left to the launch for theirs.  The rotated copies
// of a representative are kept while consecutive pairs share it.
template <int N>
__global__ void __launch_bounds__(XC_THREADS) xcorr_kernel(ClipsDev cr, ClipsDev cm, PairIO io, Threshold thr,
                                                           int64_t k0) {
  constexpr int NW = N / 32;       // words per row
  constexpr int IMG = N * NW;      // words per raster
  constexpr int ROT = IMG + 4;     // words per rotated copy (16 B apart: distinct banks)
  __shared__ uint32_t s_mem[IMG];
  __shared__ __align__(16) uint32_t s_rot[XC_NDX * ROT];
  __shared__ uint64_t s_key[XC_THREADS / 64][2];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const bool active = tid < XC_NDX * XC_NBY;
  const int ix = tid % XC_NDX, iby = tid / XC_NDX;
  const int dx = ix - XC_W, dy0 = iby * XC_R - XC_W;
  const int64_t kb = k0 + (int64_t)blockIdx.x * XC_TILE;
  const int64_t ke = min(kb + XC_TILE, io.n_pairs);
  int staged = -1;  // representative whose copies s_rot holds (workgroup-uniform)
  for (int64_t k = kb; k < ke; ++k) {
    const int j = io.rep[k], i = io.mem[k];
    if (cm.N[i] != N) continue;  // workgroup-uniform
    const int n_i = cm.npix[i], n_j = cr.npix[j];
    if (n_i == 0 || n_j == 0) {
      if (tid == 0) {
        io.bits[k] = 0;
        io.flags[k] = CA_FLAG_EMPTY;
        write_direction(io, k, 0, 0, 0, 0, 0.0, false);
        write_direction(io, k, 1, 0, 0, 0, 0.0, false);
      }
      continue;
    }
    __syncthreads();  // the previous pair's reads of s_mem, s_rot and s_key are done
    {
      const uint32_t* bm = reinterpret_cast<const uint32_t*>(cm.bits + cm.bits_off[i]);
      for (int t = tid; t < IMG; t += XC_THREADS) s_mem[t] = bm[t];
    }
    if (j != staged) {
      // copy ix (dx = ix - 16), word w of row y: representative bits from
      // s0 = (32 w - dx) mod N on, a funnel shift of two neighbouring words
      const uint32_t* br = reinterpret_cast<const uint32_t*>(cr.bits + cr.bits_off[j]);
      for (int t = tid; t < XC_NDX * IMG; t += XC_THREADS) {
        const int cx = t / IMG, rem = t - cx * IMG;
        const int y = rem / NW, w = rem - y * NW;
        const int s0 = (32 * w - (cx - XC_W) + N) & (N - 1);
        const int q = s0 >> 5;
        const uint32_t lo = br[y * NW + q], hi = br[y * NW + ((q + 1) & (NW - 1))];
        s_rot[cx * ROT + rem] = __builtin_amdgcn_alignbit(hi, lo, s0 & 31);
      }
      staged = j;
    }
    __syncthreads();

    int c[XC_R];
#pragma unroll
    for (int r = 0; r < XC_R; ++r) c[r] = 0;
    if (active) {
      const uint32_t* rot = s_rot + ix * ROT;
      // ring[(y + r) % XC_R] holds member row (y + dy0 + r) mod N; one new row
      // a step
      uint32_t ring[XC_R][NW];
#pragma unroll
      for (int r = 0; r < XC_R - 1; ++r)
#pragma unroll
        for (int w = 0; w < NW; ++w) ring[r][w] = s_mem[((dy0 + r) & (N - 1)) * NW + w];
      for (int y0 = 0; y0 < N; y0 += XC_R) {
#pragma unroll
        for (int u = 0; u < XC_R; ++u) {
          const int y = y0 + u;
          if (y < N) {  // uniform
            const int slot_new = (u + XC_R - 1) % XC_R;
#pragma unroll
            for (int w = 0; w < NW; ++w) ring[slot_new][w] = s_mem[((y + dy0 + XC_R - 1) & (N - 1)) * NW + w];
            uint32_t rv[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) rv[w] = rot[y * NW + w];
#pragma unroll
            for (int r = 0; r < XC_R; ++r)
#pragma unroll
              for (int w = 0; w < NW; ++w) c[r] += __builtin_popcount(rv[w] & ring[(u + r) % XC_R][w]);
          }
        }
      }
    }
    // best key per direction: [0] member i over its window at s, [1] member j
    // over its window at -s (the same count)
    const int w_i = cm.w[i], w_j = cr.w[j];
    uint64_t key0 = 0, key1 = 0;
    if (active) {
#pragma unroll
      for (int r = 0; r < XC_R; ++r) {
        const int dy = dy0 + r;
        if (dy > XC_W) continue;
        if (abs(dy) <= w_i && abs(dx) <= w_i) key0 = max(key0, tie_key(c[r], dy, dx));
        if (abs(dy) <= w_j && abs(dx) <= w_j) key1 = max(key1, tie_key(c[r], -dy, -dx));
      }
    }
    key0 = wave_max_u64(key0);
    key1 = wave_max_u64(key1);
    if (lane == 0) {
      s_key[wave][0] = key0;
      s_key[wave][1] = key1;
    }
    __syncthreads();
    if (tid == 0) {
      uint64_t b0 = 0, b1 = 0;
      for (int v = 0; v < XC_THREADS / 64; ++v) {
        b0 = max(b0, s_key[v][0]);
        b1 = max(b1, s_key[v][1]);
      }
      int c0, y0, x0, c1, y1, x1;
      tie_decode(b0, c0, y0, x0);
      tie_decode(b1, c1, y1, x1);
      io.flags[k] = 0;
      io.bits[k] = 0;  // write_direction sets or clears its own bit only
      write_direction(io, k, 0, y0, x0, c0, cosine_score(c0, n_i, n_j), cosine_bit(c0, n_i, n_j, thr));
      write_direction(io, k, 1, y1, x1, c1, cosine_score(c1, n_j, n_i), cosine_bit(c1, n_j, n_i, thr));
    }
  }
}

}  // namespace

hipError_t launch_xcorr(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, int N, Threshold thr,
                        hipStream_t s) {
  const int64_t per = LAUNCH_CHUNK * XC_TILE;  // pairs per launch
  for (int64_t k0 = 0; k0 < io.n_pairs; k0 += per) {
    const unsigned nb = (unsigned)((std::min<int64_t>(per, io.n_pairs - k0) + XC_TILE - 1) / XC_TILE);
    if (N == 64)
      hipLaunchKernelGGL(xcorr_kernel<64>, dim3(nb), dim3(XC_THREADS), 0, s, cr, cm, io, thr, k0);
    else if (N == 128)
      hipLaunchKernelGGL(xcorr_kernel<128>, dim3(nb), dim3(XC_THREADS), 0, s, cr, cm, io, thr, k0);
    else
      return hipErrorInvalidValue;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ca
