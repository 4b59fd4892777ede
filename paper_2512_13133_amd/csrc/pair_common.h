// Device helpers shared by the per-pair kernels: shift windows, the overlap
// count c(s) at a circular shift, and the final score / bit of a direction.
#pragma once

#include "internal.h"

namespace ca {

// Window axis of a half-window w on an N-grid: -w..w when 2w+1 <= N, else
// every residue once, named by its representative in [-N/2, N/2-1].
struct Axis {
  int L;     // positions
  int base;  // axis[l] = l - base
};

__device__ __forceinline__ Axis make_axis(int w, int N) {
  Axis a;
  if (2 * w + 1 <= N) { a.L = 2 * w + 1; a.base = w; }
  else { a.L = N; a.base = N / 2; }
  return a;
}

// Is shift value s (a representative on the union axis) inside the window of
// half-width w?  With all residues (2w+1 > N) every representative is.
__device__ __forceinline__ bool in_window(int s, int w, int N) {
  return (2 * w + 1 > N) || (s >= -w && s <= w);
}

// Representative of -s on an axis (maps N/2 back to -N/2).
__device__ __forceinline__ int neg_rep(int s, int N) {
  int v = -s;
  if (v == N / 2) v = -N / 2;
  return v;
}

// 64 bits of a circular bit row starting at bit position `start` (0 <= start < N).
__device__ __forceinline__ uint64_t row_window64(const uint64_t* row, int wpr, int start) {
  const int ws = start >> 6, o = start & 63;
  const uint64_t lo = row[ws];
  if (o == 0) return lo;
  const uint64_t hi = row[(ws + 1 == wpr) ? 0 : ws + 1];
  return (lo >> o) | (hi << (64 - o));
}

// Overlap count of one row: popcount(rep_row(y) & mem_row((y+dy) mod N) rotated by dx).
__device__ __forceinline__ int row_overlap(const uint64_t* rep, const uint64_t* mem, int N, int y,
                                           int dy, int dx) {
  const int wpr = N >> 6;
  int ym = (y + dy) % N;
  if (ym < 0) ym += N;
  int sx = dx % N;
  if (sx < 0) sx += N;
  const uint64_t* rr = rep + y * wpr;
  const uint64_t* mr = mem + ym * wpr;
  int c = 0;
  for (int k = 0; k < wpr; ++k) {
    int st = 64 * k + sx;
    if (st >= N) st -= N;
    c += __popcll(rr[k] & row_window64(mr, wpr, st));
  }
  return c;
}

// c(s) = sum_x rep(x) mem((x + s) mod N) on one thread (all rows).
__device__ __forceinline__ int thread_overlap(const uint64_t* rep, const uint64_t* mem, int N, int dy, int dx) {
  int c = 0;
  for (int y = 0; y < N; ++y) c += row_overlap(rep, mem, N, y, dy, dx);
  return c;
}

// Block-wide c(s) = sum_x rep(x) mem((x + s) mod N).  All threads must call;
// `red` is a block-sized int scratch in LDS.  Returns the count on every thread.
__device__ __forceinline__ int block_overlap(const uint64_t* rep, const uint64_t* mem, int N, int dy,
                                             int dx, int* red) {
  int c = 0;
  for (int y = threadIdx.x; y < N; y += blockDim.x) c += row_overlap(rep, mem, N, y, dy, dx);
  red[threadIdx.x] = c;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const int out = red[0];
  __syncthreads();
  return out;
}

// Tie rule of the peak as one total order: a larger key wins (larger overlap
// count c >= 0, then smaller |dy|+|dx|, then smaller dy, then smaller dx;
// shift components in [-128, 127]).
__device__ __forceinline__ uint64_t tie_key(int c, int dy, int dx) {
  const uint64_t l1 = (uint64_t)(abs(dy) + abs(dx));  // 0 .. 256
  return ((uint64_t)c << 32) | ((511u - l1) << 16) | ((uint64_t)(255 - (dy + 128)) << 8) |
         (uint64_t)(255 - (dx + 128));
}
__device__ __forceinline__ void tie_decode(uint64_t key, int& c, int& dy, int& dx) {
  c = (int)(key >> 32);
  dy = 255 - (int)((key >> 8) & 0xff) - 128;
  dx = 255 - (int)(key & 0xff) - 128;
}

// Eq. 2 as an exact integer test: c / sqrt(n_m n_r) > p / q.
__device__ __forceinline__ bool cosine_bit(int c, int n_m, int n_r, Threshold t) {
  if (n_m <= 0 || n_r <= 0) return false;
  const unsigned __int128 lhs = (unsigned __int128)((uint64_t)c * (uint64_t)c) *
                                (unsigned __int128)((uint64_t)t.q * (uint64_t)t.q);
  const unsigned __int128 rhs = (unsigned __int128)((uint64_t)t.p * (uint64_t)t.p) *
                                (unsigned __int128)((uint64_t)n_m * (uint64_t)n_r);
  return lhs > rhs;
}

__device__ __forceinline__ double cosine_score(int c, int n_m, int n_r) {
  if (n_m <= 0 || n_r <= 0) return 0.0;
  return (double)c / sqrt((double)n_m * (double)n_r);
}

// Write the result of direction d (0: mem against rep, 1: rep against mem) of pair k.
__device__ __forceinline__ void write_direction(const PairIO& io, int64_t k, int d, int dy, int dx,
                                                int c, double score, bool bit) {
  io.shift[k * 4 + d * 2 + 0] = (int16_t)dy;
  io.shift[k * 4 + d * 2 + 1] = (int16_t)dx;
  io.count[k * 2 + d] = c;
  io.score[k * 2 + d] = score;
  const uint8_t m = (uint8_t)(1u << d);
  io.bits[k] = bit ? (uint8_t)(io.bits[k] | m) : (uint8_t)(io.bits[k] & ~m);
}

// As write_direction, but the cover-bit byte is updated with a 32-bit atomic on
// its aligned word (the word lies in the same page as the byte).
__device__ __forceinline__ void write_direction_atomic(const PairIO& io, int64_t k, int d, int dy, int dx,
                                                       int c, double score, bool bit) {
  io.shift[k * 4 + d * 2 + 0] = (int16_t)dy;
  io.shift[k * 4 + d * 2 + 1] = (int16_t)dx;
  io.count[k * 2 + d] = c;
  io.score[k * 2 + d] = score;
  const uintptr_t addr = reinterpret_cast<uintptr_t>(io.bits + k);
  unsigned int* word = reinterpret_cast<unsigned int*>(addr & ~(uintptr_t)3);
  const unsigned int m = (1u << d) << (8 * (addr & 3));
  if (bit) atomicOr(word, m);
  else atomicAnd(word, ~m);
}

}  // namespace ca
