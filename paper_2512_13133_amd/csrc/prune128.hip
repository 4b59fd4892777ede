// Cosine candidate generation for 128 x 128 clips with half-windows <= 16
// (paper Sec. 3.1 stage 1; the safe bounds B1 and B2 of the library
// documentation), specialised so that every operand of the signature bound
// sits in registers.
//
// Anchors are clips in (n, id) order; B1 leaves each anchor a contiguous
// range of larger partners (computed on the host).  One wavefront owns an
// anchor; its lanes take 64 partners at a time.
//   group stage    the shifts |d| <= 16 split into two groups G; per group the
//                  partner's sliding sums maximised over the group's shifts,
//                  M_G[Y] = max_{d in G} W[(8 Y + d) mod 128], bound every
//                  shift of the group at once: U(d) <= sum_Y min(A_rep[Y],
//                  M_G[Y]).  The two groups share a packed 16-bit pair, so
//                  the stage costs 16 min/add pairs a dimension (the coarse
//                  stage 544).  It is looser than the coarse stage, so it only
//                  drops pairs the coarse stage would drop (about two thirds of
//                  the range on 128 x 128 layout clips); its survivors are
//                  queued in LDS so the coarse stage runs on full waves,
//                  reading each queued partner's own sliding sums.
//   coarse stage   U(d) <= sum_Y min(A_rep[Y], W_mem[(8 Y + d) mod 128]) over the
//                  16 row blocks Y, A = block sums of the anchor (uniform),
//                  W = sliding 8-row sums of the partner (64 registers of packed
//                  16-bit pairs); one v_pk_min_u16 / v_pk_add_u16 pair serves
//                  the shifts d and d+1 at once.  Maximised over the union of
//                  both windows, it bounds both directions.
//   exact stage    U(d) = sum_y min(r_a[y], r_b[(y + d) mod 128]) for coarse
//                  survivors, two rows per packed instruction (the partner's
//                  sums held even- and odd-aligned in registers).  Survivors
//                  of the coarse stage are queued in LDS so the exact stage
//                  always runs on full waves.
// When anchors are few (a request batch against a large library), each
// anchor's range is split into segments (grid y) so the chip still fills;
// both passes then count and write per (anchor, segment).
// The partners' sliding sums are read from a transposed copy (pair q of the
// partner at order position b at [q n + b]), so each load of the coarse stage
// is one contiguous run across the wave instead of 64 separate rows.
// Pass flags go to a bitmask over each anchor's partner range; a second
// kernel writes the surviving pairs in (anchor order, partner order).
// Anchors come from the clip set `ca` and partners from `cb` (the same set
// within one clip set; a request batch and the library when serving).
#include "kernels.h"
#include "pair_common.h"

namespace ca {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_u16x2(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t pk_u16(uint32_t lo, uint32_t hi) { return (lo & 0xffffu) | (hi << 16); }

__device__ __forceinline__ bool passes128(int64_t b, int n1, int n2, Threshold t) {
  const unsigned __int128 lhs = (unsigned __int128)((uint64_t)b * (uint64_t)b) *
                                (unsigned __int128)((uint64_t)t.q * (uint64_t)t.q);
  const unsigned __int128 rhs = (unsigned __int128)((uint64_t)t.p * (uint64_t)t.p) *
                                (unsigned __int128)((uint64_t)n1 * (uint64_t)n2);
  return lhs > rhs;
}

// Coarse bound of one dimension: max over |d| <= wmax of sum_Y min(A[Y], W[(8Y + d) mod 128]).
// A: the anchor's 16 block sums (uniform, streamed); W: 64 packed pairs (W[2m], W[2m+1]).
__device__ __forceinline__ int coarse_dim(const uint16_t* __restrict__ A, int stride, const uint32_t* W, int wmax) {
  u16x2 acc[17];
#pragma unroll
  for (int e = 0; e < 17; ++e) acc[e] = u16x2{0, 0};
#pragma unroll
  for (int Y = 0; Y < 16; ++Y) {
    const uint32_t ay = A[Y * stride];
    const u16x2 a = as_u16x2(ay * 0x10001u);
#pragma unroll
    for (int e = 0; e < 17; ++e) {  // shift pair (d, d+1), d = -16 + 2 e
      const int t = (8 * Y - 16 + 2 * e + 128) & 127;  // even
      acc[e] += __builtin_elementwise_min(as_u16x2(W[t >> 1]), a);
    }
  }
  int best = 0;
#pragma unroll
  for (int e = 0; e < 17; ++e) {
    const int d = -16 + 2 * e;
    if (d >= -wmax && d <= wmax) best = max(best, (int)acc[e].x);
    if (d + 1 >= -wmax && d + 1 <= wmax) best = max(best, (int)acc[e].y);
  }
  return best;
}

// Group bound of one dimension: max over the two shift groups of
// sum_Y min(A[Y], M_G[Y]); G: the partner's packed group maxima (block Y at
// row Y of a table of stride n).
__device__ __forceinline__ int group_dim(const uint16_t* __restrict__ A, int stride, const uint32_t* __restrict__ G,
                                         int64_t n, int64_t pos) {
  u16x2 acc = u16x2{0, 0};
#pragma unroll
  for (int Y = 0; Y < 16; ++Y) {
    const u16x2 a = as_u16x2((uint32_t)A[Y * stride] * 0x10001u);
    acc += __builtin_elementwise_min(as_u16x2(G[Y * n + pos]), a);
  }
  return max((int)acc.x, (int)acc.y);
}

// Exact bound of one dimension: per direction the max over the window of
// U(d) = sum_y min(Ra[y], Rb[(y + d) mod 128]).
// Ra: the anchor's packed pairs (uniform, streamed); Be/Bo: partner pairs aligned at even / odd rows.
__device__ __forceinline__ void exact_dim(const uint32_t* __restrict__ Ra, const uint32_t* Be, const uint32_t* Bo,
                                          int wb, int wa, int& best_b, int& best_a) {
  u16x2 acc[33];
#pragma unroll
  for (int d = 0; d < 33; ++d) acc[d] = u16x2{0, 0};
#pragma unroll
  for (int m = 0; m < 64; ++m) {
    const u16x2 ra = as_u16x2(Ra[m]);
#pragma unroll
    for (int d = -16; d <= 16; ++d) {
      const int t = (2 * m + d + 128) & 127;
      const uint32_t x = (t & 1) ? Bo[t >> 1] : Be[t >> 1];
      acc[d + 16] += __builtin_elementwise_min(ra, as_u16x2(x));
    }
  }
#pragma unroll
  for (int d = -16; d <= 16; ++d) {
    const int U = (int)acc[d + 16].x + (int)acc[d + 16].y;
    if (d >= -wb && d <= wb) best_b = max(best_b, U);   // member b against rep a at shift d
    if (-d >= -wa && -d <= wa) best_a = max(best_a, U); // member a against rep b at shift -d
  }
}

__global__ void __launch_bounds__(64) prune128_bounds_kernel(ClipsDev ca, ClipsDev cb, PruneArgs pa, Threshold thr,
                                                             const int64_t* __restrict__ range_off,
                                                             uint32_t* __restrict__ mask, int64_t block0) {
  __shared__ int q1[128], q2[128];  // group-stage and coarse-stage survivors (positions in the range)
  __shared__ int q1len, q2len;
  const int64_t a = block0 + (int64_t)blockIdx.x;
  const int lane = threadIdx.x;
  const int ia = pa.anchor_ids ? pa.anchor_ids[a] : pa.order[a];
  const int na = ca.npix[ia];
  const int wa = ca.w[ia];
  const int64_t so_a = ca.sig_off[ia];
  const int64_t start = pa.lo ? (int64_t)pa.lo[a] : a + 1;
  int64_t end = pa.hi[a];
  int64_t first = start;
  if (pa.seg > 0) {  // this workgroup's segment of the range (uniform exit)
    first = start + (int64_t)blockIdx.y * pa.seg;
    end = min(end, first + (int64_t)pa.seg);
    if (first >= end) {
      if (threadIdx.x == 0) pa.counts[a * pa.n_seg + blockIdx.y] = 0;
      return;
    }
  }
  const int64_t roff = range_off[a] - pa.mask_bit0;
  if (lane == 0) {
    q1len = 0;
    q2len = 0;
  }
  __syncthreads();
  int64_t found = 0;

  // append the lanes with `keep` to a queue (its length in LDS)
  auto push = [&](int* q, int* len, bool keep, int value) {
    const unsigned long long km = __ballot(keep);
    const int base = *len;
    if (keep) q[base + __popcll(km & ((1ull << lane) - 1ull))] = value;
    __syncthreads();
    if (lane == 0) *len = base + __popcll(km);
    __syncthreads();
  };
  // drop the first k (<= 64) entries of a queue
  auto pop = [&](int* q, int* len, int k) {
    const int rest = *len - k;
    const int v = lane < rest ? q[k + lane] : 0;
    __syncthreads();
    if (lane < rest) q[lane] = v;
    if (lane == 0) *len = rest;
    __syncthreads();
  };

  auto exact_flush = [&](int count) {
    // lanes < count take queued partners; the rest idle through the same code
    const int pos = lane < count ? q2[lane] : -1;
    const int ib = pos >= 0 ? pa.order[start + pos] : pa.order[start];
    const int nb = cb.npix[ib];
    const int wb = cb.w[ib];
    const int64_t so_b = cb.sig_off[ib];
    int bb_r = 0, ba_r = 0, bb_c = 0, ba_c = 0;
    for (int dim = 0; dim < 2; ++dim) {
      const uint16_t* sa = dim ? ca.colsum + so_a : ca.rowsum + so_a;
      const uint16_t* sb = dim ? cb.colsum + so_b : cb.rowsum + so_b;
      uint32_t Be[64], Bo[64];
      const uint32_t* sa32 = reinterpret_cast<const uint32_t*>(sa);
      const uint4* sb4 = reinterpret_cast<const uint4*>(sb);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const uint4 v = sb4[q];
        Be[4 * q] = v.x; Be[4 * q + 1] = v.y; Be[4 * q + 2] = v.z; Be[4 * q + 3] = v.w;
      }
#pragma unroll
      for (int m = 0; m < 64; ++m) Bo[m] = __builtin_amdgcn_alignbit(Be[(m + 1) & 63], Be[m], 16);
      if (dim) exact_dim(sa32, Be, Bo, wb, wa, bb_c, ba_c);
      else exact_dim(sa32, Be, Bo, wb, wa, bb_r, ba_r);
    }
    const bool ok = pos >= 0 && (passes128(min(bb_r, bb_c), na, nb, thr) || passes128(min(ba_r, ba_c), na, nb, thr));
    if (ok) {
      const int64_t bit = roff + pos;
      atomicOr(mask + (bit >> 5), 1u << (bit & 31));
    }
    found += __popcll(__ballot(ok));
  };
  // the coarse stage on the first `count` group-stage survivors (lanes <
  // count); its survivors go to the exact stage's queue
  auto coarse_flush = [&](int count) {
    const int rel = lane < count ? q1[lane] : 0;
    const int64_t pos = start + rel;
    const int ib = pa.order[pos];
    const int nb = cb.npix[ib];
    const int wb = cb.w[ib];
    const int64_t so_b = cb.sig_off[ib];
    uint32_t W[64];
    const int wmax = max(wa, wb);
    const uint4* wr = reinterpret_cast<const uint4*>(cb.winrow + so_b);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const uint4 v = wr[q];
      W[4 * q] = v.x; W[4 * q + 1] = v.y; W[4 * q + 2] = v.z; W[4 * q + 3] = v.w;
    }
    const int cr = coarse_dim(ca.winrow + so_a, 8, W, wmax);
    const uint4* wc = reinterpret_cast<const uint4*>(cb.wincol + so_b);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const uint4 v = wc[q];
      W[4 * q] = v.x; W[4 * q + 1] = v.y; W[4 * q + 2] = v.z; W[4 * q + 3] = v.w;
    }
    const int cc = coarse_dim(ca.wincol + so_a, 8, W, wmax);
    const bool keep = lane < count && passes128(min(cr, cc), na, nb, thr);
    push(q2, &q2len, keep, rel);
  };

  // one call site per stage: each pass takes the next 64 partners through the
  // group stage, then runs the coarse stage on a full queue (or the rest once
  // the range is done) and the exact stage likewise
  int64_t b0 = first;
  for (;;) {
    const bool more = b0 < end;
    if (more) {
      const int64_t b = b0 + lane;
      const bool valid = b < end;
      const int64_t pos = valid ? b : start;
      const int nb = cb.npix[pa.order[pos]];
      bool keep = valid && na > 0 && nb > 0;
      if (pa.soa_grp) {
        const int gr = group_dim(ca.winrow + so_a, 8, pa.soa_grp, pa.soa_n, pos);
        const int gc = group_dim(ca.wincol + so_a, 8, pa.soa_grp + 16 * pa.soa_n, pa.soa_n, pos);
        keep = keep && passes128(min(gr, gc), na, nb, thr);
      }
      push(q1, &q1len, keep, (int)(b - start));
      b0 += 64;
    }
    if (q1len >= 64 || (!more && q1len > 0)) {
      const int k = min(q1len, 64);
      coarse_flush(k);
      pop(q1, &q1len, k);
    }
    if (q2len >= 64 || (!more && q1len == 0 && q2len > 0)) {
      const int k = min(q2len, 64);
      exact_flush(k);
      pop(q2, &q2len, k);
    }
    if (!more && q1len == 0 && q2len == 0) break;
  }
  if (lane == 0) pa.counts[pa.seg > 0 ? a * pa.n_seg + blockIdx.y : a] = found;
}

// Ordered write of the surviving pairs of each anchor from the bitmask.
__global__ void __launch_bounds__(64) prune128_write_kernel(PruneArgs pa, const int64_t* __restrict__ range_off,
                                                            const uint32_t* __restrict__ mask, int64_t block0) {
  const int64_t a = block0 + (int64_t)blockIdx.x;
  const int lane = threadIdx.x;
  const int ia = pa.anchor_ids ? pa.anchor_ids[a] : pa.order[a];
  const int64_t start = pa.lo ? (int64_t)pa.lo[a] : a + 1;
  int64_t len = pa.hi[a] - start;
  int64_t p_first = 0;
  if (pa.seg > 0) {  // this workgroup's segment (uniform exit)
    p_first = (int64_t)blockIdx.y * pa.seg;
    len = min(len, p_first + (int64_t)pa.seg);
    if (p_first >= len) return;
  }
  const int64_t roff = range_off[a] - pa.mask_bit0;
  int64_t o = pa.offs[pa.seg > 0 ? a * pa.n_seg + blockIdx.y : a] - pa.out_base;
  for (int64_t p0 = p_first; p0 < len; p0 += 64) {
    const int64_t p = p0 + lane;
    bool on = false;
    if (p < len) {
      const int64_t bit = roff + p;
      on = (mask[bit >> 5] >> (bit & 31)) & 1u;
    }
    const unsigned long long bm = __ballot(on);
    if (on) {
      const int64_t dst = o + __popcll(bm & ((1ull << lane) - 1ull));
      const int ib = pa.order[start + p];
      if (pa.order_ids) {
        pa.out_rep[dst] = min(ia, ib);
        pa.out_mem[dst] = max(ia, ib);
      } else {
        pa.out_rep[dst] = ia;
        pa.out_mem[dst] = ib;
      }
    }
    o += __popcll(bm);
  }
}

// Transposed partner sliding sums: pair q of the clip at position p of order
// goes to [q * n + p] (threads take positions fastest, so the stores coalesce).
__global__ void prune128_soa_kernel(ClipsDev cb, const int32_t* __restrict__ order, int64_t n,
                                    uint32_t* __restrict__ soa_row, uint32_t* __restrict__ soa_col) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 64 * n) return;
  const int q = (int)(t / n);
  const int64_t p = t - (int64_t)q * n;
  const int64_t so = cb.sig_off[order[p]];
  soa_row[t] = reinterpret_cast<const uint32_t*>(cb.winrow + so)[q];
  soa_col[t] = reinterpret_cast<const uint32_t*>(cb.wincol + so)[q];
}

// Transposed group maxima of the partner sliding sums: for dimension D (rows
// 0, columns 1) and block Y, M_G[Y] = max over the shifts d of group G of
// W[(8 Y + d) mod 128], groups [-16, 0] and [1, 16], packed as (M_0, M_1) at
// row 16 D + Y of a table of stride n (the clip at position p of order in
// column p).
__global__ void prune128_group_kernel(ClipsDev cb, const int32_t* __restrict__ order, int64_t n,
                                      uint32_t* __restrict__ soa_grp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 32 * n) return;
  const int r = (int)(t / n);  // 16 D + Y
  const int64_t p = t - (int64_t)r * n;
  const int D = r >> 4, Y = r & 15;
  const int64_t so = cb.sig_off[order[p]];
  const uint16_t* W = (D ? cb.wincol : cb.winrow) + so;
  int m0 = 0, m1 = 0;
  for (int d = -16; d <= 0; ++d) m0 = max(m0, (int)W[(8 * Y + d + 128) & 127]);
  for (int d = 1; d <= 16; ++d) m1 = max(m1, (int)W[(8 * Y + d + 128) & 127]);
  soa_grp[(int64_t)(16 * D + Y) * n + p] = pk_u16((uint32_t)m0, (uint32_t)m1);
}

hipError_t launch_prune128_soa(const ClipsDev& cb, const int32_t* order, int64_t n, uint32_t* soa_row,
                               uint32_t* soa_col, uint32_t* soa_grp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t total = 64 * n;
  hipLaunchKernelGGL(prune128_soa_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, cb, order, n,
                     soa_row, soa_col);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !soa_grp) return e;
  hipLaunchKernelGGL(prune128_group_kernel, dim3((unsigned)((32 * n + 255) / 256)), dim3(256), 0, s, cb, order, n,
                     soa_grp);
  return hipGetLastError();
}

hipError_t launch_prune128(const ClipsDev& ca, const ClipsDev& cb, const PruneArgs& pa, Threshold thr,
                           const int64_t* range_off, uint32_t* mask, bool write, hipStream_t s) {
  if (!write && (!pa.soa_row || !pa.soa_col || pa.soa_n <= 0)) return hipErrorInvalidValue;  // bounds pass reads them
  for (int64_t b0 = pa.a_begin; b0 < pa.n_anchor; b0 += LAUNCH_CHUNK) {
    const unsigned nb = (unsigned)std::min<int64_t>(LAUNCH_CHUNK, pa.n_anchor - b0);
    const dim3 grid(nb, pa.seg > 0 ? pa.n_seg : 1);
    if (write)
      hipLaunchKernelGGL(prune128_write_kernel, grid, dim3(64), 0, s, pa, range_off, (const uint32_t*)mask, b0);
    else
      hipLaunchKernelGGL(prune128_bounds_kernel, grid, dim3(64), 0, s, ca, cb, pa, thr, range_off, mask, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ca
