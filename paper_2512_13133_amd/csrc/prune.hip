// Multi-stage pre-screening with safe bounds (paper Sec. 3.1 stage 1; Table 2,
// graph construction).  A pair rejected here can never pass the constraint,
// so the pruned cover equals the unpruned one.
//
// Cosine track.  Clips of one raster size are ordered by pixel count; the
// area bound B1 (cos <= sqrt(n_small / n_large)) then leaves each anchor a
// contiguous range of larger partners, computed on the host.  For each
// partner the signature bound B2 runs on one wavefront: lanes own window
// positions and sum min(row_rep[y], row_mem[(y + dy) mod N]) over rows (and
// likewise for columns), the wave takes the window maximum, and the pair
// survives if the bound can still beat the threshold in either direction.
//
// Edge track.  B3: every polygon on the side with fewer polygons (both if
// equal) needs a partner polygon whose bounding box differs by at most
// 2 T_edge in width and in height (E >= |width difference| / 2).  It implies
// that the fewer side's widest polygon has a partner at most 2 T_edge
// narrower, so max w(fewer) <= max w(other) + 2 T_edge, and likewise for the
// narrowest and for heights: four comparisons of per-clip extremes that drop
// most pairs of many-polygon clips before the polygon loops run, on queued
// survivors.
//
// Both kernels run twice: once counting survivors per anchor, once writing
// them at the anchor's exclusive-prefix offset in partner order, so the
// output order is deterministic.  The cosine kernel first applies a coarse
// form of B2 over 8-row blocks (looser, eight times cheaper) and runs the
// exact B2 only on pairs the coarse bound cannot reject.
#include "kernels.h"
#include "pair_common.h"

namespace ca {

__device__ __forceinline__ bool bound_passes(int64_t b, int n1, int n2, Threshold t) {
  const unsigned __int128 lhs = (unsigned __int128)((uint64_t)b * (uint64_t)b) *
                                (unsigned __int128)((uint64_t)t.q * (uint64_t)t.q);
  const unsigned __int128 rhs = (unsigned __int128)((uint64_t)t.p * (uint64_t)t.p) *
                                (unsigned __int128)((uint64_t)n1 * (uint64_t)n2);
  return lhs > rhs;
}

// Lane-order prefix of a wave predicate and the wave total (ordered compaction).
__device__ __forceinline__ int wave_prefix(bool pred, int lane, int* total) {
  const unsigned long long m = __ballot(pred);
  *total = __popcll(m);
  return __popcll(m & ((1ull << lane) - 1ull));
}

// One wavefront per anchor position a in `order`; lanes take partners b in
// [a+1, hi[a]), 64 at a time.
//   coarse stage: per lane, the 8-row block bound
//       U(d) <= sum_Y min(A_rep[Y], W_mem[(8 Y + d) mod N]),
//     A = the anchor's 8-row block sums, W = the partner's sliding 8-row sums
//     (held transposed in LDS so every lane reads its own column), maximised
//     over the union of both windows; it bounds both directions at once;
//   exact stage: for coarse survivors, one at a time, lanes own (rows or
//     columns, shift) positions of the signature bound B2 and the wave takes
//     the maxima of each direction's window with shuffles.
__global__ void __launch_bounds__(64) cosine_prune_kernel(ClipsDev cs, PruneArgs pa, Threshold thr,
                                                          int64_t block0) {
  extern __shared__ uint16_t sT[];  // [2][N][64] partner sliding sums, transposed
  __shared__ int ra[256], ca_[256], rb[256], cb[256];
  __shared__ int Ar[32], Ac[32];
  const int64_t a = block0 + (int64_t)blockIdx.x;
  const int lane = threadIdx.x;
  const int ia = pa.order[a];
  const int N = cs.N[ia];
  const int na = cs.npix[ia];
  const int wa = cs.w[ia];
  const int64_t so_a = cs.sig_off[ia];
  for (int y = lane; y < N; y += 64) {
    ra[y] = cs.rowsum[so_a + y];
    ca_[y] = cs.colsum[so_a + y];
  }
  if (lane < N / 8) {
    Ar[lane] = cs.winrow[so_a + 8 * lane];
    Ac[lane] = cs.wincol[so_a + 8 * lane];
  }
  __syncthreads();
  uint16_t* TR = sT;
  uint16_t* TC = sT + N * 64;
  int64_t written = 0;
  const int64_t end = pa.hi[a];
  for (int64_t b0 = a + 1; b0 < end; b0 += 64) {
    const int64_t b = b0 + lane;
    const bool valid = b < end;
    const int ib = valid ? pa.order[b] : ia;
    const int nb = cs.npix[ib];
    const int wb = cs.w[ib];
    const int64_t so_b = cs.sig_off[ib];
    // partner sliding sums into this lane's LDS column
    for (int t = 0; t < N; t += 8) {
      const uint4 vr = *reinterpret_cast<const uint4*>(cs.winrow + so_b + t);
      const uint4 vc = *reinterpret_cast<const uint4*>(cs.wincol + so_b + t);
      const uint32_t r4[4] = {vr.x, vr.y, vr.z, vr.w};
      const uint32_t c4[4] = {vc.x, vc.y, vc.z, vc.w};
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        TR[(t + e) * 64 + lane] = (uint16_t)(r4[e >> 1] >> (16 * (e & 1)));
        TC[(t + e) * 64 + lane] = (uint16_t)(c4[e >> 1] >> (16 * (e & 1)));
      }
    }
    const Axis ax = make_axis(max(wa, wb), N);
    int best_r = 0, best_c = 0;
    for (int l = 0; l < ax.L; ++l) {
      int sd = (l - ax.base) % N;
      if (sd < 0) sd += N;
      int ur = 0, uc = 0;
      for (int Y = 0; Y < N / 8; ++Y) {
        const int t = (8 * Y + sd) & (N - 1);
        ur += min(Ar[Y], (int)TR[t * 64 + lane]);
        uc += min(Ac[Y], (int)TC[t * 64 + lane]);
      }
      best_r = max(best_r, ur);
      best_c = max(best_c, uc);
    }
    const bool pass_c = valid && na > 0 && nb > 0 && bound_passes(min(best_r, best_c), na, nb, thr);
    bool pass = false;
    unsigned long long todo = __ballot(pass_c);
    while (todo) {
      const int src = __ffsll((unsigned long long)todo) - 1;
      todo &= todo - 1ull;
      const int ibs = __shfl(ib, src), nbs = __shfl(nb, src), wbs = __shfl(wb, src);
      const int64_t sob = cs.sig_off[ibs];
      __syncthreads();
      for (int y = lane; y < N; y += 64) {
        rb[y] = cs.rowsum[sob + y];
        cb[y] = cs.colsum[sob + y];
      }
      __syncthreads();
      // U(d) = sum_y min(sig_a[y], sig_b[(y + d) mod N]) serves member b against
      // rep a at shift d, and member a against rep b at shift -d
      const Axis axs = make_axis(max(wa, wbs), N);
      int bb_r = 0, bb_c = 0, ba_r = 0, ba_c = 0;
      for (int qpos = lane; qpos < 2 * axs.L; qpos += 64) {
        const int dim = qpos >= axs.L;
        const int d = qpos - dim * axs.L - axs.base;
        int sd = d % N;
        if (sd < 0) sd += N;
        const int* sa = dim ? ca_ : ra;
        const int* sbv = dim ? cb : rb;
        int U = 0;
        for (int y = 0; y < N; ++y) {
          int yy = y + sd;
          if (yy >= N) yy -= N;
          U += min(sa[y], sbv[yy]);
        }
        if (in_window(d, wbs, N)) { if (dim) bb_c = max(bb_c, U); else bb_r = max(bb_r, U); }
        if (in_window(neg_rep(d, N), wa, N)) { if (dim) ba_c = max(ba_c, U); else ba_r = max(ba_r, U); }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        bb_r = max(bb_r, __shfl_xor(bb_r, off));
        bb_c = max(bb_c, __shfl_xor(bb_c, off));
        ba_r = max(ba_r, __shfl_xor(ba_r, off));
        ba_c = max(ba_c, __shfl_xor(ba_c, off));
      }
      const bool ok = bound_passes(min(bb_r, bb_c), na, nbs, thr) || bound_passes(min(ba_r, ba_c), na, nbs, thr);
      if (lane == src) pass = ok;
    }
    int total = 0;
    const int before = wave_prefix(pass, lane, &total);
    if (pass && pa.offs) {
      const int64_t o = pa.offs[a] - pa.out_base + written + before;
      pa.out_rep[o] = ia;
      pa.out_mem[o] = ib;
    }
    written += total;
  }
  if (!pa.offs && lane == 0) pa.counts[a] = written;
}

// B3 for the pair (anchor with Pa polygons, box sizes from ba and hashes
// from ha; partner at position b with Pb polygons): the polygons of the fewer
// side (both if equal) each need a size-compatible (and, over contours,
// equally hashed) partner.
__device__ __forceinline__ bool b3_pass(const PruneArgs& pa, const int16_t* ba, const uint32_t* ha, int Pa,
                                        int64_t b, int Pb, int tol, bool topo) {
  auto wh_a = [&](int q) { return (uint32_t)(uint16_t)(ba[4 * q + 1] - ba[4 * q]) |
                                  ((uint32_t)(uint16_t)(ba[4 * q + 3] - ba[4 * q + 2]) << 16); };
  auto wh_b = [&](int qq) { return pa.soa_wh[(int64_t)qq * pa.soa_n + b]; };
  bool pass = true;
  for (int side = 0; side < 2 && pass; ++side) {
    const bool check = side == 0 ? (Pa <= Pb) : (Pb <= Pa);
    if (!check) continue;
    const int PX = side == 0 ? Pa : Pb, PY = side == 0 ? Pb : Pa;
    for (int p = 0; p < PX && pass; ++p) {
      const uint32_t x = side == 0 ? wh_a(p) : wh_b(p);
      const int wx = (int)(x & 0xffffu), hx = (int)(x >> 16);
      const uint32_t tx = !topo ? 0u : (side == 0 ? ha[p] : pa.soa_hash[(int64_t)p * pa.soa_n + b]);
      bool hit = false;
      for (int qq = 0; qq < PY && !hit; ++qq) {
        const uint32_t y = side == 0 ? wh_b(qq) : wh_a(qq);
        const int wy = (int)(y & 0xffffu), hy = (int)(y >> 16);
        hit = abs(wx - wy) <= tol && abs(hx - hy) <= tol;
        if (hit && topo) hit = tx == (side == 0 ? pa.soa_hash[(int64_t)qq * pa.soa_n + b] : ha[qq]);
      }
      if (!hit) pass = false;
    }
  }
  return pass;
}

// Edge track: one 64-lane workgroup per anchor a; lanes take partners b in
// [a+1, hi[a]) of the same raster size, 64 at a time, through the extremes
// test; its survivors are queued in LDS and run B3 on full waves, and their
// pass bits are ORed into the mask, one atomic per mask word a wave touches.
// The caller zeroes the mask; the anchor's range starts on a 64-bit word
// (range_off[a] in bits); counts[a] gets the survivors.
__global__ void __launch_bounds__(64) edge_prune_kernel(ClipsDev cs, PruneArgs pa, Threshold thr,
                                                        const int64_t* __restrict__ range_off,
                                                        unsigned long long* __restrict__ mask, int64_t block0) {
  __shared__ int q[128];  // extremes-test survivors (offsets in the range)
  __shared__ int qlen;
  const int64_t a = block0 + (int64_t)blockIdx.x;
  const int lane = threadIdx.x;
  const int ia = pa.order[a];
  const bool topo = pa.soa_hash != nullptr;
  // over contours, a clip without contour data matches nothing
  const int Pa = (topo && cs.cstat[ia] < 0) ? -1 : cs.npoly[ia];
  const int16_t* ba = cs.boxes + (int64_t)ia * MAX_POLY * 4;
  const uint32_t* ha = topo ? cs.chash + (int64_t)ia * MAX_POLY : nullptr;
  const int64_t end = pa.hi[a];
  const int tol = (int)(2 * thr.p);
  unsigned long long* m = mask + ((range_off[a] - pa.mask_bit0) >> 6);
  int64_t found = 0;
  if (Pa <= 0) {  // uniform: an anchor without polygons matches nothing
    if (lane == 0) pa.counts[a] = 0;
    return;
  }
  const uint32_t ea_w = pa.soa_ext[a], ea_h = pa.soa_ext[pa.soa_n + a];
  if (lane == 0) qlen = 0;
  __syncthreads();
  // the extremes of the fewer side X within tol of those of the other side Y
  auto ext_ok = [&](uint32_t xw, uint32_t xh, uint32_t yw, uint32_t yh) {
    return (int)(xw >> 16) <= (int)(yw >> 16) + tol && (int)(xw & 0xffffu) + tol >= (int)(yw & 0xffffu) &&
           (int)(xh >> 16) <= (int)(yh >> 16) + tol && (int)(xh & 0xffffu) + tol >= (int)(yh & 0xffffu);
  };
  for (int64_t b0 = a + 1;;) {
    const bool more = b0 < end;
    if (qlen >= 64 || (!more && qlen > 0)) {
      // B3 on the first `count` queued partners (lanes < count)
      const int count = min(qlen, 64);
      const int rel = lane < count ? q[lane] : -1;
      bool pass = false;
      if (rel >= 0) {
        const int64_t b = a + 1 + rel;
        pass = b3_pass(pa, ba, ha, Pa, b, pa.soa_np[b], tol, topo);
      }
      // lanes holding the same mask word are consecutive (the queue keeps the
      // range order): OR their bits down the run, then its first lane alone
      // writes the word
      const int word = rel >= 0 ? (rel >> 6) : -1;
      unsigned long long bits = pass ? 1ull << (rel & 63) : 0ull;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int w2 = __shfl_down(word, off);
        const unsigned long long b2 = __shfl_down(bits, off);
        if (lane + off < 64 && w2 == word) bits |= b2;
      }
      const int wprev = __shfl_up(word, 1);
      if (word >= 0 && bits && (lane == 0 || wprev != word)) atomicOr(m + word, bits);
      found += __popcll(__ballot(pass));
      const int rest = qlen - count;
      const int v = lane < rest ? q[count + lane] : 0;
      __syncthreads();
      if (lane < rest) q[lane] = v;
      if (lane == 0) qlen = rest;
      __syncthreads();
      continue;
    }
    if (!more) break;
    const int64_t b = b0 + lane;
    bool keep = false;
    if (b < end) {
      const int Pb = pa.soa_np[b];
      if (Pb > 0) {
        const uint32_t eb_w = pa.soa_ext[b], eb_h = pa.soa_ext[pa.soa_n + b];
        keep = (Pa > Pb || ext_ok(ea_w, ea_h, eb_w, eb_h)) && (Pb > Pa || ext_ok(eb_w, eb_h, ea_w, ea_h));
      }
    }
    const unsigned long long km = __ballot(keep);
    const int base = qlen;
    if (keep) q[base + __popcll(km & ((1ull << lane) - 1ull))] = (int)(b - a - 1);
    __syncthreads();
    if (lane == 0) qlen = base + __popcll(km);
    __syncthreads();
    b0 += 64;
  }
  if (lane == 0) pa.counts[a] = found;
}

}  // namespace ca

namespace ca {

hipError_t launch_cosine_prune(const ClipsDev& cs, const PruneArgs& pa, Threshold thr, int maxN, hipStream_t s) {
  for (int64_t b0 = pa.a_begin; b0 < pa.n_anchor; b0 += LAUNCH_CHUNK) {
    const unsigned nb = (unsigned)std::min<int64_t>(LAUNCH_CHUNK, pa.n_anchor - b0);
    hipLaunchKernelGGL(cosine_prune_kernel, dim3(nb), dim3(64), (size_t)256 * maxN, s, cs, pa, thr, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Transposed polygon box sizes and counts of the clips in `order`: polygon q of
// the clip at position p at [q * n + p] (threads take positions fastest).
__global__ void edge_soa_kernel(ClipsDev cs, const int32_t* __restrict__ order, int64_t n,
                                uint32_t* __restrict__ soa_wh, int32_t* __restrict__ soa_np,
                                uint32_t* __restrict__ soa_hash) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)MAX_POLY * n) return;
  const int q = (int)(t / n);
  const int64_t p = t - (int64_t)q * n;
  const int i = order[p];
  // over contours (soa_hash given) a clip without contour data matches nothing
  const int np = (soa_hash && cs.cstat[i] < 0) ? -1 : cs.npoly[i];
  uint32_t v = 0, h = 0;
  if (q < np) {
    const int16_t* bx = cs.boxes + ((int64_t)i * MAX_POLY + q) * 4;
    v = (uint32_t)(uint16_t)(bx[1] - bx[0]) | ((uint32_t)(uint16_t)(bx[3] - bx[2]) << 16);
    if (soa_hash) h = cs.chash[(int64_t)i * MAX_POLY + q];
  }
  soa_wh[t] = v;
  if (soa_hash) soa_hash[t] = h;
  if (q == 0) soa_np[p] = np;
}

// Extremes of the polygon box sizes of the clip at position p of order:
// (min w | max w << 16) at [p], (min h | max h << 16) at [n + p]; zeros for a
// clip without polygons (or, over contours, without contour data).
__global__ void edge_ext_kernel(ClipsDev cs, const int32_t* __restrict__ order, int64_t n, bool topo,
                                uint32_t* __restrict__ soa_ext) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int i = order[p];
  const int np = (topo && cs.cstat[i] < 0) ? -1 : min(cs.npoly[i], MAX_POLY);
  int w0 = 0xffff, w1 = 0, h0 = 0xffff, h1 = 0;
  for (int q = 0; q < np; ++q) {
    const int16_t* bx = cs.boxes + ((int64_t)i * MAX_POLY + q) * 4;
    const int w = bx[1] - bx[0], h = bx[3] - bx[2];
    w0 = min(w0, w); w1 = max(w1, w);
    h0 = min(h0, h); h1 = max(h1, h);
  }
  if (np <= 0) w0 = h0 = 0;
  soa_ext[p] = (uint32_t)w0 | ((uint32_t)w1 << 16);
  soa_ext[n + p] = (uint32_t)h0 | ((uint32_t)h1 << 16);
}

hipError_t launch_edge_soa(const ClipsDev& cs, const int32_t* order, int64_t n, uint32_t* soa_wh, int32_t* soa_np,
                           hipStream_t s, uint32_t* soa_hash, uint32_t* soa_ext) {
  if (n == 0) return hipSuccess;
  if (soa_hash && !cs.cstat) return hipErrorInvalidValue;  // hashes need the contour tables
  const int64_t total = (int64_t)MAX_POLY * n;
  hipLaunchKernelGGL(edge_soa_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, cs, order, n, soa_wh,
                     soa_np, soa_hash);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !soa_ext) return e;
  hipLaunchKernelGGL(edge_ext_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cs, order, n,
                     soa_hash != nullptr, soa_ext);
  return hipGetLastError();
}

hipError_t launch_edge_prune(const ClipsDev& cs, const PruneArgs& pa, Threshold thr, const int64_t* range_off,
                             unsigned long long* mask, hipStream_t s) {
  if (pa.n_anchor == 0) return hipSuccess;
  if (!pa.soa_wh || !pa.soa_np || !pa.soa_ext || pa.soa_n <= 0) return hipErrorInvalidValue;  // the kernel reads them
  for (int64_t b0 = pa.a_begin; b0 < pa.n_anchor; b0 += LAUNCH_CHUNK) {
    const unsigned nb = (unsigned)std::min<int64_t>(LAUNCH_CHUNK, pa.n_anchor - b0);
    hipLaunchKernelGGL(edge_prune_kernel, dim3(nb), dim3(64), 0, s, cs, pa, thr, range_off, mask, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ca
