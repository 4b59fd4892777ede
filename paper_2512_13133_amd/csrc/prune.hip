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
// 2 T_edge in width and in height (E >= |width difference| / 2).
//
// Both kernels run twice: once counting survivors per anchor, once writing
// them at the anchor's exclusive-prefix offset in partner order, so the
// output order is deterministic.
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

// One 64-lane workgroup per anchor position a in `order`.
__global__ void __launch_bounds__(64) cosine_prune_kernel(ClipsDev cs, PruneArgs pa, Threshold thr) {
  __shared__ uint16_t ra[256], ca_[256], rb[256], cb[256];
  __shared__ int red[64];
  const int64_t a = blockIdx.x;
  const int lane = threadIdx.x;
  const int ia = pa.order[a];
  const int N = cs.N[ia];
  const int na = cs.npix[ia];
  const int wa = cs.w[ia];
  for (int y = lane; y < N; y += 64) {
    ra[y] = cs.rowsum[cs.sig_off[ia] + y];
    ca_[y] = cs.colsum[cs.sig_off[ia] + y];
  }
  int64_t written = 0;
  const int64_t end = pa.hi[a];
  for (int64_t b = a + 1; b < end; ++b) {
    const int ib = pa.order[b];
    const int nb = cs.npix[ib];
    const int wb = cs.w[ib];
    __syncthreads();
    for (int y = lane; y < N; y += 64) {
      rb[y] = cs.rowsum[cs.sig_off[ib] + y];
      cb[y] = cs.colsum[cs.sig_off[ib] + y];
    }
    __syncthreads();
    // U(d) = sum_y min(sig_a[y], sig_b[(y + d) mod N]) for member b against rep a;
    // the member-a direction sees U(-d).
    const Axis ax = make_axis(max(wa, wb), N);
    int best_row_b = 0, best_col_b = 0, best_row_a = 0, best_col_a = 0;
    for (int l = lane; l < ax.L; l += 64) {
      const int dshift = l - ax.base;
      int sd = dshift % N;
      if (sd < 0) sd += N;
      int ur = 0, uc = 0;
      for (int y = 0; y < N; ++y) {
        int yy = y + sd;
        if (yy >= N) yy -= N;
        ur += min((int)ra[y], (int)rb[yy]);
        uc += min((int)ca_[y], (int)cb[yy]);
      }
      if (in_window(dshift, wb, N)) { best_row_b = max(best_row_b, ur); best_col_b = max(best_col_b, uc); }
      const int nd = neg_rep(dshift, N);
      if (in_window(nd, wa, N)) { best_row_a = max(best_row_a, ur); best_col_a = max(best_col_a, uc); }
    }
    // wave maxima of the four values (LDS tree)
    int vals[4] = {best_row_b, best_col_b, best_row_a, best_col_a};
    int res[4];
    for (int t = 0; t < 4; ++t) {
      red[lane] = vals[t];
      __syncthreads();
      for (int s = 32; s > 0; s >>= 1) {
        if (lane < s) red[lane] = max(red[lane], red[lane + s]);
        __syncthreads();
      }
      res[t] = red[0];
      __syncthreads();
    }
    const int64_t bnd_b = min(res[0], res[1]);
    const int64_t bnd_a = min(res[2], res[3]);
    const bool pass = na > 0 && nb > 0 &&
                      (bound_passes(bnd_b, na, nb, thr) || bound_passes(bnd_a, na, nb, thr));
    if (pass) {
      if (pa.offs && lane == 0) {
        const int64_t o = pa.offs[a] + written;
        pa.out_rep[o] = ia;
        pa.out_mem[o] = ib;
      }
      ++written;
    }
  }
  if (!pa.offs && lane == 0) pa.counts[a] = written;
}

// Edge track: one 64-lane workgroup per anchor a; lanes take partners b in
// [a+1, hi[a]) of the same raster size, 64 at a time.
__global__ void __launch_bounds__(64) edge_prune_kernel(ClipsDev cs, PruneArgs pa, Threshold thr) {
  __shared__ int wsum[64];
  const int64_t a = blockIdx.x;
  const int lane = threadIdx.x;
  const int ia = pa.order[a];
  const int Pa = cs.npoly[ia];
  const int16_t* ba = cs.boxes + (int64_t)ia * MAX_POLY * 4;
  const int64_t end = pa.hi[a];
  const int tol = (int)(2 * thr.p);
  int64_t written = 0;
  for (int64_t b0 = a + 1; b0 < end; b0 += 64) {
    const int64_t b = b0 + lane;
    int pass = 0;
    int ib = -1;
    if (b < end) {
      ib = pa.order[b];
      const int Pb = cs.npoly[ib];
      if (Pa > 0 && Pb > 0) {
        const int16_t* bb = cs.boxes + (int64_t)ib * MAX_POLY * 4;
        pass = 1;
        // polygons of the fewer side each need a size-compatible partner
        for (int side = 0; side < 2 && pass; ++side) {
          const bool check = side == 0 ? (Pa <= Pb) : (Pb <= Pa);
          if (!check) continue;
          const int16_t* X = side == 0 ? ba : bb;
          const int16_t* Y = side == 0 ? bb : ba;
          const int PX = side == 0 ? Pa : Pb, PY = side == 0 ? Pb : Pa;
          for (int p = 0; p < PX && pass; ++p) {
            const int wx = X[4 * p + 1] - X[4 * p], hx = X[4 * p + 3] - X[4 * p + 2];
            bool found = false;
            for (int qq = 0; qq < PY && !found; ++qq) {
              const int wy = Y[4 * qq + 1] - Y[4 * qq], hy = Y[4 * qq + 3] - Y[4 * qq + 2];
              found = abs(wx - wy) <= tol && abs(hx - hy) <= tol;
            }
            if (!found) pass = 0;
          }
        }
      }
    }
    // ordered compaction within the chunk
    wsum[lane] = pass;
    __syncthreads();
    int before = 0, total = 0;
    for (int t = 0; t < 64; ++t) {
      before += (t < lane) ? wsum[t] : 0;
      total += wsum[t];
    }
    if (pass && pa.offs) {
      const int64_t o = pa.offs[a] + written + before;
      const int x = min(ia, ib), y = max(ia, ib);
      pa.out_rep[o] = x;
      pa.out_mem[o] = y;
    }
    written += total;
    __syncthreads();
  }
  if (!pa.offs && lane == 0) pa.counts[a] = written;
}

}  // namespace ca

namespace ca {

hipError_t launch_cosine_prune(const ClipsDev& cs, const PruneArgs& pa, Threshold thr, hipStream_t s) {
  if (pa.n_anchor == 0) return hipSuccess;
  hipLaunchKernelGGL(cosine_prune_kernel, dim3((unsigned)pa.n_anchor), dim3(64), 0, s, cs, pa, thr);
  return hipGetLastError();
}

hipError_t launch_edge_prune(const ClipsDev& cs, const PruneArgs& pa, Threshold thr, hipStream_t s) {
  if (pa.n_anchor == 0) return hipSuccess;
  hipLaunchKernelGGL(edge_prune_kernel, dim3((unsigned)pa.n_anchor), dim3(64), 0, s, cs, pa, thr);
  return hipGetLastError();
}

}  // namespace ca
