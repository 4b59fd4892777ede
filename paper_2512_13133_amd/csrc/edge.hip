// Edge track (paper Sec. 2.2.2 edge movement constraint; Sec. 3.2.2, Eq. 6).
//
// One 64-lane wavefront per unordered pair, both directions in turn.  For a
// direction (member m against representative r):
//   1. T0 = per-axis Min-Max midpoint of the two global bounding boxes;
//   2. the overlap relation member-polygon x rep-polygon at T0, from the row
//      runs of both clips (linear shift, zero fill): lanes sweep rep rows,
//      merge them with the shifted member row and OR (p, q) bits into two
//      64 x 64-bit LDS masks (by member row and by rep column);
//   3. the fewer side (both if equal) must overlap exactly one polygon each;
//   4. per axis, s = clamp(round-half-toward-zero((d_min + d_max)/2), +-w) over
//      the bounding-box edge displacements of the matched pairs, residual
//      E = max(d_max - s, s - d_min), E = max(E_x, E_y);
//   5. the relation is rebuilt at s and the matching must be unchanged;
//   6. bit = correspondence ok and E <= T_edge.
#include "kernels.h"
#include "pair_common.h"

namespace ca {

__device__ __forceinline__ int rhtz_half(int m2) { return m2 >= 0 ? m2 / 2 : -((-m2) / 2); }

__device__ __forceinline__ void minmax_axis(int lo, int hi, int w, int& s, int& E) {
  s = rhtz_half(lo + hi);
  s = max(-w, min(w, s));
  E = max(hi - s, s - lo);
}

// Build the overlap relation at shift (dy, dx).  relM[p] bit q: member p
// overlaps rep q; relR[q] bit p likewise.  Wave-synchronous (64 threads).
__device__ void overlap_relation(const ClipsDev& cs, int m, int r, int N, int dy, int dx,
                                 unsigned long long* relM, unsigned long long* relR) {
  const int lane = threadIdx.x;
  relM[lane] = 0ull;
  relR[lane] = 0ull;
  __syncthreads();
  const uint16_t* rp_m = cs.run_rowptr + cs.rowptr_off[m];
  const uint16_t* rp_r = cs.run_rowptr + cs.rowptr_off[r];
  const uint32_t* ru_m = cs.runs + cs.run_off[m];
  const uint32_t* ru_r = cs.runs + cs.run_off[r];
  const int y0 = max(0, -dy), y1 = min(N, N - dy);
  for (int y = y0 + lane; y < y1; y += 64) {
    const int ym = y + dy;
    int a = rp_r[y], ae = rp_r[y + 1];
    int b = rp_m[ym], be = rp_m[ym + 1];
    while (a < ae && b < be) {
      const uint32_t ra = ru_r[a], rb = ru_m[b];
      const int a0 = ra & 511, a1 = (ra >> 9) & 511, qa = (ra >> 18) & 63;
      const int b0 = (int)(rb & 511) - dx, b1 = (int)((rb >> 9) & 511) - dx, pb = (rb >> 18) & 63;
      if (max(a0, b0) < min(a1, b1)) {
        atomicOr(&relM[pb], 1ull << qa);
        atomicOr(&relR[qa], 1ull << pb);
      }
      if (a1 < b1) ++a;
      else ++b;
    }
  }
  __syncthreads();
}

// Exactly-one rule from the fewer side (both if equal).  Wave-wide result.
__device__ bool correspondence_ok(const unsigned long long* relM, const unsigned long long* relR,
                                  int Pm, int Pr, int* flag) {
  const int lane = threadIdx.x;
  if (lane == 0) *flag = 1;
  __syncthreads();
  if (Pm <= Pr && lane < Pm && __popcll(relM[lane]) != 1) *flag = 0;
  if (Pr <= Pm && lane < Pr && __popcll(relR[lane]) != 1) *flag = 0;
  __syncthreads();
  const bool ok = *flag != 0;
  __syncthreads();
  return ok;
}

__global__ void __launch_bounds__(64) edge_kernel(ClipsDev cs, PairIO io, Threshold thr) {
  __shared__ unsigned long long relM[MAX_POLY], relR[MAX_POLY];
  __shared__ unsigned long long relM0[MAX_POLY], relR0[MAX_POLY];
  __shared__ int sflag;
  __shared__ int red[4][64];
  const int64_t k = blockIdx.x;
  const int lane = threadIdx.x;
  const int j = io.rep[k], i = io.mem[k];
  const int N = cs.N[i];
  if (lane == 0) { io.bits[k] = 0; io.flags[k] = 0; }
  for (int d = 0; d < 2; ++d) {
    const int m = d == 0 ? i : j, r = d == 0 ? j : i;
    const int w = cs.w[m];
    const int Pm = cs.npoly[m], Pr = cs.npoly[r];
    const uint32_t nomatch = d == 0 ? CA_FLAG_NO_MATCH_FWD : CA_FLAG_NO_MATCH_REV;
    const uint32_t recheck = d == 0 ? CA_FLAG_RECHECK_FWD : CA_FLAG_RECHECK_REV;
    if (Pm <= 0 || Pr <= 0) {
      if (lane == 0) {
        write_direction(io, k, d, 0, 0, -1, 0.0, false);
        io.flags[k] |= nomatch | ((Pm == 0 || Pr == 0) ? CA_FLAG_EMPTY : 0u);
      }
      continue;
    }
    const int16_t* gm = cs.gbox + 4 * m;
    const int16_t* gr = cs.gbox + 4 * r;
    int s0x, s0y, e_unused;
    {
      const int a = gm[0] - gr[0], b = gm[1] - gr[1];
      minmax_axis(min(a, b), max(a, b), w, s0x, e_unused);
      const int c = gm[2] - gr[2], e = gm[3] - gr[3];
      minmax_axis(min(c, e), max(c, e), w, s0y, e_unused);
    }
    overlap_relation(cs, m, r, N, s0y, s0x, relM0, relR0);
    if (!correspondence_ok(relM0, relR0, Pm, Pr, &sflag)) {
      if (lane == 0) {
        write_direction(io, k, d, s0y, s0x, -1, 0.0, false);
        io.flags[k] |= nomatch;
      }
      __syncthreads();
      continue;
    }
    // displacement extremes over matched pairs (fewer side drives the matching)
    const int16_t* bm = cs.boxes + (int64_t)m * MAX_POLY * 4;
    const int16_t* br = cs.boxes + (int64_t)r * MAX_POLY * 4;
    int xlo = 1 << 20, xhi = -(1 << 20), ylo = 1 << 20, yhi = -(1 << 20);
    const bool from_member = Pm <= Pr;
    const int P = from_member ? Pm : Pr;
    if (lane < P) {
      int p, qq;
      if (from_member) { p = lane; qq = __ffsll((unsigned long long)relM0[lane]) - 1; }
      else { qq = lane; p = __ffsll((unsigned long long)relR0[lane]) - 1; }
      const int16_t* a = bm + 4 * p;
      const int16_t* b = br + 4 * qq;
      const int d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2], d3 = a[3] - b[3];
      xlo = min(d0, d1); xhi = max(d0, d1);
      ylo = min(d2, d3); yhi = max(d2, d3);
    }
    red[0][lane] = xlo; red[1][lane] = xhi; red[2][lane] = ylo; red[3][lane] = yhi;
    __syncthreads();
    for (int s = 32; s > 0; s >>= 1) {
      if (lane < s) {
        red[0][lane] = min(red[0][lane], red[0][lane + s]);
        red[1][lane] = max(red[1][lane], red[1][lane + s]);
        red[2][lane] = min(red[2][lane], red[2][lane + s]);
        red[3][lane] = max(red[3][lane], red[3][lane + s]);
      }
      __syncthreads();
    }
    int sx, sy, ex, ey;
    minmax_axis(red[0][0], red[1][0], w, sx, ex);
    minmax_axis(red[2][0], red[3][0], w, sy, ey);
    const int E = max(ex, ey);
    __syncthreads();
    overlap_relation(cs, m, r, N, sy, sx, relM, relR);
    bool ok = correspondence_ok(relM, relR, Pm, Pr, &sflag);
    if (ok) {
      if (lane == 0) sflag = 1;
      __syncthreads();
      if (Pm <= Pr && lane < Pm && relM[lane] != relM0[lane]) sflag = 0;
      if (Pr <= Pm && lane < Pr && relR[lane] != relR0[lane]) sflag = 0;
      __syncthreads();
      ok = sflag != 0;
      __syncthreads();
    }
    if (lane == 0) {
      write_direction(io, k, d, sy, sx, E, 0.0, ok && (int64_t)E <= thr.p);
      if (!ok) io.flags[k] |= recheck;
    }
    __syncthreads();
  }
}

}  // namespace ca

namespace ca {

hipError_t launch_edge(const ClipsDev& cs, const PairIO& io, Threshold thr, hipStream_t s) {
  if (io.n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(edge_kernel, dim3((unsigned)io.n_pairs), dim3(64), 0, s, cs, io, thr);
  return hipGetLastError();
}

}  // namespace ca
