// Edge track (paper Sec. 2.2.2 edge movement constraint; Sec. 3.2.2, Eq. 6).
//
// One 64-lane wavefront takes a batch of pairs.  For a direction (member m
// against representative r):
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

// Displacement extremes (member minus representative) over the contour edges
// of member polygon p of clip m and representative polygon q of clip r, edge k
// against edge k of the two canonical lists; false when the direction codes
// or contour boundaries differ (the polygons have no edge correspondence).
__device__ bool contour_pair(const ClipsDev& cs, int m, int r, int p, int q, int& xlo, int& xhi, int& ylo, int& yhi) {
  const uint16_t* pm = cs.cpoly + (int64_t)m * (MAX_POLY + 1);
  const uint16_t* pr = cs.cpoly + (int64_t)r * (MAX_POLY + 1);
  const int a0 = pm[p], n = pm[p + 1] - a0, b0 = pr[q];
  if (pr[q + 1] - b0 != n) return false;
  const uint16_t* em = cs.cedges + cs.cedge_off[m] + a0;
  const uint16_t* er = cs.cedges + cs.cedge_off[r] + b0;
  for (int k = 0; k < n; ++k) {
    const int u = em[k], v = er[k];
    if ((u ^ v) >> 9) return false;
    const int d = (u & 511) - (v & 511);
    if (u & (1 << 9)) {  // S or N: a vertical edge, displaced along x
      xlo = min(xlo, d);
      xhi = max(xhi, d);
    } else {
      ylo = min(ylo, d);
      yhi = max(yhi, d);
    }
  }
  return true;
}

// Largest |d - s| over the same corresponding edges at shift (sy, sx); false
// when the polygons have no edge correspondence.
__device__ bool contour_residual(const ClipsDev& cs, int m, int r, int p, int q, int sy, int sx, int& res) {
  int xlo = 1 << 20, xhi = -(1 << 20), ylo = 1 << 20, yhi = -(1 << 20);
  if (!contour_pair(cs, m, r, p, q, xlo, xhi, ylo, yhi)) return false;
  res = max(max(xhi - sx, sx - xlo), max(yhi - sy, sy - ylo));
  return true;
}

// LDS path: any polygon count up to the cap, relation masks in LDS.  CONTOUR:
// the Min-Max runs over the full boundary edges of the matched polygons.
template <bool CONTOUR>
__device__ void edge_pair_lds(const ClipsDev& cs, const PairIO& io, Threshold thr, int64_t k,
                              unsigned long long* relM, unsigned long long* relR, unsigned long long* relM0,
                              unsigned long long* relR0, int* sflag_p, int (*red)[64]) {
  int& sflag = *sflag_p;
  const int lane = threadIdx.x;
  const int j = io.rep[k], i = io.mem[k];
  const int N = cs.N[i];
  if (lane == 0) { io.bits[k] = 0; io.flags[k] = 0; }
  for (int d = 0; d < 2; ++d) {
    const int m = d == 0 ? i : j, r = d == 0 ? j : i;
    const int w = cs.w[m];
    const int Pm = cs.npoly[m], Pr = cs.npoly[r];
    __syncthreads();
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
    bool same = true;
    if (lane < P) {
      int p, qq;
      if (from_member) { p = lane; qq = __ffsll((unsigned long long)relM0[lane]) - 1; }
      else { qq = lane; p = __ffsll((unsigned long long)relR0[lane]) - 1; }
      if constexpr (CONTOUR) {
        same = contour_pair(cs, m, r, p, qq, xlo, xhi, ylo, yhi);
      } else {
        const int16_t* a = bm + 4 * p;
        const int16_t* b = br + 4 * qq;
        const int d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2], d3 = a[3] - b[3];
        xlo = min(d0, d1); xhi = max(d0, d1);
        ylo = min(d2, d3); yhi = max(d2, d3);
      }
    }
    if (CONTOUR && __ballot(!same)) {  // wave-uniform: no edge correspondence
      if (lane == 0) {
        write_direction(io, k, d, s0y, s0x, -1, 0.0, false);
        io.flags[k] |= nomatch;
      }
      __syncthreads();
      continue;
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

// ---------------------------------------------------------------------------
// Register path for polygon counts <= 8 on both sides: the relation is one
// 64-bit word (bit 8 p + q: member polygon p overlaps rep polygon q), built by
// each lane over its rows and OR-reduced across the wave with shuffles; no LDS
// and no barriers.  Larger counts take the LDS path above.

__device__ __forceinline__ unsigned long long wave_or64(unsigned long long x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x |= __shfl_xor(x, off);
  return x;
}

// Exactly-one rule on an 8 x 8 relation word (uniform).
__device__ __forceinline__ bool corr8_ok(unsigned long long rel, int Pm, int Pr) {
  if (Pm <= Pr)
    for (int p = 0; p < Pm; ++p)
      if (__popcll((rel >> (8 * p)) & 0xffull) != 1) return false;
  if (Pr <= Pm)
    for (int q = 0; q < Pr; ++q)
      if (__popcll(rel & (0x0101010101010101ull << q)) != 1) return false;
  return true;
}

// 64 bits of a bit row starting at bit `start`, zero outside [0, N) (linear shift).
__device__ __forceinline__ uint64_t row_bits_linear(const uint64_t* row, int wpr, int start) {
  const int N = wpr * 64;
  if (start <= -64 || start >= N) return 0ull;
  if (start < 0) return row[0] << (-start);
  const int ws = start >> 6, o = start & 63;
  const uint64_t lo = row[ws];
  if (o == 0) return lo;
  const uint64_t hi = (ws + 1 < wpr) ? row[ws + 1] : 0ull;
  return (lo >> o) | (hi << (64 - o));
}

// Does a member shifted by (dy, dx) overlap a representative (linear shift)?
// Wave-wide; rs_* are row sums and b_* bit rasters.  Rows are first tried with
// a pigeonhole bound on the row sums: r_rep[y] + r_mem[y + dy] > N + |dx|
// forces a common pixel; only if no row proves it are the bit rows intersected.
__device__ bool overlap11(const uint16_t* rs_m, const uint16_t* rs_r, const uint64_t* b_m, const uint64_t* b_r,
                          int N, int dy, int dx, int lane) {
  const int y0 = max(0, -dy), y1 = min(N, N - dy);
  if (y0 >= y1 || dx >= N || dx <= -N) return false;
  const int lim = N + abs(dx);
  bool hit = false;
  for (int y = y0 + lane; y < y1; y += 64) hit |= (int)rs_r[y] + (int)rs_m[y + dy] > lim;
  if (__ballot(hit)) return true;
  const int wpr = N >> 6;
  for (int y = y0 + lane; y < y1; y += 64) {
    const uint64_t* rr = b_r + y * wpr;
    const uint64_t* mr = b_m + (y + dy) * wpr;
    for (int k = 0; k < wpr; ++k) hit |= (rr[k] & row_bits_linear(mr, wpr, 64 * k + dx)) != 0ull;
  }
  return __ballot(hit) != 0ull;
}

// One row of the same test, on one lane: row y of the representative against
// row y + dy of the member shifted by dx (pigeonhole bound, then bit rows).
__device__ __forceinline__ bool overlap_row(const uint16_t* rs_m, const uint16_t* rs_r, const uint64_t* b_m,
                                            const uint64_t* b_r, int N, int dy, int dx, int y) {
  if ((int)rs_r[y] + (int)rs_m[y + dy] > N + abs(dx)) return true;
  const int wpr = N >> 6;
  const uint64_t* rr = b_r + y * wpr;
  const uint64_t* mr = b_m + (y + dy) * wpr;
  bool hit = false;
  for (int k = 0; k < wpr; ++k) hit |= (rr[k] & row_bits_linear(mr, wpr, 64 * k + dx)) != 0ull;
  return hit;
}

// Quick per-lane proof of overlap from the middle row of the rows the shift
// keeps (for two single polygons whose boxes are centred on each other at T0
// it almost always overlaps); false means "not proven", not "no overlap".
__device__ __forceinline__ bool overlap11_quick(const uint16_t* rs_m, const uint16_t* rs_r, const uint64_t* b_m,
                                                const uint64_t* b_r, int N, int dy, int dx) {
  const int y0 = max(0, -dy), y1 = min(N, N - dy);
  if (y0 >= y1 || dx >= N || dx <= -N) return false;
  return overlap_row(rs_m, rs_r, b_m, b_r, N, dy, dx, (y0 + y1) >> 1);
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Relation of a member (row pointers rp_m, runs ru_m) shifted by (dy, dx)
// against a representative (rp_r, ru_r): bit 8 p + q when member polygon p
// overlaps rep polygon q (linear shift, zero fill).  Wave-wide, uniform result.
__device__ unsigned long long relation_runs(const uint16_t* rp_m, const uint32_t* ru_m, const uint16_t* rp_r,
                                            const uint32_t* ru_r, int N, int dy, int dx, int lane) {
  const int y0 = max(0, -dy), y1 = min(N, N - dy);
  unsigned long long rel = 0ull;
  // two rows of the lane at a time: their row pointers, then their first
  // runs, are loaded together, so a row costs no round trip of its own unless
  // it holds more than one run on a side
  for (int yb = y0 + lane; yb < y1; yb += 128) {
    int a[2], ae[2], b[2], be[2];
    uint32_t ra[2], rb[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int y = yb + 64 * k;
      const bool in = y < y1;
      a[k] = in ? rp_r[y] : 0;
      ae[k] = in ? rp_r[y + 1] : 0;
      b[k] = in ? rp_m[y + dy] : 0;
      be[k] = in ? rp_m[y + dy + 1] : 0;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      ra[k] = a[k] < ae[k] ? ru_r[a[k]] : 0u;
      rb[k] = b[k] < be[k] ? ru_m[b[k]] : 0u;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      int ia = a[k], ib = b[k];
      uint32_t va = ra[k], vb = rb[k];
      while (ia < ae[k] && ib < be[k]) {
        const int a0 = va & 511, a1 = (va >> 9) & 511, qa = (va >> 18) & 63;
        const int b0 = (int)(vb & 511) - dx, b1 = (int)((vb >> 9) & 511) - dx, pb = (vb >> 18) & 63;
        if (max(a0, b0) < min(a1, b1)) rel |= 1ull << (8 * pb + qa);
        if (a1 < b1) {
          if (++ia < ae[k]) va = ru_r[ia];
        } else {
          if (++ib < be[k]) vb = ru_m[ib];
        }
      }
    }
  }
  return wave_or64(rel);
}

// Min-Max shift and residual of the correspondence in rel (member polygons
// p, rep polygons q, from the fewer side), over the polygon boxes.
__device__ void matched_shift(unsigned long long rel, int Pm, int Pr, const int16_t* bm, const int16_t* br, int w,
                              int& sy, int& sx, int& E) {
  int xlo = 1 << 20, xhi = -(1 << 20), ylo = 1 << 20, yhi = -(1 << 20);
  const bool from_member = Pm <= Pr;
  const int P = from_member ? Pm : Pr;
  for (int t = 0; t < P; ++t) {
    int p, q;
    if (from_member) { p = t; q = __ffsll((unsigned long long)((rel >> (8 * t)) & 0xffull)) - 1; }
    else {
      q = t;
      const unsigned long long col = rel & (0x0101010101010101ull << t);
      p = (__ffsll(col) - 1) >> 3;
    }
    const int16_t* a = bm + 4 * p;
    const int16_t* b = br + 4 * q;
    const int d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2], d3 = a[3] - b[3];
    xlo = min(xlo, min(d0, d1)); xhi = max(xhi, max(d0, d1));
    ylo = min(ylo, min(d2, d3)); yhi = max(yhi, max(d2, d3));
  }
  int ex, ey;
  minmax_axis(xlo, xhi, w, sx, ex);
  minmax_axis(ylo, yhi, w, sy, ey);
  E = max(ex, ey);
}

// The relation at the solved shift keeps the matching of the fewer side(s).
__device__ __forceinline__ bool same_matching(unsigned long long rel1, unsigned long long rel0, int Pm, int Pr) {
  bool same = corr8_ok(rel1, Pm, Pr);
  if (Pm <= Pr)
    for (int p = 0; p < Pm; ++p) same = same && (((rel1 ^ rel0) >> (8 * p)) & 0xffull) == 0;
  if (Pr <= Pm)
    for (int q = 0; q < Pr; ++q) same = same && ((rel1 ^ rel0) & (0x0101010101010101ull << q)) == 0;
  return same;
}

constexpr int EDGE_PAIRS_PER_GROUP = 64;  // pairs per wave: one per lane

// Pairs are held one per lane: shifts, residuals, correspondences and outputs
// are per-lane arithmetic over 64 pairs at once, and the wave shares only the
// pixel work of each pair (the single-polygon overlap test, the polygon
// relation), whose answers return to the pair's lane.  Clips with more than 8
// polygons take the LDS path, one pair at a time.
__global__ void __launch_bounds__(64, 8) edge_batch_kernel(ClipsDev cs, PairIO io, Threshold thr, int64_t block0) {
  __shared__ unsigned long long relM[MAX_POLY], relR[MAX_POLY];
  __shared__ unsigned long long relM0[MAX_POLY], relR0[MAX_POLY];
  __shared__ int sflag;
  __shared__ int red[4][64];
  const int lane = threadIdx.x;
  const int64_t k0 = (block0 + (int64_t)blockIdx.x) * EDGE_PAIRS_PER_GROUP;
  const int cnt = (int)min((int64_t)EDGE_PAIRS_PER_GROUP, io.n_pairs - k0);
  const int64_t k = k0 + lane;

  int i = 0, j = 0, N = 0, Pi = 0, Pj = 0, wi = 0, wj = 0;
  bool big = false, empty = false, single = false, multi = false, mirror = true;
  int T0y[2] = {0, 0}, T0x[2] = {0, 0}, E0[2] = {0, 0};
  if (lane < cnt) {
    i = io.mem[k];
    j = io.rep[k];
    Pi = cs.npoly[i];
    Pj = cs.npoly[j];
    big = Pi > 8 || Pj > 8 || Pi < 0 || Pj < 0;
    empty = !big && (Pi == 0 || Pj == 0);
    single = !big && Pi == 1 && Pj == 1;
    multi = !big && !empty && !single;
    if (single || multi) {
      N = cs.N[i];
      wi = cs.w[i];
      wj = cs.w[j];
      mirror = wi == wj;
      const int16_t* gi = cs.gbox + 4 * i;
      const int16_t* gj = cs.gbox + 4 * j;
      const int dx0 = gi[0] - gj[0], dx1 = gi[1] - gj[1], dy0 = gi[2] - gj[2], dy1 = gi[3] - gj[3];
      int ex, ey;
      // T0 of member i against rep j, then of member j against rep i
      minmax_axis(min(dx0, dx1), max(dx0, dx1), wi, T0x[0], ex);
      minmax_axis(min(dy0, dy1), max(dy0, dy1), wi, T0y[0], ey);
      E0[0] = max(ex, ey);
      minmax_axis(min(-dx0, -dx1), max(-dx0, -dx1), wj, T0x[1], ex);
      minmax_axis(min(-dy0, -dy1), max(-dy0, -dy1), wj, T0y[1], ey);
      E0[1] = max(ex, ey);
    }
  }
  int sy[2] = {0, 0}, sx[2] = {0, 0}, E[2] = {-1, -1};
  bool matched[2] = {false, false}, ok[2] = {false, false};

  // single-polygon pairs: one overlap test decides the correspondence and its
  // re-check (each polygon's box is the global box, so the shift stays T0)
  {
    int64_t a_rs_i = 0, a_rs_j = 0, a_b_i = 0, a_b_j = 0;
    if (single) {
      a_rs_i = (int64_t)(cs.rowsum + cs.sig_off[i]);
      a_rs_j = (int64_t)(cs.rowsum + cs.sig_off[j]);
      a_b_i = (int64_t)(cs.bits + cs.bits_off[i]);
      a_b_j = (int64_t)(cs.bits + cs.bits_off[j]);
    }
    // each lane first tries its own pair's middle row; the wave-wide test of
    // all rows runs only for the directions that row does not settle
    bool q0 = false, q1 = false;
    if (single) {
      const uint16_t* rs_i = (const uint16_t*)a_rs_i;
      const uint16_t* rs_j = (const uint16_t*)a_rs_j;
      const uint64_t* b_i = (const uint64_t*)a_b_i;
      const uint64_t* b_j = (const uint64_t*)a_b_j;
      q0 = overlap11_quick(rs_i, rs_j, b_i, b_j, N, T0y[0], T0x[0]);
      if (!mirror) q1 = overlap11_quick(rs_j, rs_i, b_j, b_i, N, T0y[1], T0x[1]);
    }
    unsigned long long hit0 = __ballot(q0), hit1 = __ballot(q1);
    for (unsigned long long m = __ballot(single && !q0); m; m &= m - 1ull) {
      const int t = __ffsll(m) - 1;
      const uint16_t* rs_i = (const uint16_t*)readlane64(a_rs_i, t);
      const uint16_t* rs_j = (const uint16_t*)readlane64(a_rs_j, t);
      const uint64_t* b_i = (const uint64_t*)readlane64(a_b_i, t);
      const uint64_t* b_j = (const uint64_t*)readlane64(a_b_j, t);
      if (overlap11(rs_i, rs_j, b_i, b_j, __builtin_amdgcn_readlane(N, t), __builtin_amdgcn_readlane(T0y[0], t),
                    __builtin_amdgcn_readlane(T0x[0], t), lane))
        hit0 |= 1ull << t;
    }
    for (unsigned long long m = __ballot(single && !mirror && !q1); m; m &= m - 1ull) {
      const int t = __ffsll(m) - 1;
      const uint16_t* rs_i = (const uint16_t*)readlane64(a_rs_i, t);
      const uint16_t* rs_j = (const uint16_t*)readlane64(a_rs_j, t);
      const uint64_t* b_i = (const uint64_t*)readlane64(a_b_i, t);
      const uint64_t* b_j = (const uint64_t*)readlane64(a_b_j, t);
      if (overlap11(rs_j, rs_i, b_j, b_i, __builtin_amdgcn_readlane(N, t), __builtin_amdgcn_readlane(T0y[1], t),
                    __builtin_amdgcn_readlane(T0x[1], t), lane))
        hit1 |= 1ull << t;
    }
    if (single) {
      matched[0] = ok[0] = (hit0 >> lane) & 1ull;
      matched[1] = ok[1] = (hit1 >> lane) & 1ull;
      for (int d = 0; d < 2; ++d) {
        sy[d] = T0y[d];
        sx[d] = T0x[d];
        E[d] = matched[d] ? E0[d] : -1;
      }
    }
  }

  // pairs with 2..8 polygons on a side: relation at T0, per-lane matching and
  // Min-Max shift, relation at the shift, per-lane re-check
  {
    int64_t a_rp_i = 0, a_rp_j = 0, a_ru_i = 0, a_ru_j = 0;
    if (multi) {
      a_rp_i = (int64_t)(cs.run_rowptr + cs.rowptr_off[i]);
      a_rp_j = (int64_t)(cs.run_rowptr + cs.rowptr_off[j]);
      a_ru_i = (int64_t)(cs.runs + cs.run_off[i]);
      a_ru_j = (int64_t)(cs.runs + cs.run_off[j]);
    }
    unsigned long long rel0[2] = {0ull, 0ull}, rel1[2] = {0ull, 0ull};
    auto relation_of = [&](int t, int d, int dy, int dx) {
      const uint16_t* rp_i = (const uint16_t*)readlane64(a_rp_i, t);
      const uint16_t* rp_j = (const uint16_t*)readlane64(a_rp_j, t);
      const uint32_t* ru_i = (const uint32_t*)readlane64(a_ru_i, t);
      const uint32_t* ru_j = (const uint32_t*)readlane64(a_ru_j, t);
      const int Nt = __builtin_amdgcn_readlane(N, t);
      return d == 0 ? relation_runs(rp_i, ru_i, rp_j, ru_j, Nt, dy, dx, lane)
                    : relation_runs(rp_j, ru_j, rp_i, ru_i, Nt, dy, dx, lane);
    };
    const unsigned long long mm = __ballot(multi);
    for (unsigned long long m = mm; m; m &= m - 1ull) {
      const int t = __ffsll(m) - 1;
      const int nd = __builtin_amdgcn_readlane((int)mirror, t) ? 1 : 2;
#pragma unroll
      for (int d = 0; d < 2; ++d) {  // unrolled, so rel0 stays in registers
        if (d < nd) {
          const unsigned long long r =
              relation_of(t, d, __builtin_amdgcn_readlane(T0y[d], t), __builtin_amdgcn_readlane(T0x[d], t));
          if (lane == t) rel0[d] = r;
        }
      }
    }
    if (multi) {
      for (int d = 0; d < 2; ++d) {
        const int Pm = d == 0 ? Pi : Pj, Pr = d == 0 ? Pj : Pi;
        matched[d] = corr8_ok(rel0[d], Pm, Pr);
        sy[d] = T0y[d];
        sx[d] = T0x[d];
        E[d] = -1;
        if (matched[d]) {
          const int mc = d == 0 ? i : j, rc = d == 0 ? j : i;
          matched_shift(rel0[d], Pm, Pr, cs.boxes + (int64_t)mc * MAX_POLY * 4, cs.boxes + (int64_t)rc * MAX_POLY * 4,
                        d == 0 ? wi : wj, sy[d], sx[d], E[d]);
        }
      }
    }
    for (unsigned long long m = __ballot(multi && matched[0]); m; m &= m - 1ull) {
      const int t = __ffsll(m) - 1;
      const unsigned long long r =
          relation_of(t, 0, __builtin_amdgcn_readlane(sy[0], t), __builtin_amdgcn_readlane(sx[0], t));
      if (lane == t) rel1[0] = r;
    }
    for (unsigned long long m = __ballot(multi && !mirror && matched[1]); m; m &= m - 1ull) {
      const int t = __ffsll(m) - 1;
      const unsigned long long r =
          relation_of(t, 1, __builtin_amdgcn_readlane(sy[1], t), __builtin_amdgcn_readlane(sx[1], t));
      if (lane == t) rel1[1] = r;
    }
    if (multi)
      for (int d = 0; d < 2; ++d)
        ok[d] = matched[d] && same_matching(rel1[d], rel0[d], d == 0 ? Pi : Pj, d == 0 ? Pj : Pi);
  }

  if (single || multi || empty) {
    uint32_t fl = empty ? (uint32_t)CA_FLAG_EMPTY : 0u;
    if (mirror && !empty) {  // equal windows: the reverse direction is the exact mirror
      sy[1] = -sy[0]; sx[1] = -sx[0]; E[1] = E[0]; matched[1] = matched[0]; ok[1] = ok[0];
    }
    uint8_t bits = 0;
    for (int d = 0; d < 2; ++d) {
      io.shift[k * 4 + 2 * d] = (int16_t)sy[d];
      io.shift[k * 4 + 2 * d + 1] = (int16_t)sx[d];
      io.count[k * 2 + d] = E[d];
      io.score[k * 2 + d] = 0.0;
      if (!matched[d]) fl |= d == 0 ? CA_FLAG_NO_MATCH_FWD : CA_FLAG_NO_MATCH_REV;
      else if (!ok[d]) fl |= d == 0 ? CA_FLAG_RECHECK_FWD : CA_FLAG_RECHECK_REV;
      if (ok[d] && (int64_t)E[d] <= thr.p) bits |= (uint8_t)(1u << d);
    }
    io.bits[k] = bits;
    io.flags[k] = fl;
  }

  // clips with more than 8 polygons, one pair at a time on the LDS path
  for (unsigned long long m = __ballot(big); m; m &= m - 1ull)
    edge_pair_lds<false>(cs, io, thr, k0 + (__ffsll(m) - 1), relM, relR, relM0, relR0, &sflag, red);
}

// ---------------------------------------------------------------------------
// Edge track over full boundary edges (CA_EDGES_CONTOUR).  The correspondence
// at T0, the exactly-one rule and the re-check at the solved shift are those
// of the box track; the Min-Max solve runs over every edge of the matched
// polygons (contour_pair: edge k against edge k of the canonical lists, no
// correspondence when the code sequences differ).  One pair per lane for
// clips of up to 8 polygons (the wave shares each pair's relation sweep), the
// LDS path one pair at a time above that.

// Min-Max shift and residual over the contour edges of the correspondence in
// the 8 x 8 relation word rel; false when a matched pair has no edge
// correspondence.
__device__ bool contour_matched_shift(const ClipsDev& cs, int m, int r, unsigned long long rel, int Pm, int Pr, int w,
                                      int& sy, int& sx, int& E) {
  int xlo = 1 << 20, xhi = -(1 << 20), ylo = 1 << 20, yhi = -(1 << 20);
  const bool from_member = Pm <= Pr;
  const int P = from_member ? Pm : Pr;
  for (int t = 0; t < P; ++t) {
    int p, q;
    if (from_member) { p = t; q = __ffsll((unsigned long long)((rel >> (8 * t)) & 0xffull)) - 1; }
    else {
      q = t;
      const unsigned long long col = rel & (0x0101010101010101ull << t);
      p = (__ffsll(col) - 1) >> 3;
    }
    if (!contour_pair(cs, m, r, p, q, xlo, xhi, ylo, yhi)) return false;
  }
  int ex, ey;
  minmax_axis(xlo, xhi, w, sx, ex);
  minmax_axis(ylo, yhi, w, sy, ey);
  E = max(ex, ey);
  return true;
}

__global__ void __launch_bounds__(64) edge_contour_kernel(ClipsDev cs, PairIO io, Threshold thr, int64_t block0) {
  __shared__ unsigned long long relM[MAX_POLY], relR[MAX_POLY];
  __shared__ unsigned long long relM0[MAX_POLY], relR0[MAX_POLY];
  __shared__ int sflag;
  __shared__ int red[4][64];
  const int lane = threadIdx.x;
  const int64_t k0 = (block0 + (int64_t)blockIdx.x) * EDGE_PAIRS_PER_GROUP;
  const int cnt = (int)min((int64_t)EDGE_PAIRS_PER_GROUP, io.n_pairs - k0);
  const int64_t k = k0 + lane;

  int i = 0, j = 0, N = 0, Pi = 0, Pj = 0, wi = 0, wj = 0;
  bool none = false, empty = false, small = false, big = false, mirror = true;
  int T0y[2] = {0, 0}, T0x[2] = {0, 0};
  if (lane < cnt) {
    i = io.mem[k];
    j = io.rep[k];
    Pi = cs.npoly[i];
    Pj = cs.npoly[j];
    empty = Pi == 0 || Pj == 0;
    none = empty || Pi < 0 || Pj < 0 || cs.cstat[i] < 0 || cs.cstat[j] < 0;
    small = !none && Pi <= 8 && Pj <= 8;
    big = !none && !small;
    if (small) {
      N = cs.N[i];
      wi = cs.w[i];
      wj = cs.w[j];
      mirror = wi == wj;
      const int16_t* gi = cs.gbox + 4 * i;
      const int16_t* gj = cs.gbox + 4 * j;
      const int dx0 = gi[0] - gj[0], dx1 = gi[1] - gj[1], dy0 = gi[2] - gj[2], dy1 = gi[3] - gj[3];
      int e_unused;
      minmax_axis(min(dx0, dx1), max(dx0, dx1), wi, T0x[0], e_unused);
      minmax_axis(min(dy0, dy1), max(dy0, dy1), wi, T0y[0], e_unused);
      minmax_axis(min(-dx0, -dx1), max(-dx0, -dx1), wj, T0x[1], e_unused);
      minmax_axis(min(-dy0, -dy1), max(-dy0, -dy1), wj, T0y[1], e_unused);
    }
  }
  int sy[2] = {0, 0}, sx[2] = {0, 0}, E[2] = {-1, -1};
  bool matched[2] = {false, false}, ok[2] = {false, false};
  {
    int64_t a_rp_i = 0, a_rp_j = 0, a_ru_i = 0, a_ru_j = 0;
    if (small) {
      a_rp_i = (int64_t)(cs.run_rowptr + cs.rowptr_off[i]);
      a_rp_j = (int64_t)(cs.run_rowptr + cs.rowptr_off[j]);
      a_ru_i = (int64_t)(cs.runs + cs.run_off[i]);
      a_ru_j = (int64_t)(cs.runs + cs.run_off[j]);
    }
    unsigned long long rel0[2] = {0ull, 0ull}, rel1[2] = {0ull, 0ull};
    auto relation_of = [&](int t, int d, int dy, int dx) {
      const uint16_t* rp_i = (const uint16_t*)readlane64(a_rp_i, t);
      const uint16_t* rp_j = (const uint16_t*)readlane64(a_rp_j, t);
      const uint32_t* ru_i = (const uint32_t*)readlane64(a_ru_i, t);
      const uint32_t* ru_j = (const uint32_t*)readlane64(a_ru_j, t);
      const int Nt = __builtin_amdgcn_readlane(N, t);
      return d == 0 ? relation_runs(rp_i, ru_i, rp_j, ru_j, Nt, dy, dx, lane)
                    : relation_runs(rp_j, ru_j, rp_i, ru_i, Nt, dy, dx, lane);
    };
    for (unsigned long long m = __ballot(small); m; m &= m - 1ull) {
      const int t = __ffsll(m) - 1;
      const int nd = __builtin_amdgcn_readlane((int)mirror, t) ? 1 : 2;
      for (int d = 0; d < nd; ++d) {
        const unsigned long long r =
            relation_of(t, d, __builtin_amdgcn_readlane(T0y[d], t), __builtin_amdgcn_readlane(T0x[d], t));
        if (lane == t) rel0[d] = r;
      }
    }
    if (small) {
      for (int d = 0; d < (mirror ? 1 : 2); ++d) {
        const int Pm = d == 0 ? Pi : Pj, Pr = d == 0 ? Pj : Pi;
        sy[d] = T0y[d];
        sx[d] = T0x[d];
        matched[d] = corr8_ok(rel0[d], Pm, Pr) &&
                     contour_matched_shift(cs, d == 0 ? i : j, d == 0 ? j : i, rel0[d], Pm, Pr, d == 0 ? wi : wj,
                                           sy[d], sx[d], E[d]);
        if (!matched[d]) {
          sy[d] = T0y[d];
          sx[d] = T0x[d];
          E[d] = -1;
        }
      }
    }
    for (unsigned long long m = __ballot(small && matched[0]); m; m &= m - 1ull) {
      const int t = __ffsll(m) - 1;
      const unsigned long long r =
          relation_of(t, 0, __builtin_amdgcn_readlane(sy[0], t), __builtin_amdgcn_readlane(sx[0], t));
      if (lane == t) rel1[0] = r;
    }
    for (unsigned long long m = __ballot(small && !mirror && matched[1]); m; m &= m - 1ull) {
      const int t = __ffsll(m) - 1;
      const unsigned long long r =
          relation_of(t, 1, __builtin_amdgcn_readlane(sy[1], t), __builtin_amdgcn_readlane(sx[1], t));
      if (lane == t) rel1[1] = r;
    }
    if (small)
      for (int d = 0; d < (mirror ? 1 : 2); ++d)
        ok[d] = matched[d] && same_matching(rel1[d], rel0[d], d == 0 ? Pi : Pj, d == 0 ? Pj : Pi);
  }

  if (small || none) {
    uint32_t fl = empty ? (uint32_t)CA_FLAG_EMPTY : 0u;
    if (mirror && small) {  // equal windows: the reverse direction is the exact mirror
      sy[1] = -sy[0]; sx[1] = -sx[0]; E[1] = E[0]; matched[1] = matched[0]; ok[1] = ok[0];
    }
    uint8_t bits = 0;
    for (int d = 0; d < 2; ++d) {
      io.shift[k * 4 + 2 * d] = (int16_t)sy[d];
      io.shift[k * 4 + 2 * d + 1] = (int16_t)sx[d];
      io.count[k * 2 + d] = E[d];
      io.score[k * 2 + d] = 0.0;
      if (!matched[d]) fl |= d == 0 ? CA_FLAG_NO_MATCH_FWD : CA_FLAG_NO_MATCH_REV;
      else if (!ok[d]) fl |= d == 0 ? CA_FLAG_RECHECK_FWD : CA_FLAG_RECHECK_REV;
      if (ok[d] && (int64_t)E[d] <= thr.p) bits |= (uint8_t)(1u << d);
    }
    io.bits[k] = bits;
    io.flags[k] = fl;
  }

  for (unsigned long long m = __ballot(big); m; m &= m - 1ull)
    edge_pair_lds<true>(cs, io, thr, k0 + (__ffsll(m) - 1), relM, relR, relM0, relR0, &sflag, red);
}

}  // namespace ca

namespace ca {

// Center verification (edge track, Sec. 2.2.2 at the member's center): the
// shift lies in the member's window, the fewer side's polygons (both sides if
// the counts are equal) each overlap exactly one polygon of the other clip at
// the shift, and over the matched bounding-box edges the residual
// max |d - s| per axis is at most T.  One wave per member.
template <bool CONTOUR>
__global__ void __launch_bounds__(64) edge_verify_kernel(ClipsDev cs, int64_t n, int64_t t0, const int32_t* mem,
                                                         const int32_t* rep, const int16_t* shift, Threshold thr,
                                                         unsigned long long* viol, unsigned long long* first) {
  __shared__ unsigned long long relM[MAX_POLY], relR[MAX_POLY];
  __shared__ int sflag;
  __shared__ int red[4][64];
  const int lane = threadIdx.x;
  const int64_t t = t0 + blockIdx.x;
  if (t >= n) return;  // block-uniform
  const int m = mem[t], r = rep[t];
  const int N = cs.N[m];
  const int sy = shift[2 * t], sx = shift[2 * t + 1];
  const int w = cs.w[m];
  const int Pm = cs.npoly[m], Pr = cs.npoly[r];
  bool ok = cs.N[r] == N && sy >= -w && sy <= w && sx >= -w && sx <= w && Pm > 0 && Pr > 0;
  if (ok) {
    overlap_relation(cs, m, r, N, sy, sx, relM, relR);
    ok = correspondence_ok(relM, relR, Pm, Pr, &sflag);
  }
  if (ok) {
    const int16_t* bm = cs.boxes + (int64_t)m * MAX_POLY * 4;
    const int16_t* br = cs.boxes + (int64_t)r * MAX_POLY * 4;
    const bool from_member = Pm <= Pr;
    const int P = from_member ? Pm : Pr;
    int ex = 0, ey = 0;  // residual of this lane's matched pair at the given shift
    if (lane < P) {
      int p, q;
      if (from_member) { p = lane; q = __ffsll((unsigned long long)relM[lane]) - 1; }
      else { q = lane; p = __ffsll((unsigned long long)relR[lane]) - 1; }
      if constexpr (CONTOUR) {
        // no edge correspondence: a residual above any threshold
        if (!contour_residual(cs, m, r, p, q, sy, sx, ex)) ex = 1 << 30;
      } else {
        const int16_t* a = bm + 4 * p;
        const int16_t* b = br + 4 * q;
        ex = max(abs(a[0] - b[0] - sx), abs(a[1] - b[1] - sx));
        ey = max(abs(a[2] - b[2] - sy), abs(a[3] - b[3] - sy));
      }
    }
    red[0][lane] = max(ex, ey);
    __syncthreads();
    for (int st = 32; st > 0; st >>= 1) {
      if (lane < st) red[0][lane] = max(red[0][lane], red[0][lane + st]);
      __syncthreads();
    }
    ok = (int64_t)red[0][0] <= thr.p;
  }
  if (!ok && lane == 0) {
    atomicAdd(viol, 1ull);
    atomicMin(first, (unsigned long long)t);
  }
}

hipError_t launch_verify_edge(const ClipsDev& cs, int64_t n, const int32_t* mem, const int32_t* rep,
                              const int16_t* shift, Threshold thr, unsigned long long* viol, unsigned long long* first,
                              hipStream_t s, bool contour) {
  for (int64_t t0 = 0; t0 < n; t0 += LAUNCH_CHUNK) {
    const int64_t nt = std::min<int64_t>(LAUNCH_CHUNK, n - t0);
    if (contour)
      hipLaunchKernelGGL(edge_verify_kernel<true>, dim3((unsigned)nt), dim3(64), 0, s, cs, n, t0, mem, rep, shift, thr,
                         viol, first);
    else
      hipLaunchKernelGGL(edge_verify_kernel<false>, dim3((unsigned)nt), dim3(64), 0, s, cs, n, t0, mem, rep, shift,
                         thr, viol, first);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// XY-separation alignment of the cosine track (paper Sec. 3.2.1(2)).
//
// Per direction (member m against representative r) the polygon
// correspondence of the edge track is taken at T0.  Every matched pair gives
// an x interval and a y interval: [min, max] of the displacements (member
// minus representative) of its two box edges on that axis.  Per axis the
// narrowest interval wins (ties: the first pair in (member polygon, rep
// polygon) order), and its midpoint, rounded half toward zero and clamped to
// the member's window, is the shift on that axis.  Without a correspondence
// (no polygon on a side, the exactly-one rule fails, more than 64 polygons)
// the pair of global boxes gives the shift, which is T0.  Shifts are then
// named as the cosine window names them (every residue in [-N/2, N/2 - 1]
// when 2 w + 1 > N).  xysep_count_kernel evaluates Eq. 2 at the shifts.

// A clamped shift named as the cosine window names it (N a power of two).
__device__ __forceinline__ int cos_residue(int s, int w, int N) {
  return (2 * w + 1 > N) ? ((s + N / 2) & (N - 1)) - N / 2 : s;
}

// 8 x 8 bit matrix transpose: bit 8 r + c -> bit 8 c + r.
__device__ __forceinline__ unsigned long long transpose8(unsigned long long x) {
  unsigned long long t;
  t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
  x = x ^ t ^ (t << 7);
  t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
  x = x ^ t ^ (t << 14);
  t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
  x = x ^ t ^ (t << 28);
  return x;
}

// Interval of one matched pair on one axis: the key orders pairs by width,
// then by (p, q); the smaller key wins.
__device__ __forceinline__ void xy_interval(int d0, int d1, int p, int q, int& key, int& lo, int& hi) {
  lo = min(d0, d1);
  hi = max(d0, d1);
  key = ((hi - lo) << 12) | (p << 6) | q;
}

// The shift from the winning intervals (x: [xlo, xhi], y: [ylo, yhi]).
__device__ __forceinline__ void xy_shift(int xlo, int xhi, int ylo, int yhi, int w, int N, int& sy, int& sx) {
  int e;
  minmax_axis(xlo, xhi, w, sx, e);
  minmax_axis(ylo, yhi, w, sy, e);
  sx = cos_residue(sx, w, N);
  sy = cos_residue(sy, w, N);
}

// Winning intervals over the correspondence in an 8 x 8 relation word
// (member polygons p, rep polygons q), on one lane.
__device__ void xy_select8(unsigned long long rel, int Pm, int Pr, const int16_t* bm, const int16_t* br, int w,
                           int N, int& sy, int& sx) {
  int kx = 1 << 30, xlo = 0, xhi = 0, ky = 1 << 30, ylo = 0, yhi = 0;
  const bool from_member = Pm <= Pr;
  const int P = from_member ? Pm : Pr;
  for (int t = 0; t < P; ++t) {
    int p, q;
    if (from_member) {
      p = t;
      q = __ffsll((unsigned long long)((rel >> (8 * t)) & 0xffull)) - 1;
    } else {
      q = t;
      p = (__ffsll(rel & (0x0101010101010101ull << t)) - 1) >> 3;
    }
    const int16_t* a = bm + 4 * p;
    const int16_t* b = br + 4 * q;
    int k, lo, hi;
    xy_interval(a[0] - b[0], a[1] - b[1], p, q, k, lo, hi);
    if (k < kx) { kx = k; xlo = lo; xhi = hi; }
    xy_interval(a[2] - b[2], a[3] - b[3], p, q, k, lo, hi);
    if (k < ky) { ky = k; ylo = lo; yhi = hi; }
  }
  xy_shift(xlo, xhi, ylo, yhi, w, N, sy, sx);
}

// Clips with more than 8 polygons on a side (at most 64): one direction of
// one pair on the whole wave, relation masks in LDS.  Returns the shift in
// (sy, sx) on every lane.
__device__ void xy_pair_lds(const ClipsDev& cs, int m, int r, int N, int w, int t0y, int t0x,
                            unsigned long long* relM, unsigned long long* relR, int* sflag, int& sy, int& sx) {
  const int lane = threadIdx.x;
  const int Pm = cs.npoly[m], Pr = cs.npoly[r];
  overlap_relation(cs, m, r, N, t0y, t0x, relM, relR);
  if (!correspondence_ok(relM, relR, Pm, Pr, sflag)) {
    sy = cos_residue(t0y, w, N);
    sx = cos_residue(t0x, w, N);
    return;
  }
  const bool from_member = Pm <= Pr;
  const int P = from_member ? Pm : Pr;
  int kx = 1 << 30, ky = 1 << 30, xlo = 0, xhi = 0, ylo = 0, yhi = 0;
  if (lane < P) {
    int p, q;
    if (from_member) { p = lane; q = __ffsll((unsigned long long)relM[lane]) - 1; }
    else { q = lane; p = __ffsll((unsigned long long)relR[lane]) - 1; }
    const int16_t* a = cs.boxes + (int64_t)m * MAX_POLY * 4 + 4 * p;
    const int16_t* b = cs.boxes + (int64_t)r * MAX_POLY * 4 + 4 * q;
    xy_interval(a[0] - b[0], a[1] - b[1], p, q, kx, xlo, xhi);
    xy_interval(a[2] - b[2], a[3] - b[3], p, q, ky, ylo, yhi);
  }
  int mx = kx, my = ky;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mx = min(mx, __shfl_xor(mx, off));
    my = min(my, __shfl_xor(my, off));
  }
  // keys are distinct (they carry (p, q)), so exactly one lane holds each minimum
  const int lx = __ffsll(__ballot(kx == mx)) - 1, ly = __ffsll(__ballot(ky == my)) - 1;
  xy_shift(__shfl(xlo, lx), __shfl(xhi, lx), __shfl(ylo, ly), __shfl(yhi, ly), w, N, sy, sx);
}

// Shifts of both directions of 64 pairs per one-wave workgroup, one pair per
// lane; the wave shares the relation work of each multi-polygon pair.
// Writes io.shift and io.flags (CA_FLAG_EMPTY for an empty clip).
__global__ void __launch_bounds__(64) xysep_shift_kernel(ClipsDev cs, PairIO io, int64_t block0) {
  __shared__ unsigned long long relM[MAX_POLY], relR[MAX_POLY];
  __shared__ int sflag;
  const int lane = threadIdx.x;
  const int64_t k0 = (block0 + (int64_t)blockIdx.x) * EDGE_PAIRS_PER_GROUP;
  const int cnt = (int)min((int64_t)EDGE_PAIRS_PER_GROUP, io.n_pairs - k0);
  const int64_t k = k0 + lane;

  int i = 0, j = 0, N = 0, Pi = 0, Pj = 0, wi = 0, wj = 0;
  bool big = false, empty = false, multi = false, mirror = true;
  int sy[2] = {0, 0}, sx[2] = {0, 0}, T0y[2] = {0, 0}, T0x[2] = {0, 0};
  if (lane < cnt) {
    i = io.mem[k];
    j = io.rep[k];
    N = cs.N[i];
    Pi = cs.npoly[i];
    Pj = cs.npoly[j];
    empty = Pi == 0 || Pj == 0;
    const bool capped = Pi < 0 || Pj < 0;
    big = !empty && !capped && (Pi > 8 || Pj > 8);
    multi = !empty && !capped && !big && !(Pi == 1 && Pj == 1);
    if (!empty) {
      wi = cs.w[i];
      wj = cs.w[j];
      mirror = wi == wj;
      const int16_t* gi = cs.gbox + 4 * i;
      const int16_t* gj = cs.gbox + 4 * j;
      const int dx0 = gi[0] - gj[0], dx1 = gi[1] - gj[1], dy0 = gi[2] - gj[2], dy1 = gi[3] - gj[3];
      int e;
      minmax_axis(min(dx0, dx1), max(dx0, dx1), wi, T0x[0], e);
      minmax_axis(min(dy0, dy1), max(dy0, dy1), wi, T0y[0], e);
      minmax_axis(min(-dx0, -dx1), max(-dx0, -dx1), wj, T0x[1], e);
      minmax_axis(min(-dy0, -dy1), max(-dy0, -dy1), wj, T0y[1], e);
      // single polygons, more than 64 polygons, or no correspondence: T0
      sy[0] = cos_residue(T0y[0], wi, N);
      sx[0] = cos_residue(T0x[0], wi, N);
      sy[1] = cos_residue(T0y[1], wj, N);
      sx[1] = cos_residue(T0x[1], wj, N);
    }
  }

  // 2..8 polygons a side: relation at T0 (wave-shared), then per lane
  {
    int64_t a_rp_i = 0, a_rp_j = 0, a_ru_i = 0, a_ru_j = 0;
    if (multi) {
      a_rp_i = (int64_t)(cs.run_rowptr + cs.rowptr_off[i]);
      a_rp_j = (int64_t)(cs.run_rowptr + cs.rowptr_off[j]);
      a_ru_i = (int64_t)(cs.runs + cs.run_off[i]);
      a_ru_j = (int64_t)(cs.runs + cs.run_off[j]);
    }
    unsigned long long rel0[2] = {0ull, 0ull};
    for (unsigned long long m = __ballot(multi); m; m &= m - 1ull) {
      const int t = __ffsll(m) - 1;
      const uint16_t* rp_i = (const uint16_t*)readlane64(a_rp_i, t);
      const uint16_t* rp_j = (const uint16_t*)readlane64(a_rp_j, t);
      const uint32_t* ru_i = (const uint32_t*)readlane64(a_ru_i, t);
      const uint32_t* ru_j = (const uint32_t*)readlane64(a_ru_j, t);
      const int Nt = __builtin_amdgcn_readlane(N, t);
      const unsigned long long r0 = relation_runs(rp_i, ru_i, rp_j, ru_j, Nt, __builtin_amdgcn_readlane(T0y[0], t),
                                                  __builtin_amdgcn_readlane(T0x[0], t), lane);
      // equal windows: T0 of the reverse direction is the mirror, and its
      // relation the transpose
      unsigned long long r1 = transpose8(r0);
      if (!__builtin_amdgcn_readlane((int)mirror, t))
        r1 = relation_runs(rp_j, ru_j, rp_i, ru_i, Nt, __builtin_amdgcn_readlane(T0y[1], t),
                           __builtin_amdgcn_readlane(T0x[1], t), lane);
      if (lane == t) {
        rel0[0] = r0;
        rel0[1] = r1;
      }
    }
    if (multi) {
      for (int d = 0; d < 2; ++d) {
        const int Pm = d == 0 ? Pi : Pj, Pr = d == 0 ? Pj : Pi;
        if (corr8_ok(rel0[d], Pm, Pr)) {
          const int mc = d == 0 ? i : j, rc = d == 0 ? j : i;
          xy_select8(rel0[d], Pm, Pr, cs.boxes + (int64_t)mc * MAX_POLY * 4, cs.boxes + (int64_t)rc * MAX_POLY * 4,
                     d == 0 ? wi : wj, N, sy[d], sx[d]);
        }
      }
    }
  }

  // more than 8 polygons on a side: one direction at a time on the LDS path
  for (unsigned long long m = __ballot(big); m; m &= m - 1ull) {
    const int t = __ffsll(m) - 1;
    const int ti = __builtin_amdgcn_readlane(i, t), tj = __builtin_amdgcn_readlane(j, t);
    const int Nt = __builtin_amdgcn_readlane(N, t);
    for (int d = 0; d < 2; ++d) {
      int y, x;
      xy_pair_lds(cs, d == 0 ? ti : tj, d == 0 ? tj : ti, Nt, __builtin_amdgcn_readlane(d == 0 ? wi : wj, t),
                  __builtin_amdgcn_readlane(T0y[d], t), __builtin_amdgcn_readlane(T0x[d], t), relM, relR, &sflag, y,
                  x);
      if (lane == t) {
        sy[d] = y;
        sx[d] = x;
      }
    }
  }

  if (lane < cnt) {
    for (int d = 0; d < 2; ++d) {
      io.shift[k * 4 + 2 * d] = (int16_t)sy[d];
      io.shift[k * 4 + 2 * d + 1] = (int16_t)sx[d];
    }
    io.flags[k] = empty ? (uint32_t)CA_FLAG_EMPTY : 0u;
  }
}

// Eq. 2 at the shifts of both directions: one wave per pair.
__global__ void __launch_bounds__(256) xysep_count_kernel(ClipsDev cs, PairIO io, Threshold thr, int64_t k0) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t k = k0 + (int64_t)blockIdx.x * 4 + wave;
  if (k >= io.n_pairs) return;
  const int i = io.mem[k], j = io.rep[k];
  const int N = cs.N[i];
  const int sy0 = io.shift[k * 4 + 0], sx0 = io.shift[k * 4 + 1];
  const int sy1 = io.shift[k * 4 + 2], sx1 = io.shift[k * 4 + 3];
  const uint64_t* bi = cs.bits + cs.bits_off[i];
  const uint64_t* bj = cs.bits + cs.bits_off[j];
  int c0 = 0, c1 = 0;
  for (int y = lane; y < N; y += 64) {
    c0 += row_overlap(bj, bi, N, y, sy0, sx0);  // member i against rep j
    c1 += row_overlap(bi, bj, N, y, sy1, sx1);  // member j against rep i
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    c0 += __shfl_xor(c0, off);
    c1 += __shfl_xor(c1, off);
  }
  if (lane == 0) {
    const int ni = cs.npix[i], nj = cs.npix[j];
    io.count[k * 2 + 0] = c0;
    io.count[k * 2 + 1] = c1;
    io.score[k * 2 + 0] = cosine_score(c0, ni, nj);
    io.score[k * 2 + 1] = cosine_score(c1, nj, ni);
    io.bits[k] = (uint8_t)((cosine_bit(c0, ni, nj, thr) ? 1u : 0u) | (cosine_bit(c1, nj, ni, thr) ? 2u : 0u));
  }
}

hipError_t launch_xysep(const ClipsDev& cs, const PairIO& io, Threshold thr, hipStream_t s) {
  if (io.n_pairs == 0) return hipSuccess;
  const int64_t groups = (io.n_pairs + EDGE_PAIRS_PER_GROUP - 1) / EDGE_PAIRS_PER_GROUP;
  for (int64_t b0 = 0; b0 < groups; b0 += LAUNCH_CHUNK) {
    const unsigned nb = (unsigned)std::min<int64_t>(LAUNCH_CHUNK, groups - b0);
    hipLaunchKernelGGL(xysep_shift_kernel, dim3(nb), dim3(64), 0, s, cs, io, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (int64_t k0 = 0; k0 < io.n_pairs; k0 += LAUNCH_CHUNK * 4) {
    const int64_t nk = std::min<int64_t>(LAUNCH_CHUNK * 4, io.n_pairs - k0);
    hipLaunchKernelGGL(xysep_count_kernel, dim3((unsigned)((nk + 3) / 4)), dim3(256), 0, s, cs, io, thr, k0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_edge_contour(const ClipsDev& cs, const PairIO& io, Threshold thr, hipStream_t s) {
  if (io.n_pairs == 0) return hipSuccess;
  if (!cs.cstat) return hipErrorInvalidValue;  // the kernel reads the contour tables
  const int64_t groups = (io.n_pairs + EDGE_PAIRS_PER_GROUP - 1) / EDGE_PAIRS_PER_GROUP;
  for (int64_t b0 = 0; b0 < groups; b0 += LAUNCH_CHUNK) {
    const unsigned nb = (unsigned)std::min<int64_t>(LAUNCH_CHUNK, groups - b0);
    hipLaunchKernelGGL(edge_contour_kernel, dim3(nb), dim3(64), 0, s, cs, io, thr, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_edge(const ClipsDev& cs, const PairIO& io, Threshold thr, hipStream_t s) {
  if (io.n_pairs == 0) return hipSuccess;
  const int64_t groups = (io.n_pairs + EDGE_PAIRS_PER_GROUP - 1) / EDGE_PAIRS_PER_GROUP;
  for (int64_t b0 = 0; b0 < groups; b0 += LAUNCH_CHUNK) {
    const unsigned nb = (unsigned)std::min<int64_t>(LAUNCH_CHUNK, groups - b0);
    hipLaunchKernelGGL(edge_batch_kernel, dim3(nb), dim3(64), 0, s, cs, io, thr, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ca
