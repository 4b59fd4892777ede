// Polygon contours for the edge track over full boundary edges (paper
// Sec. 2.2.2: the displacement of every pair of corresponding edges of
// matched polygons), and the per-polygon topological hash of the pre-screen
// (Sec. 3.1 stage 1).
//
// Boundary sides are directed with the polygon on their right in image
// coordinates (y down): top sides run east, right sides south, bottom sides
// west, left sides north.  A vertex is a corner of the (N+1) x (N+1) corner
// grid whose 2 x 2 pixel window is neither uniform nor a straight boundary;
// a window whose two set pixels are diagonal carries two passages, and a
// contour arriving there turns right (the two pixels stay apart, as
// 4-connectivity has them).  An edge runs from a vertex to the next vertex
// along its direction, so a contour is walked vertex to vertex.
//
// Per clip, one 64-lane workgroup:
//   count pass: vertex passages (= edges) over the clip, or -1 when the
//     clip has no contour data (the labeller kept no polygons, or more than
//     MAX_EDGES edges);
//   trace pass: raster and vertex rows in LDS.  One lane scans the vertex
//     rows in raster order and walks every contour from the first of its
//     vertices it meets (its raster-first vertex), marking visited passages;
//     then each lane takes one contour and finds the start of the least
//     rotation of its direction codes (two-pointer minimum-rotation scan),
//     and each lane takes one polygon and writes its contours (outer first,
//     holes in discovery order), edge words and FNV-1a hash.
#include "kernels.h"

namespace ca {
namespace {

constexpr int DIR_E = 0, DIR_S = 1, DIR_W = 2, DIR_N = 3;
constexpr int MAX_CONTOURS = MAX_EDGES / 4;  // a contour has at least four edges
constexpr uint64_t FNV_OFFSET = 0xcbf29ce484222325ull;
constexpr uint64_t FNV_PRIME = 0x100000001b3ull;

// Vertex and diagonal-window masks of corner row Y (corners X = 0..N, bit X
// of the N/64 + 1 words).  up, dn: pixel rows Y - 1 and Y (null: outside).
template <int N>
__device__ __forceinline__ void vertex_row(const uint64_t* up, const uint64_t* dn, uint64_t* vtx, uint64_t* sad) {
  constexpr int WPR = N / 64, CW = WPR + 1;
  uint64_t pu = 0, pd = 0;  // previous words (pixel X - 1 of bit 0)
#pragma unroll
  for (int w = 0; w < CW; ++w) {
    const uint64_t B = (up && w < WPR) ? up[w] : 0ull;  // pixel (Y - 1, X)
    const uint64_t D = (dn && w < WPR) ? dn[w] : 0ull;  // pixel (Y, X)
    const uint64_t A = (B << 1) | (pu >> 63);           // pixel (Y - 1, X - 1)
    const uint64_t C = (D << 1) | (pd >> 63);           // pixel (Y, X - 1)
    pu = B;
    pd = D;
    const uint64_t mask = w < WPR ? ~0ull : 1ull;       // corner X = N is bit 0 of the last word
    const uint64_t plain = (~(A ^ B) & ~(C ^ D)) | (~(A ^ C) & ~(B ^ D));
    vtx[w] = ~plain & mask;
    if (sad) sad[w] = ((A & D & ~B & ~C) | (B & C & ~A & ~D)) & mask;
  }
}

template <int N>
__device__ __forceinline__ int count_edges(const uint64_t* bits, int lane) {
  constexpr int WPR = N / 64, CW = WPR + 1;
  int cnt = 0;
  for (int Y = lane; Y <= N; Y += 64) {
    uint64_t v[CW], s[CW];
    vertex_row<N>(Y >= 1 ? bits + (Y - 1) * WPR : nullptr, Y < N ? bits + Y * WPR : nullptr, v, s);
#pragma unroll
    for (int w = 0; w < CW; ++w) cnt += __popcll(v[w]) + __popcll(s[w]);
  }
  return cnt;
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

__global__ void __launch_bounds__(64) contour_count_kernel(ClipsDev cs, int64_t block0, int32_t* __restrict__ out) {
  const int64_t i = block0 + (int64_t)blockIdx.x;
  if (i >= cs.n) return;  // block-uniform
  const int lane = threadIdx.x;
  const int N = cs.N[i];
  if (cs.npoly[i] < 0) {
    if (lane == 0) out[i] = -1;
    return;
  }
  const uint64_t* bits = cs.bits + cs.bits_off[i];
  int cnt = 0;
  if (N == 64) cnt = count_edges<64>(bits, lane);
  else if (N == 128) cnt = count_edges<128>(bits, lane);
  else cnt = count_edges<256>(bits, lane);
  cnt = wave_sum(cnt);
  if (lane == 0) out[i] = cnt > MAX_EDGES ? -1 : cnt;
}

// Label of pixel (y, x), which is set: the run of row y that holds x (-1 if
// no run holds it, which a consistent clip set never gives).
__device__ int label_at(const uint16_t* rp, const uint32_t* ru, int y, int x) {
  for (int k = rp[y]; k < rp[y + 1]; ++k) {
    const uint32_t r = ru[k];
    if ((int)(r & 511) <= x && x < (int)((r >> 9) & 511)) return (int)((r >> 18) & 63);
  }
  return -1;
}

template <int NMAX>
struct TraceLds {
  static constexpr int CWM = NMAX / 64 + 1;
  uint64_t bits[NMAX * NMAX / 64];
  uint64_t vtx[(NMAX + 1) * CWM];     // vertex rows: bit X of row Y
  uint64_t vcol[(NMAX + 1) * CWM];    // the same bits by column: bit Y of column X
  uint64_t vis[2][(NMAX + 1) * CWM];  // passages leaving E or S / W or N
  uint64_t busy[(NMAX + 64) / 64];    // corner rows holding a vertex
  uint16_t edge[MAX_EDGES];           // coordinate | direction << 9, in walk order
  uint16_t c_start[MAX_CONTOURS], c_len[MAX_CONTOURS], c_rot[MAX_CONTOURS];
  uint8_t c_label[MAX_CONTOURS];
  int n_contours, n_edges, bad;
};

template <int N, int NMAX>
__device__ void trace_clip(const ClipsDev& cs, int64_t i, TraceLds<NMAX>& L) {
  constexpr int WPR = N / 64, CW = WPR + 1;
  const int lane = threadIdx.x;
  const uint64_t* gbits = cs.bits + cs.bits_off[i];
  for (int t = lane; t < N * WPR; t += 64) L.bits[t] = gbits[t];
  __syncthreads();
  for (int Y0 = 0; Y0 <= N; Y0 += 64) {
    const int Y = Y0 + lane;
    uint64_t any = 0ull;
    if (Y <= N) {
      vertex_row<N>(Y >= 1 ? L.bits + (Y - 1) * WPR : nullptr, Y < N ? L.bits + Y * WPR : nullptr, L.vtx + Y * CW,
                    nullptr);
#pragma unroll
      for (int w = 0; w < CW; ++w) {
        any |= L.vtx[Y * CW + w];
        L.vis[0][Y * CW + w] = 0ull;
        L.vis[1][Y * CW + w] = 0ull;
      }
    }
    const unsigned long long rows = __ballot(any != 0ull);
    if (lane == 0) L.busy[Y0 >> 6] = rows;
  }
  __syncthreads();
  // column bitmaps, one column per lane at a time
  for (int X = lane; X <= N; X += 64) {
#pragma unroll
    for (int wy = 0; wy < CW; ++wy) {
      uint64_t col = 0ull;
      const int y1 = min(N, 64 * wy + 63);
      for (int Y = 64 * wy; Y <= y1; ++Y) col |= ((L.vtx[Y * CW + (X >> 6)] >> (X & 63)) & 1ull) << (Y & 63);
      L.vcol[X * CW + wy] = col;
    }
  }
  __syncthreads();

  if (lane == 0) {
    const uint16_t* rp = cs.run_rowptr + cs.rowptr_off[i];
    const uint32_t* ru = cs.runs + cs.run_off[i];
    auto pix = [&](int y, int x) -> int {
      if (y < 0 || y >= N || x < 0 || x >= N) return 0;
      return (int)((L.bits[y * WPR + (x >> 6)] >> (x & 63)) & 1ull);
    };
    // next set bit above `from` (or below it, down = true) in a bitmap of CW
    // words; -1 when none
    auto next_bit = [&](const uint64_t* words, int from, bool down) -> int {
      if (!down) {
        int t = from + 1, w = t >> 6;
        if (w >= CW) return -1;
        uint64_t m = words[w] & (~0ull << (t & 63));
        while (!m && ++w < CW) m = words[w];
        return m ? w * 64 + __builtin_ctzll(m) : -1;
      }
      int t = from - 1, w = t >> 6;
      if (t < 0) return -1;
      uint64_t m = words[w] & (~0ull >> (63 - (t & 63)));
      while (!m && --w >= 0) m = words[w];
      return m ? w * 64 + 63 - __builtin_clzll(m) : -1;
    };
    auto visited = [&](int y, int x, int d) -> bool {
      return (L.vis[d == DIR_E || d == DIR_S ? 0 : 1][y * CW + (x >> 6)] >> (x & 63)) & 1ull;
    };
    auto mark = [&](int y, int x, int d) {
      L.vis[d == DIR_E || d == DIR_S ? 0 : 1][y * CW + (x >> 6)] |= 1ull << (x & 63);
    };
    int ne = 0, nc = 0, bad = 0;
    for (int Y0 = 0; Y0 <= N && !bad; ++Y0) {
      if (!((L.busy[Y0 >> 6] >> (Y0 & 63)) & 1ull)) continue;
      for (int w0 = 0; w0 < CW && !bad; ++w0) {
        uint64_t row = L.vtx[Y0 * CW + w0];
        while (row && !bad) {
          const int X0 = w0 * 64 + __builtin_ctzll(row);
          row &= row - 1ull;
          const int a = pix(Y0 - 1, X0 - 1), b = pix(Y0 - 1, X0), c = pix(Y0, X0 - 1), dd = pix(Y0, X0);
          const bool out[4] = {dd && !b, c && !dd, a && !c, b && !a};
          for (int d0 = 0; d0 < 4 && !bad; ++d0) {
            if (!out[d0] || visited(Y0, X0, d0)) continue;
            if (nc >= MAX_CONTOURS) { bad = 1; break; }
            // the polygon pixel right of the first side names the contour's polygon
            const int py = (d0 == DIR_E || d0 == DIR_S) ? Y0 : Y0 - 1;
            const int px = (d0 == DIR_E || d0 == DIR_N) ? X0 : X0 - 1;
            const int start = ne;
            int X = X0, Y = Y0, d = d0;
            for (;;) {
              if (ne >= MAX_EDGES) { bad = 1; break; }
              mark(Y, X, d);
              L.edge[ne++] = (uint16_t)(((d == DIR_E || d == DIR_W) ? Y : X) | (d << 9));
              // along d to the next vertex (one exists: the contour closes)
              if (d == DIR_E || d == DIR_W) X = next_bit(L.vtx + Y * CW, X, d == DIR_W);
              else Y = next_bit(L.vcol + X * CW, Y, d == DIR_N);
              if (X < 0 || X > N || Y < 0 || Y > N) { bad = 1; break; }
              const int a2 = pix(Y - 1, X - 1), b2 = pix(Y - 1, X), c2 = pix(Y, X - 1), d2 = pix(Y, X);
              if ((a2 && d2 && !b2 && !c2) || (b2 && c2 && !a2 && !d2)) d = (d + 1) & 3;
              else if (d2 && !b2) d = DIR_E;
              else if (c2 && !d2) d = DIR_S;
              else if (a2 && !c2) d = DIR_W;
              else d = DIR_N;
              if (X == X0 && Y == Y0 && d == d0) break;
            }
            if (bad) break;
            const int label = label_at(rp, ru, py, px);
            if (label < 0) { bad = 1; break; }  // the clip then has no contour data
            L.c_start[nc] = (uint16_t)start;
            L.c_len[nc] = (uint16_t)(ne - start);
            L.c_label[nc] = (uint8_t)label;
            ++nc;
          }
        }
      }
    }
    L.n_contours = nc;
    L.n_edges = ne;
    L.bad = bad;
  }
  __syncthreads();
  const int nc = L.n_contours;
  // least rotation of each contour's direction codes (unique: a closed
  // rectilinear contour's code sequence has no shorter period)
  for (int c = lane; c < nc; c += 64) {
    const uint16_t* e = L.edge + L.c_start[c];
    const int n = L.c_len[c];
    int p = 0, q = 1, k = 0;
    while (p < n && q < n && k < n) {
      int ip = p + k, iq = q + k;
      if (ip >= n) ip -= n;
      if (iq >= n) iq -= n;
      const int cp = (e[ip] >> 9) & 3, cq = (e[iq] >> 9) & 3;
      if (cp == cq) {
        ++k;
        continue;
      }
      if (cp > cq) p += k + 1;
      else q += k + 1;
      if (p == q) ++q;
      k = 0;
    }
    L.c_rot[c] = (uint16_t)min(p, q);
  }
  __syncthreads();
}

template <int NMAX>
__global__ void __launch_bounds__(64) contour_trace_kernel(ClipsDev cs, int64_t block0) {
  __shared__ TraceLds<NMAX> L;
  const int64_t i = block0 + (int64_t)blockIdx.x;
  if (i >= cs.n) return;  // block-uniform
  const int lane = threadIdx.x;
  const int total = cs.cstat[i];
  uint16_t* cp = cs.cpoly + i * (MAX_POLY + 1);
  uint32_t* ch = cs.chash + i * MAX_POLY;
  if (total <= 0) {  // no contour data, or no polygon
    for (int t = lane; t <= MAX_POLY; t += 64) cp[t] = 0;
    if (lane < MAX_POLY) ch[lane] = 0;
    return;
  }
  const int N = cs.N[i];
  if (N == 64) trace_clip<64, NMAX>(cs, i, L);
  else if constexpr (NMAX >= 128) {
    if (N == 128) trace_clip<128, NMAX>(cs, i, L);
    else if constexpr (NMAX >= 256) trace_clip<256, NMAX>(cs, i, L);
  }
  const int P = cs.npoly[i];
  const int nc = L.n_contours;
  // edges per polygon, then their offsets (lane p holds polygon p)
  int mine = 0;
  if (lane < P)
    for (int c = 0; c < nc; ++c)
      if (L.c_label[c] == lane) mine += L.c_len[c];
  int incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  const int off = incl - mine;
  const bool ok = L.bad == 0 && L.n_edges == total && __shfl(incl, 63) == total;
  if (!ok) {  // cannot happen when the count pass is consistent; no contour data then
    if (lane == 0) cs.cstat[i] = -1;
    for (int t = lane; t <= MAX_POLY; t += 64) cp[t] = 0;
    if (lane < MAX_POLY) ch[lane] = 0;
    return;
  }
  uint16_t* out = cs.cedges + cs.cedge_off[i];
  if (lane < P) {
    int pos = off;
    uint64_t h = FNV_OFFSET;
    for (int c = 0; c < nc; ++c) {
      if (L.c_label[c] != lane) continue;
      const uint16_t* e = L.edge + L.c_start[c];
      const int n = L.c_len[c], r = L.c_rot[c];
      for (int k = 0; k < n; ++k) {
        int t = r + k;
        if (t >= n) t -= n;
        const uint16_t wv = e[t];
        out[pos++] = (uint16_t)(wv | (k == 0 ? (1u << 11) : 0u));
        h = (h ^ (uint64_t)((wv >> 9) & 3)) * FNV_PRIME;
      }
      h = (h ^ 4ull) * FNV_PRIME;
    }
    cp[lane] = (uint16_t)off;
    ch[lane] = (uint32_t)h;
  } else if (lane < MAX_POLY) {
    ch[lane] = 0;
  }
  for (int t = P + lane; t <= MAX_POLY; t += 64) cp[t] = (uint16_t)total;  // end of the last polygon
}

}  // namespace

hipError_t launch_contour_count(const ClipsDev& cs, int32_t* counts, hipStream_t s) {
  for (int64_t b0 = 0; b0 < cs.n; b0 += LAUNCH_CHUNK) {
    const unsigned nb = (unsigned)std::min<int64_t>(LAUNCH_CHUNK, cs.n - b0);
    hipLaunchKernelGGL(contour_count_kernel, dim3(nb), dim3(64), 0, s, cs, b0, counts);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_contour_trace(const ClipsDev& cs, int maxN, hipStream_t s) {
  for (int64_t b0 = 0; b0 < cs.n; b0 += LAUNCH_CHUNK) {
    const unsigned nb = (unsigned)std::min<int64_t>(LAUNCH_CHUNK, cs.n - b0);
    if (maxN <= 64) hipLaunchKernelGGL(contour_trace_kernel<64>, dim3(nb), dim3(64), 0, s, cs, b0);
    else if (maxN <= 128) hipLaunchKernelGGL(contour_trace_kernel<128>, dim3(nb), dim3(64), 0, s, cs, b0);
    else hipLaunchKernelGGL(contour_trace_kernel<256>, dim3(nb), dim3(64), 0, s, cs, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ca
