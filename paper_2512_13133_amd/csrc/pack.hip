// Rasterise and pack clips (paper Sec. 2.1 Eq. 1; Sec. 2.2.1 step 1).
//
// pack_kernel: one workgroup per clip.  The N x N raster is built in LDS as
// bit-packed rows (bit x of row y in word y*N/64 + x/64), one thread per
// 64-bit word ORing the span masks of every rectangle that crosses its row.
// It then writes the packed bits, the pixel count, row and column sums and
// the number of row runs.
//
// label_kernel: one workgroup per clip.  Row runs are extracted in parallel,
// then the 4-connected polygons are labelled by a lock-free union-find over
// runs of adjacent rows (one thread per row pair), giving each polygon its
// bounding box, and each run its polygon label.
#include "kernels.h"

namespace ca {

__device__ __forceinline__ uint64_t span_mask(int a, int b) {
  // bits a..b-1 of a word, 0 <= a < b <= 64
  uint64_t hi = (b >= 64) ? ~0ull : ((1ull << b) - 1ull);
  uint64_t lo = (1ull << a) - 1ull;
  return hi & ~lo;
}

__global__ void __launch_bounds__(256) pack_kernel(const int64_t* __restrict__ rect_ptr,
                                                   const int32_t* __restrict__ rects,
                                                   ClipsDev cs, int64_t block0) {
  __shared__ uint64_t sb[256 * 4];
  __shared__ int red[256];
  __shared__ int srow[256], scol[256];
  const int64_t i = block0 + (int64_t)blockIdx.x;
  const int tid = threadIdx.x;
  const int N = cs.N[i];
  const int wpr = N / 64;
  const int nw = N * wpr;
  const int64_t lo = rect_ptr[i], hi = rect_ptr[i + 1];
  for (int t = tid; t < nw; t += blockDim.x) {
    const int y = t / wpr, k = t - y * wpr;
    uint64_t m = 0;
    for (int64_t r = lo; r < hi; ++r) {
      const int32_t* rc = rects + 4 * r;
      int x0 = max(rc[0], 0), x1 = min(rc[1], N);
      int y0 = max(rc[2], 0), y1 = min(rc[3], N);
      if (y < y0 || y >= y1) continue;
      int a = max(x0, 64 * k), b = min(x1, 64 * k + 64);
      if (a < b) m |= span_mask(a - 64 * k, b - 64 * k);
    }
    sb[t] = m;
  }
  __syncthreads();
  uint64_t* gbits = cs.bits + cs.bits_off[i];
  for (int t = tid; t < nw; t += blockDim.x) gbits[t] = sb[t];
  // row sums, run counts and the pixel total: one thread per row
  int cnt = 0;
  int runs = 0;
  uint16_t* rs = cs.rowsum + cs.sig_off[i];
  uint16_t* cls = cs.colsum + cs.sig_off[i];
  if (tid < N) {
    int c = 0, prev = 0;
    for (int k = 0; k < wpr; ++k) {
      uint64_t wv = sb[tid * wpr + k];
      c += __popcll(wv);
      // run starts: set bits whose left neighbour is clear
      uint64_t starts = wv & ~((wv << 1) | (uint64_t)prev);
      runs += __popcll(starts);
      prev = (int)(wv >> 63);
    }
    rs[tid] = (uint16_t)c;
    srow[tid] = c;
    cnt = c;
    // column sum of column tid
    int cc = 0;
    const int kk = tid >> 6, bb = tid & 63;
    for (int y = 0; y < N; ++y) cc += (int)((sb[y * wpr + kk] >> bb) & 1ull);
    cls[tid] = (uint16_t)cc;
    scol[tid] = cc;
  }
  // sliding 8-row / 8-column sums for the coarse pruning bound
  __syncthreads();
  if (tid < N) {
    int wr = 0, wc = 0;
    for (int t = 0; t < 8; ++t) {
      const int y = (tid + t) & (N - 1);
      wr += srow[y];
      wc += scol[y];
    }
    cs.winrow[cs.sig_off[i] + tid] = (uint16_t)wr;
    cs.wincol[cs.sig_off[i] + tid] = (uint16_t)wc;
  }
  red[tid] = cnt;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) cs.npix[i] = red[0];
  __syncthreads();
  red[tid] = runs;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) cs.nruns[i] = red[0];
}

// Root of x in a forest whose links only point to smaller indices
// (parent[x] <= x); reads may race with links made by other threads, which
// only move a root further up.
__device__ __forceinline__ int uf_root(volatile int* parent, int x) {
  int p = parent[x];
  while (p != x) {
    x = p;
    p = parent[x];
  }
  return x;
}

// Join the sets of a and b: the larger root is linked under the smaller one
// by a compare-and-swap that succeeds only while it is still a root.
__device__ __forceinline__ void uf_unite(int* parent, int a, int b) {
  while (true) {
    a = uf_root(parent, a);
    b = uf_root(parent, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    if (atomicCAS(parent + a, a, b) == a) return;
  }
}

// Polygons are the 4-connected components of the row runs.  Rows are merged
// with their predecessor in parallel (one thread per row pair); each
// component's root is its smallest run index, i.e. its first run in raster
// order, and labels number the roots in that order (an exclusive scan).
__global__ void __launch_bounds__(256) label_kernel(ClipsDev cs, int64_t block0) {
  __shared__ uint32_t srun[MAX_RUNS];   // x0 | x1 << 9 | y << 18
  __shared__ int parent[MAX_RUNS];
  __shared__ int16_t slabel[MAX_RUNS];
  __shared__ uint16_t rowp[257];
  __shared__ uint16_t rcount[256];
  __shared__ int box[MAX_POLY][4];
  __shared__ int wsum[4];
  __shared__ int gbx[4];
  const int64_t i = block0 + (int64_t)blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int N = cs.N[i];
  const int wpr = N / 64;
  const int total = cs.nruns[i];
  int16_t* gb = cs.gbox + 4 * i;
  int16_t* bx = cs.boxes + (int64_t)i * MAX_POLY * 4;
  if (total > MAX_RUNS) {  // too fragmented for the labeller: no polygons kept
    if (tid == 0) {
      cs.npoly[i] = -1;
      gb[0] = gb[1] = gb[2] = gb[3] = 0;
    }
    return;
  }
  const uint64_t* bits = cs.bits + cs.bits_off[i];
  // per-row run counts -> exclusive prefix in rowp (serial over <= 256 rows)
  if (tid < N) {
    int runs = 0;
    int prev = 0;
    for (int k = 0; k < wpr; ++k) {
      uint64_t wv = bits[tid * wpr + k];
      runs += __popcll(wv & ~((wv << 1) | (uint64_t)prev));
      prev = (int)(wv >> 63);
    }
    rcount[tid] = (uint16_t)runs;
  }
  if (tid < MAX_POLY) {
    box[tid][0] = box[tid][2] = 1 << 20;
    box[tid][1] = box[tid][3] = -1;
  }
  if (tid < 4) gbx[tid] = (tid & 1) ? -1 : (1 << 20);
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int y = 0; y < N; ++y) {
      rowp[y] = (uint16_t)acc;
      acc += rcount[y];
    }
    rowp[N] = (uint16_t)acc;
  }
  __syncthreads();
  // extract runs of each row in x order
  if (tid < N) {
    int o = rowp[tid];
    int x = 0;
    while (x < N) {
      // find next set bit at or after x
      int k = x >> 6;
      uint64_t wv = bits[tid * wpr + k] & (~0ull << (x & 63));
      while (wv == 0 && ++k < wpr) wv = bits[tid * wpr + k];
      if (k >= wpr) break;
      int a = 64 * k + __ffsll((unsigned long long)wv) - 1;
      // find next clear bit at or after a
      int k2 = a >> 6;
      uint64_t nv = ~bits[tid * wpr + k2] & (~0ull << (a & 63));
      while (nv == 0 && ++k2 < wpr) nv = ~bits[tid * wpr + k2];
      int b = (k2 >= wpr) ? N : 64 * k2 + __ffsll((unsigned long long)nv) - 1;
      srun[o++] = (uint32_t)a | ((uint32_t)b << 9) | ((uint32_t)tid << 18);
      x = b;
    }
  }
  for (int t = tid; t < total; t += blockDim.x) parent[t] = t;
  __syncthreads();
  // union runs of row y-1 and row y that share a column (4-connectivity)
  for (int y = 1 + tid; y < N; y += blockDim.x) {
    int a = rowp[y - 1], ae = rowp[y];
    int b = rowp[y], be = rowp[y + 1];
    while (a < ae && b < be) {
      const int a0 = srun[a] & 511, a1 = (srun[a] >> 9) & 511;
      const int b0 = srun[b] & 511, b1 = (srun[b] >> 9) & 511;
      if (a0 < b1 && b0 < a1) uf_unite(parent, a, b);
      if (a1 < b1) ++a;
      else ++b;
    }
  }
  __syncthreads();
  // labels of the roots: exclusive count of roots before them, in chunks of
  // the workgroup size
  int base = 0;
  for (int c0 = 0; c0 < total; c0 += blockDim.x) {
    const int r = c0 + tid;
    const bool root = r < total && parent[r] == r;
    const unsigned long long m = __ballot(root);
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int before = base;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (root) slabel[r] = (int16_t)(before + __popcll(m & ((1ull << lane) - 1ull)));
    base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
  const int np = base;
  // every run takes its root's label; boxes by LDS atomics
  for (int r = tid; r < total; r += blockDim.x) {
    const int root = uf_root(parent, r);
    const int lab = slabel[root];
    if (root != r) slabel[r] = (int16_t)lab;
    const uint32_t w = srun[r];
    const int x0 = w & 511, x1 = (w >> 9) & 511, y = (w >> 18) & 511;
    if (lab < MAX_POLY) {
      atomicMin(&box[lab][0], x0);
      atomicMax(&box[lab][1], x1);
      atomicMin(&box[lab][2], y);
      atomicMax(&box[lab][3], y + 1);
    }
    atomicMin(&gbx[0], x0);
    atomicMax(&gbx[1], x1);
    atomicMin(&gbx[2], y);
    atomicMax(&gbx[3], y + 1);
  }
  __syncthreads();
  if (tid == 0) {
    if (total == 0) gb[0] = gb[1] = gb[2] = gb[3] = 0;
    else {
      gb[0] = (int16_t)gbx[0]; gb[1] = (int16_t)gbx[1]; gb[2] = (int16_t)gbx[2]; gb[3] = (int16_t)gbx[3];
    }
    cs.npoly[i] = np > MAX_POLY ? -1 : np;
  }
  const int npb = min(np, MAX_POLY);
  for (int t = tid; t < npb * 4; t += blockDim.x) bx[t] = (int16_t)box[t >> 2][t & 3];
  uint32_t* gr = cs.runs + cs.run_off[i];
  for (int t = tid; t < total; t += blockDim.x)
    gr[t] = (srun[t] & 0x3ffffu) | ((uint32_t)min((int)slabel[t], MAX_POLY - 1) << 18);
  uint16_t* grp = cs.run_rowptr + cs.rowptr_off[i];
  for (int t = tid; t <= N; t += blockDim.x) grp[t] = rowp[t];
}

}  // namespace ca

namespace ca {

// Pair validation: ids in range, equal raster sizes, and (for the edge track)
// polygon tables within the cap, and (need_poly 2: full boundary edges)
// contour data.  Sets *bad to 1 (ids/sizes), 2 (polygons) or 4 (contours).
__global__ void validate_pairs_kernel(ClipsDev cr, ClipsDev cm, int64_t n_pairs, const int32_t* __restrict__ rep,
                                      const int32_t* __restrict__ mem, int need_poly, int* bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_pairs) return;
  const int a = rep[k], b = mem[k];
  if (a < 0 || b < 0 || a >= cr.n || b >= cm.n || cr.N[a] != cm.N[b]) {
    atomicOr(bad, 1);
    return;
  }
  if (need_poly && (cr.npoly[a] < 0 || cm.npoly[b] < 0)) atomicOr(bad, 2);
  else if (need_poly == 2 && (cr.cstat[a] < 0 || cm.cstat[b] < 0)) atomicOr(bad, 4);
}

hipError_t launch_pack(const int64_t* rect_ptr, const int32_t* rects, const ClipsDev& cs, int64_t n,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  for (int64_t b0 = 0; b0 < n; b0 += LAUNCH_CHUNK) {
    const unsigned nb = (unsigned)std::min<int64_t>(LAUNCH_CHUNK, n - b0);
    hipLaunchKernelGGL(pack_kernel, dim3(nb), dim3(256), 0, s, rect_ptr, rects, cs, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_label(const ClipsDev& cs, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  for (int64_t b0 = 0; b0 < n; b0 += LAUNCH_CHUNK) {
    const unsigned nb = (unsigned)std::min<int64_t>(LAUNCH_CHUNK, n - b0);
    hipLaunchKernelGGL(label_kernel, dim3(nb), dim3(256), 0, s, cs, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Clears device counters with a kernel (usable under graph capture, where
// memset nodes are avoided).
__global__ void zero_u64_kernel(unsigned long long* p, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// Copy of a pair list with every pair whose ids fall outside [0, n_r) x
// [0, n_m) replaced by (0, 0) and marked (bad[k] = 1; *n_bad counts them).
__global__ void sanitize_pairs_kernel(int64_t n, const int32_t* __restrict__ rep, const int32_t* __restrict__ mem,
                                      int64_t n_r, int64_t n_m, int32_t* __restrict__ rep_o,
                                      int32_t* __restrict__ mem_o, uint8_t* __restrict__ bad,
                                      unsigned long long* n_bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int a = rep[k], b = mem[k];
  const bool ok = a >= 0 && b >= 0 && a < n_r && b < n_m;
  rep_o[k] = ok ? a : 0;
  mem_o[k] = ok ? b : 0;
  bad[k] = ok ? 0 : 1;
  if (!ok) atomicAdd(n_bad, 1ull);
}

// Results of the marked pairs: no result (bits 0, shifts 0, counts -1, scores 0, CA_FLAG_INVALID).
__global__ void reject_pairs_kernel(int64_t n, const uint8_t* __restrict__ bad, PairIO io) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || !bad[k]) return;
  io.bits[k] = 0;
  io.flags[k] = CA_FLAG_INVALID;
  for (int e = 0; e < 4; ++e) io.shift[4 * k + e] = 0;
  for (int e = 0; e < 2; ++e) {
    io.count[2 * k + e] = -1;
    io.score[2 * k + e] = 0.0;
  }
}

hipError_t launch_sanitize_pairs(int64_t n, const int32_t* rep, const int32_t* mem, int64_t n_r, int64_t n_m,
                                 int32_t* rep_o, int32_t* mem_o, uint8_t* bad, unsigned long long* n_bad,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(sanitize_pairs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, rep, mem, n_r, n_m,
                     rep_o, mem_o, bad, n_bad);
  return hipGetLastError();
}

hipError_t launch_reject_pairs(int64_t n, const uint8_t* bad, const PairIO& io, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(reject_pairs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, bad, io);
  return hipGetLastError();
}

hipError_t launch_validate(const ClipsDev& cr, const ClipsDev& cm, int64_t n_pairs, const int32_t* rep,
                           const int32_t* mem, int need_poly, int* bad, hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n_pairs + 255) / 256);
  hipLaunchKernelGGL(validate_pairs_kernel, dim3(blocks), dim3(256), 0, s, cr, cm, n_pairs, rep, mem,
                     need_poly, bad);
  return hipGetLastError();
}

}  // namespace ca
