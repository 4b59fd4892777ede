// Cover compaction and center verification (paper Sec. 3.1 stage 2: the
// sparse similarity graph that the set cover of Sec. 3.3 consumes; Sec. 2.3:
// every member must satisfy the constraint at its center against its
// representative).
//
// Compaction turns the per-pair results of an alignment call (both
// directions of each unordered candidate pair) into a CSR relation sorted by
// (representative, member): row r lists the members r covers.
//   1. count: one atomic per set direction on the row of its representative;
//   2. (host) exclusive scan of the row counts into row pointers;
//   3. scatter: each set direction appends the key (member << 32 | 2 k + d)
//      to its row (any order: per-row atomic cursor);
//   4. sort each row by key.  Members are distinct within a row (each
//      unordered pair occurs once in a candidate list), so the order is
//      unique whatever the scatter order was.  Rows of <= 64 keys: one wave,
//      rank by counting; <= 4,096: one workgroup, bitonic sort in LDS;
//      longer: 4,096-key chunks sorted in LDS, then merge passes in global
//      memory where each key's output position is its index in its run plus
//      its rank in the sibling run (binary search);
//   5. gather: column, shift, count and score of each sorted key.
// A candidate list too long to align at once is aligned in pieces; each
// piece keeps only its pairs with a set direction (with their results, in any
// order: the row sort makes the relation unique), and steps 1-5 run on the
// kept pairs.
#include "kernels.h"
#include "pair_common.h"

namespace ca {

namespace {

constexpr int SORT_LDS = 4096;  // keys per LDS sort

__global__ void cover_count_kernel(int64_t n_pairs, const int32_t* __restrict__ rep, const int32_t* __restrict__ mem,
                                   const uint8_t* __restrict__ bits, unsigned long long* __restrict__ rowcnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_pairs) return;
  const uint8_t b = bits[k];
  if (b & 1u) atomicAdd(&rowcnt[rep[k]], 1ull);
  if (b & 2u) atomicAdd(&rowcnt[mem[k]], 1ull);
}

__global__ void cover_scatter_kernel(int64_t n_pairs, const int32_t* __restrict__ rep,
                                     const int32_t* __restrict__ mem, const uint8_t* __restrict__ bits,
                                     const int64_t* __restrict__ row_ptr, unsigned long long* __restrict__ fill,
                                     uint64_t* __restrict__ keys) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_pairs) return;
  const uint8_t b = bits[k];
  const int32_t a = rep[k], m = mem[k];
  if (b & 1u) {  // direction 0: rep covers mem
    const int64_t pos = row_ptr[a] + (int64_t)atomicAdd(&fill[a], 1ull);
    keys[pos] = ((uint64_t)(uint32_t)m << 32) | (uint64_t)(2 * k);
  }
  if (b & 2u) {  // direction 1: mem covers rep
    const int64_t pos = row_ptr[m] + (int64_t)atomicAdd(&fill[m], 1ull);
    keys[pos] = ((uint64_t)(uint32_t)a << 32) | (uint64_t)(2 * k + 1);
  }
}

// Pairs of a piece with at least one set direction (keep_count: how many).
__global__ void cover_keep_count_kernel(int64_t n_pairs, const uint8_t* __restrict__ bits,
                                        unsigned long long* __restrict__ n_keep) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = k < n_pairs && (bits[k] & 3u) != 0;
  const unsigned long long m = __ballot(on);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(n_keep, (unsigned long long)__popcll(m));
}

// Copies the kept pairs and both directions' results (shift: 4 int16, count:
// 2 int32, score: 2 double per pair) to slots taken from *slot, one atomic
// per wave.
__global__ void cover_keep_kernel(int64_t n_pairs, const int32_t* __restrict__ rep, const int32_t* __restrict__ mem,
                                  const uint8_t* __restrict__ bits, const uint64_t* __restrict__ shift,
                                  const uint64_t* __restrict__ count, const double* __restrict__ score,
                                  unsigned long long* __restrict__ slot, int32_t* __restrict__ k_rep,
                                  int32_t* __restrict__ k_mem, uint8_t* __restrict__ k_bits,
                                  uint64_t* __restrict__ k_shift, uint64_t* __restrict__ k_count,
                                  double* __restrict__ k_score) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const uint8_t b = k < n_pairs ? bits[k] : 0;
  const bool on = (b & 3u) != 0;
  const unsigned long long m = __ballot(on);
  if (!m) return;  // wave-uniform
  const int leader = __ffsll((long long)m) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(slot, (unsigned long long)__popcll(m));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)base, leader);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(base >> 32), leader);
  if (!on) return;
  const int64_t j = (int64_t)(((uint64_t)hi << 32) | lo) + __popcll(m & ((1ull << lane) - 1ull));
  k_rep[j] = rep[k];
  k_mem[j] = mem[k];
  k_bits[j] = b;
  k_shift[j] = shift[k];
  k_count[j] = count[k];
  k_score[2 * j] = score[2 * k];
  k_score[2 * j + 1] = score[2 * k + 1];
}

// Rows of at most 64 keys, one wave per row (four rows per workgroup): each
// lane's key goes to its rank among the row's keys.
__global__ void __launch_bounds__(256) cover_sort_small_kernel(const int32_t* __restrict__ rows, int64_t n_rows,
                                                               const int64_t* __restrict__ row_ptr,
                                                               uint64_t* __restrict__ keys) {
  __shared__ uint64_t s_key[4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + wave;
  if (t >= n_rows) return;  // wave-uniform: no barrier below
  const int r = rows[t];
  const int64_t b = row_ptr[r];
  const int L = (int)(row_ptr[r + 1] - b);
  const uint64_t key = lane < L ? keys[b + lane] : ~0ull;
  s_key[wave][lane] = key;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int rank = 0;
  for (int j = 0; j < L; ++j) rank += s_key[wave][j] < key ? 1 : 0;
  if (lane < L) keys[b + rank] = key;
}

// Bitonic sort of P keys (P a power of two <= SORT_LDS) in LDS by the block.
__device__ void lds_bitonic(uint64_t* s, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += blockDim.x) {
        const int lo = 2 * j * (t / j) + (t % j), hi = lo + j;
        const bool up = (lo & k) == 0;
        const uint64_t a = s[lo], c = s[hi];
        if ((a > c) == up) {
          s[lo] = c;
          s[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

// Sort keys[b, b + L) with L <= SORT_LDS in LDS.
__device__ void sort_chunk(uint64_t* keys, int64_t b, int L, uint64_t* s) {
  int P = 1;
  while (P < L) P <<= 1;
  for (int t = threadIdx.x; t < P; t += blockDim.x) s[t] = t < L ? keys[b + t] : ~0ull;
  __syncthreads();
  lds_bitonic(s, P);
  for (int t = threadIdx.x; t < L; t += blockDim.x) keys[b + t] = s[t];
  __syncthreads();
}

// Number of keys in run[0, n) smaller than x (run sorted ascending).
__device__ __forceinline__ int64_t rank_in(const uint64_t* run, int64_t n, uint64_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (run[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Rows longer than 64 keys, one workgroup per row.  Rows up to SORT_LDS keys
// are sorted in LDS; longer rows are sorted in SORT_LDS chunks and merged in
// passes between keys and tmp (the same offsets), ending in keys.
__global__ void __launch_bounds__(256) cover_sort_large_kernel(const int32_t* __restrict__ rows,
                                                               const int64_t* __restrict__ row_ptr, uint64_t* keys,
                                                               uint64_t* tmp) {
  __shared__ uint64_t s[SORT_LDS];
  const int r = rows[blockIdx.x];
  const int64_t b = row_ptr[r];
  const int64_t L = row_ptr[r + 1] - b;
  if (L <= SORT_LDS) {
    sort_chunk(keys, b, (int)L, s);
    return;
  }
  for (int64_t c = 0; c < L; c += SORT_LDS) sort_chunk(keys, b + c, (int)min((int64_t)SORT_LDS, L - c), s);
  uint64_t* src = keys + b;
  uint64_t* dst = tmp + b;
  for (int64_t w = SORT_LDS; w < L; w <<= 1) {
    for (int64_t e = threadIdx.x; e < L; e += blockDim.x) {
      const int64_t base = (e / (2 * w)) * (2 * w);
      const int64_t na = min(w, L - base), nb = max((int64_t)0, min(w, L - base - w));
      const uint64_t x = src[e];
      int64_t out;
      if (e - base < na) out = base + (e - base) + rank_in(src + base + na, nb, x);
      else out = base + (e - base - na) + rank_in(src + base, na, x);
      dst[out] = x;
    }
    __syncthreads();
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  if (src != keys + b) {
    for (int64_t e = threadIdx.x; e < L; e += blockDim.x) keys[b + e] = src[e];
  }
}

__global__ void cover_gather_kernel(int64_t nnz, const uint64_t* __restrict__ keys, const int16_t* __restrict__ shift,
                                    const int32_t* __restrict__ count, const double* __restrict__ score,
                                    int32_t* __restrict__ col, int16_t* __restrict__ col_shift,
                                    int32_t* __restrict__ value, double* __restrict__ col_score) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const uint64_t key = keys[e];
  const int64_t idx = (int64_t)(key & 0xffffffffull);  // 2 k + d
  col[e] = (int32_t)(key >> 32);
  col_shift[2 * e] = shift[2 * idx];
  col_shift[2 * e + 1] = shift[2 * idx + 1];
  value[e] = count[idx];
  col_score[e] = score[idx];
}

// Dense bit matrix from the CSR: bit m of row r (word r * words + m / 64).
__global__ void cover_dense_kernel(int64_t n, int64_t words, const int64_t* __restrict__ row_ptr,
                                   const int32_t* __restrict__ col, unsigned long long* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  unsigned long long* row = out + r * words;
  row[r >> 6] |= 1ull << (r & 63);  // the diagonal: every clip covers itself
  for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
    const int m = col[e];
    row[m >> 6] |= 1ull << (m & 63);
  }
}

// Cosine center verification: one wave per member (Eq. 2 at the member's
// center, exact): the shift must be a window residue of the member, and the
// overlap count c at it must satisfy c^2 q^2 > p^2 n_m n_r.
__global__ void __launch_bounds__(256) verify_cosine_kernel(ClipsDev cs, int64_t n, int64_t t0,
                                                            const int32_t* __restrict__ mem,
                                                            const int32_t* __restrict__ rep,
                                                            const int16_t* __restrict__ shift, Threshold thr,
                                                            unsigned long long* viol, unsigned long long* first) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t t = t0 + (int64_t)blockIdx.x * 4 + wave;
  if (t >= n) return;
  const int m = mem[t], r = rep[t];
  const int N = cs.N[m];
  const int dy = shift[2 * t], dx = shift[2 * t + 1];
  bool ok = cs.N[r] == N;
  if (ok) {
    const int w = cs.w[m];
    const bool all = 2 * w + 1 > N;  // every residue, named in [-N/2, N/2 - 1]
    ok = all ? (dy >= -N / 2 && dy < N / 2 && dx >= -N / 2 && dx < N / 2)
             : (dy >= -w && dy <= w && dx >= -w && dx <= w);
  }
  int c = 0;
  if (ok) {
    const uint64_t* br = cs.bits + cs.bits_off[r];
    const uint64_t* bm = cs.bits + cs.bits_off[m];
    for (int y = lane; y < N; y += 64) c += row_overlap(br, bm, N, y, dy, dx);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    ok = cosine_bit(c, cs.npix[m], cs.npix[r], thr);
  }
  if (!ok && lane == 0) {
    atomicAdd(viol, 1ull);
    atomicMin(first, (unsigned long long)t);
  }
}

}  // namespace

hipError_t launch_cover_count(int64_t n_pairs, const int32_t* rep, const int32_t* mem, const uint8_t* bits,
                              unsigned long long* rowcnt, hipStream_t s) {
  for (int64_t k0 = 0; k0 < n_pairs; k0 += LAUNCH_CHUNK * 256) {
    const int64_t nk = std::min<int64_t>(LAUNCH_CHUNK * 256, n_pairs - k0);
    hipLaunchKernelGGL(cover_count_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s, nk, rep + k0,
                       mem + k0, bits + k0, rowcnt);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cover_keep_count(int64_t n_pairs, const uint8_t* bits, unsigned long long* n_keep, hipStream_t s) {
  for (int64_t k0 = 0; k0 < n_pairs; k0 += LAUNCH_CHUNK * 256) {
    const int64_t nk = std::min<int64_t>(LAUNCH_CHUNK * 256, n_pairs - k0);
    hipLaunchKernelGGL(cover_keep_count_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s, nk, bits + k0,
                       n_keep);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cover_keep(int64_t n_pairs, const int32_t* rep, const int32_t* mem, const uint8_t* bits,
                             const int16_t* shift, const int32_t* count, const double* score,
                             unsigned long long* slot, int32_t* k_rep, int32_t* k_mem, uint8_t* k_bits,
                             int16_t* k_shift, int32_t* k_count, double* k_score, hipStream_t s) {
  for (int64_t k0 = 0; k0 < n_pairs; k0 += LAUNCH_CHUNK * 256) {
    const int64_t nk = std::min<int64_t>(LAUNCH_CHUNK * 256, n_pairs - k0);
    hipLaunchKernelGGL(cover_keep_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s, nk, rep + k0,
                       mem + k0, bits + k0, reinterpret_cast<const uint64_t*>(shift + 4 * k0),
                       reinterpret_cast<const uint64_t*>(count + 2 * k0), score + 2 * k0, slot, k_rep, k_mem,
                       k_bits, reinterpret_cast<uint64_t*>(k_shift), reinterpret_cast<uint64_t*>(k_count), k_score);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cover_scatter(int64_t n_pairs, const int32_t* rep, const int32_t* mem, const uint8_t* bits,
                                const int64_t* row_ptr, unsigned long long* fill, uint64_t* keys, hipStream_t s) {
  // pair indices enter the keys as 2 k + d < 2^32, and one launch covers the list
  if (n_pairs >= (1ll << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cover_scatter_kernel, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, s, n_pairs, rep,
                     mem, bits, row_ptr, fill, keys);
  return hipGetLastError();
}

hipError_t launch_cover_sort(const int32_t* small_rows, int64_t n_small, const int32_t* large_rows, int64_t n_large,
                             const int64_t* row_ptr, uint64_t* keys, uint64_t* tmp, hipStream_t s) {
  for (int64_t r0 = 0; r0 < n_small; r0 += 4 * LAUNCH_CHUNK) {
    const int64_t nr = std::min<int64_t>(4 * LAUNCH_CHUNK, n_small - r0);
    hipLaunchKernelGGL(cover_sort_small_kernel, dim3((unsigned)((nr + 3) / 4)), dim3(256), 0, s, small_rows + r0, nr,
                       row_ptr, keys);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (int64_t r0 = 0; r0 < n_large; r0 += LAUNCH_CHUNK) {
    const int64_t nr = std::min<int64_t>(LAUNCH_CHUNK, n_large - r0);
    hipLaunchKernelGGL(cover_sort_large_kernel, dim3((unsigned)nr), dim3(256), 0, s, large_rows + r0, row_ptr, keys,
                       tmp);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cover_gather(int64_t nnz, const uint64_t* keys, const int16_t* shift, const int32_t* count,
                               const double* score, int32_t* col, int16_t* col_shift, int32_t* value,
                               double* col_score, hipStream_t s) {
  for (int64_t e0 = 0; e0 < nnz; e0 += LAUNCH_CHUNK * 256) {
    const int64_t ne = std::min<int64_t>(LAUNCH_CHUNK * 256, nnz - e0);
    hipLaunchKernelGGL(cover_gather_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, ne, keys + e0, shift,
                       count, score, col + e0, col_shift + 2 * e0, value + e0, col_score + e0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cover_dense(int64_t n, int64_t words, const int64_t* row_ptr, const int32_t* col,
                              unsigned long long* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cover_dense_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, words, row_ptr, col,
                     out);
  return hipGetLastError();
}

hipError_t launch_verify_cosine(const ClipsDev& cs, int64_t n, const int32_t* mem, const int32_t* rep,
                                const int16_t* shift, Threshold thr, unsigned long long* viol,
                                unsigned long long* first, hipStream_t s) {
  for (int64_t t0 = 0; t0 < n; t0 += 4 * LAUNCH_CHUNK) {
    const int64_t nt = std::min<int64_t>(4 * LAUNCH_CHUNK, n - t0);
    hipLaunchKernelGGL(verify_cosine_kernel, dim3((unsigned)((nt + 3) / 4)), dim3(256), 0, s, cs, n, t0, mem, rep,
                       shift, thr, viol, first);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ca
