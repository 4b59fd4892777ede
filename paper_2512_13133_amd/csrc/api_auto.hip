// CA_PATH_AUTO: one call over pairs of uneven raster sizes and windows.
//
// Pairs are partitioned, stably, into buckets by raster size and window class
// (the larger half-window of the pair).  Each bucket runs the path its entry
// in the context's tuning table names; a bucket met for the first time is
// tuned on a calibration sample of its own pairs: every applicable path is
// timed there, a path counts only if its results (bits, shifts, counts,
// scores) equal the FP64 path's bit for bit, and the fastest one is kept.
// Results go back to the caller's pair order.
#include <chrono>
#include <cstdio>
#include <string>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "host_internal.h"
#include "kernels.h"

namespace capriv {
ca_status fail_ctx(ca_ctx* ctx, ca_status st, const char* msg);
ca_status alloc_ctx(ca_ctx* ctx, void** p, size_t bytes);
void free_ctx(ca_ctx* ctx, void* p, size_t bytes);
ca_run_stats* stats_of(ca_ctx* ctx);
void set_stats(ca_ctx* ctx, const ca_run_stats& st);
const ca::ClipsDev& dev_of(const ca_clipset* cs);
bool has_fp32_of(const ca_clipset* cs);
bool has_image_of(const ca_clipset* cs);
std::map<int, TuneEntry>& tune_of(ca_ctx* ctx);
int64_t check_sample_of(const ca_ctx* ctx);
void set_check_sample(ca_ctx* ctx, int64_t v);
ca_status align_cosine_sets(ca_ctx* ctx, const ca_clipset* crs, const ca_clipset* cms, hipStream_t s,
                            ca::Threshold thr, int path, const ca::PairIO& io, bool checked, int direct_n,
                            int bucket_w);
}  // namespace capriv

using namespace ca;
using namespace capriv;

namespace {

// Window classes by the larger half-window of a pair: <= 4, <= 7, <= 15, 16,
// <= 23, <= 31, larger.  Raster codes: 64, 128, 256.
constexpr int N_WCLASS = 7;
constexpr int W_BOUND[N_WCLASS] = {4, 7, 15, 16, 23, 31, 1 << 20};
constexpr int N_KEYS = 3 * N_WCLASS;
constexpr int64_t TUNE_SAMPLE = 4096;
constexpr int64_t TUNE_MIN = 1024;  // a smaller bucket is repeated to this many pairs, so timings are throughputs
// Pairs the admitted paths are timed on (a contiguous run of the bucket, so
// that candidate lists keep their representatives together): enough tiles for
// the persistent batched kernels to fill the device, fewer for larger rasters.
constexpr int64_t tune_time_pairs(int N) { return N <= 64 ? 32768 : (N <= 128 ? 16384 : 8192); }

__host__ __device__ inline int wclass_of(int w) {
  int c = 0;
  while (c < N_WCLASS - 1 && w > W_BOUND[c]) ++c;
  return c;
}
__host__ __device__ inline int ncode_of(int N) { return N <= 64 ? 0 : (N <= 128 ? 1 : 2); }

#define HIP_TRY(ctx, expr)                                                     \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) return fail_ctx((ctx), CA_EDEVICE, hipGetErrorString(e_)); \
  } while (0)

// Bucket key of every pair and the bucket sizes: a histogram per workgroup in
// LDS, added to the global one with one atomic per bucket and workgroup (one
// global atomic per pair serialised on a few counters).
__global__ void bucket_keys_kernel(ClipsDev cs, int64_t n, const int32_t* __restrict__ rep,
                                   const int32_t* __restrict__ mem, uint8_t* __restrict__ keys,
                                   int32_t* __restrict__ idx, unsigned* __restrict__ hist) {
  __shared__ unsigned s_hist[N_KEYS];
  for (int t = threadIdx.x; t < N_KEYS; t += blockDim.x) s_hist[t] = 0u;
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    const int i = mem[k], j = rep[k];
    const int key = ncode_of(cs.N[i]) * N_WCLASS + wclass_of(max((int)cs.w[i], (int)cs.w[j]));
    keys[k] = (uint8_t)key;
    idx[k] = (int32_t)k;
    atomicAdd(&s_hist[key], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < N_KEYS; t += blockDim.x)
    if (s_hist[t]) atomicAdd(hist + t, s_hist[t]);
}

__global__ void gather_pairs_kernel(int64_t n, const int32_t* __restrict__ idx, const int32_t* __restrict__ rep,
                                    const int32_t* __restrict__ mem, int32_t* __restrict__ rep_b,
                                    int32_t* __restrict__ mem_b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  rep_b[t] = rep[idx[t]];
  mem_b[t] = mem[idx[t]];
}

// Calibration pairs: the bucket's first pairs, repeated cyclically when the
// bucket is shorter than the sample.
__global__ void sample_pairs_kernel(int64_t m, int64_t nb, const int32_t* __restrict__ rep,
                                   const int32_t* __restrict__ mem, int32_t* __restrict__ rep_s,
                                   int32_t* __restrict__ mem_s) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  rep_s[t] = rep[t % nb];
  mem_s[t] = mem[t % nb];
}

// dst at the original position idx[t] of bucket-ordered result t
__global__ void scatter_results_kernel(int64_t n, const int32_t* __restrict__ idx, PairIO src, PairIO dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t k = idx[t];
  dst.bits[k] = src.bits[t];
  dst.flags[k] = src.flags[t];
  for (int e = 0; e < 4; ++e) dst.shift[4 * k + e] = src.shift[4 * t + e];
  for (int e = 0; e < 2; ++e) {
    dst.count[2 * k + e] = src.count[2 * t + e];
    dst.score[2 * k + e] = src.score[2 * t + e];
  }
}

// Number of pairs whose bits, shifts, counts or scores differ.
__global__ void compare_results_kernel(int64_t n, PairIO a, PairIO b, unsigned* __restrict__ bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  bool same = a.bits[t] == b.bits[t];
  for (int e = 0; e < 4; ++e) same = same && a.shift[4 * t + e] == b.shift[4 * t + e];
  for (int e = 0; e < 2; ++e) same = same && a.count[2 * t + e] == b.count[2 * t + e] && a.score[2 * t + e] == b.score[2 * t + e];
  if (!same) atomicAdd(bad, 1u);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Result arrays of m pairs carved from one allocation.
size_t aup(size_t x) { return (x + 255) & ~(size_t)255; }
size_t result_bytes(int64_t m) {
  return aup(m) + aup(8 * (size_t)m) + aup(8 * (size_t)m) + aup(16 * (size_t)m) + aup(4 * (size_t)m);
}
PairIO result_view(char* p, int64_t m, const int32_t* rep, const int32_t* mem) {
  PairIO io;
  io.n_pairs = m;
  io.rep = rep;
  io.mem = mem;
  io.bits = (uint8_t*)p; p += aup(m);
  io.shift = (int16_t*)p; p += aup(8 * (size_t)m);
  io.count = (int32_t*)p; p += aup(8 * (size_t)m);
  io.score = (double*)p; p += aup(16 * (size_t)m);
  io.flags = (uint32_t*)p;
  return io;
}

double wall_us() {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Tune one bucket on `io` (its first pairs): time each applicable path and keep
// the fastest whose results equal the FP64 path's.
// `timing`: a run of the bucket's own pairs (outputs in the bucket's result
// slices, which the bucket's launch overwrites) on which the admitted paths
// other than FP64 are timed again when it is longer than the sample.
ca_status tune_bucket(ca_ctx* ctx, const ca_clipset* cs, hipStream_t s, Threshold thr, int key, const PairIO& io,
                      const PairIO& timing, char* ref_mem, char* tmp_mem, unsigned* bad, TuneEntry* out) {
  const int N = 64 << (key / N_WCLASS);
  const int wc = key % N_WCLASS;
  const ca_run_stats saved = *stats_of(ctx);
  // the timed runs compare paths on equal terms: no FP64 check of decided pairs
  const int64_t check = check_sample_of(ctx);
  set_check_sample(ctx, 0);
  struct Restore {
    ca_ctx* c;
    int64_t v;
    ~Restore() { set_check_sample(c, v); }
  } restore{ctx, check};
  const int64_t m = io.n_pairs;
  PairIO ref = result_view(ref_mem, m, io.rep, io.mem);
  PairIO tmp = result_view(tmp_mem, m, io.rep, io.mem);
  TuneEntry e;
  e.sample = m;
  auto run = [&](int path, const PairIO& o, double* us) -> ca_status {
    ca_status st = align_cosine_sets(ctx, cs, cs, s, thr, path, o, true, N, W_BOUND[wc]);  // warm
    if (st) return st;
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const double t0 = wall_us();
    st = align_cosine_sets(ctx, cs, cs, s, thr, path, o, true, N, W_BOUND[wc]);
    if (st) return st;
    HIP_TRY(ctx, hipStreamSynchronize(s));
    *us = (wall_us() - t0) * 1000.0 / (double)o.n_pairs;
    return CA_OK;
  };
  double us = 0.0;
  ca_status st = run(CA_PATH_FP64, ref, &us);
  if (st) return st;
  e.us_per_kpair[CA_PATH_FP64] = us;
  e.path = CA_PATH_FP64;
  double best = us;
  const bool mixed_ok = true;  // the batched MFMA kernels cover every raster size and window class
  const bool direct_ok = W_BOUND[wc] <= 7 && has_image_of(cs);
  for (int path : {CA_PATH_MIXED, CA_PATH_DIRECT, CA_PATH_FP32}) {
    if (path == CA_PATH_MIXED && !mixed_ok) continue;
    if (path == CA_PATH_DIRECT && !direct_ok) continue;
    if (path == CA_PATH_FP32 && !has_fp32_of(cs)) continue;
    st = run(path, tmp, &us);
    if (st) return st;
    HIP_TRY(ctx, hipMemsetAsync(bad, 0, sizeof(unsigned), s));
    hipLaunchKernelGGL(compare_results_kernel, dim3(blocks_for(m)), dim3(256), 0, s, m, ref, tmp, bad);
    HIP_TRY(ctx, hipGetLastError());
    unsigned hbad = 1;
    HIP_TRY(ctx, hipMemcpyAsync(&hbad, bad, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (hbad != 0) continue;  // not valid on this bucket: never chosen
    if (timing.n_pairs > m) {
      st = run(path, timing, &us);
      if (st) return st;
    }
    e.us_per_kpair[path] = us;
    if (us < best) {
      best = us;
      e.path = path;
    }
  }
  set_stats(ctx, saved);
  *out = e;
  return CA_OK;
}

const char* path_name(int p) {
  switch (p) {
    case CA_PATH_MIXED: return "mixed";
    case CA_PATH_FP32: return "fp32";
    case CA_PATH_FP64: return "fp64";
    case CA_PATH_DIRECT: return "direct";
    default: return "none";
  }
}

}  // namespace

namespace capriv {

ca_status align_auto(ca_ctx* ctx, const ca_clipset* cs, hipStream_t s, Threshold thr, const PairIO& io) {
  const int64_t n = io.n_pairs;
  const ClipsDev& d = dev_of(cs);
  // device work space: keys (2), indices (2), histogram, pairs in bucket order,
  // results in bucket order, sort scratch, calibration results (2)
  size_t sort_bytes = 0;
  {
    const hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (const uint8_t*)nullptr,
                                                            (uint8_t*)nullptr, (const int32_t*)nullptr,
                                                            (int32_t*)nullptr, (int)n, 0, 5, s);
    if (e != hipSuccess) return fail_ctx(ctx, CA_EDEVICE, hipGetErrorString(e));
  }
  const size_t b_keys = aup(n), b_idx = aup(4 * (size_t)n), b_hist = 256, b_res = result_bytes(n),
               b_sort = aup(sort_bytes), b_cal = result_bytes(TUNE_SAMPLE), b_spair = aup(4 * (size_t)TUNE_SAMPLE);
  const size_t total = 2 * b_keys + 2 * b_idx + b_hist + 2 * b_idx + b_res + b_sort + 2 * b_cal + 2 * b_spair;
  void* mem;
  ca_status st = alloc_ctx(ctx, &mem, total);
  if (st) return st;
  char* p = (char*)mem;
  uint8_t* keys = (uint8_t*)p; p += b_keys;
  uint8_t* keys_s = (uint8_t*)p; p += b_keys;
  int32_t* idx = (int32_t*)p; p += b_idx;
  int32_t* idx_s = (int32_t*)p; p += b_idx;
  unsigned* hist = (unsigned*)p; p += b_hist;
  int32_t* rep_b = (int32_t*)p; p += b_idx;
  int32_t* mem_b = (int32_t*)p; p += b_idx;
  char* res = p; p += b_res;
  void* sort_tmp = p; p += b_sort;
  char* cal_ref = p; p += b_cal;
  char* cal_tmp = p; p += b_cal;
  int32_t* rep_s = (int32_t*)p; p += b_spair;
  int32_t* mem_s = (int32_t*)p;
  auto done = [&](ca_status r) {
    (void)hipStreamSynchronize(s);
    free_ctx(ctx, mem, total);
    return r;
  };
#define AUTO_TRY(expr)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return done(fail_ctx(ctx, CA_EDEVICE, hipGetErrorString(e_))); \
  } while (0)
  AUTO_TRY(hipMemsetAsync(hist, 0, b_hist, s));
  hipLaunchKernelGGL(bucket_keys_kernel, dim3(blocks_for(n)), dim3(256), 0, s, d, n, io.rep, io.mem, keys, idx, hist);
  AUTO_TRY(hipGetLastError());
  size_t sb = sort_bytes;
  AUTO_TRY(hipcub::DeviceRadixSort::SortPairs(sort_tmp, sb, keys, keys_s, idx, idx_s, (int)n, 0, 5, s));
  hipLaunchKernelGGL(gather_pairs_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, idx_s, io.rep, io.mem, rep_b, mem_b);
  AUTO_TRY(hipGetLastError());
  unsigned h[N_KEYS];
  AUTO_TRY(hipMemcpyAsync(h, hist, sizeof(h), hipMemcpyDeviceToHost, s));
  AUTO_TRY(hipStreamSynchronize(s));
  PairIO out = result_view(res, n, rep_b, mem_b);
  auto& table = tune_of(ctx);
  int64_t off = 0;
  for (int key = 0; key < N_KEYS; ++key) {
    const int64_t m = h[key];
    if (m == 0) continue;
    PairIO bio = out;
    bio.n_pairs = m;
    bio.rep = rep_b + off;
    bio.mem = mem_b + off;
    bio.bits = out.bits + off;
    bio.shift = out.shift + 4 * off;
    bio.count = out.count + 2 * off;
    bio.score = out.score + 2 * off;
    bio.flags = out.flags + off;
    auto it = table.find(key);
    if (it == table.end()) {
      PairIO sample = bio;
      sample.n_pairs = std::min<int64_t>(std::max<int64_t>(m, TUNE_MIN), TUNE_SAMPLE);
      hipLaunchKernelGGL(sample_pairs_kernel, dim3(blocks_for(sample.n_pairs)), dim3(256), 0, s, sample.n_pairs, m,
                         bio.rep, bio.mem, rep_s, mem_s);
      AUTO_TRY(hipGetLastError());
      sample.rep = rep_s;
      sample.mem = mem_s;
      PairIO timing = bio;
      timing.n_pairs = std::min<int64_t>(m, tune_time_pairs(64 << (key / N_WCLASS)));
      TuneEntry e;
      st = tune_bucket(ctx, cs, s, thr, key, sample, timing, cal_ref, cal_tmp, hist + 32, &e);
      if (st) return done(st);
      it = table.emplace(key, e).first;
    }
    st = align_cosine_sets(ctx, cs, cs, s, thr, it->second.path, bio, true, 64 << (key / N_WCLASS),
                           W_BOUND[key % N_WCLASS]);
    if (st) return done(st);
    off += m;
  }
  hipLaunchKernelGGL(scatter_results_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, idx_s, out, io);
  AUTO_TRY(hipGetLastError());
#undef AUTO_TRY
  return done(CA_OK);
}

}  // namespace capriv

extern "C" ca_status ca_autotune_report(ca_ctx* ctx, char* buf, int64_t cap, int64_t* len) {
  if (!ctx || !len) return CA_EINVAL;
  std::string r;
  char line[256];
  for (const auto& kv : tune_of(ctx)) {
    const int key = kv.first;
    const TuneEntry& e = kv.second;
    std::snprintf(line, sizeof line,
                  "N=%d w<=%d path=%s us_per_kpair mixed=%.1f direct=%.1f fp32=%.1f fp64=%.1f sample=%lld\n",
                  64 << (key / N_WCLASS), W_BOUND[key % N_WCLASS], path_name(e.path), e.us_per_kpair[CA_PATH_MIXED],
                  e.us_per_kpair[CA_PATH_DIRECT], e.us_per_kpair[CA_PATH_FP32], e.us_per_kpair[CA_PATH_FP64],
                  (long long)e.sample);
    r += line;
  }
  *len = (int64_t)r.size();
  if (buf && cap > 0) {
    const int64_t c = std::min<int64_t>(cap - 1, (int64_t)r.size());
    std::memcpy(buf, r.data(), (size_t)c);
    buf[c] = '\0';
    if (c < (int64_t)r.size()) return CA_ETRUNC;
  }
  return CA_OK;
}

extern "C" ca_status ca_autotune_save(ca_ctx* ctx, const char* path) {
  if (!ctx || !path) return CA_EINVAL;
  FILE* f = std::fopen(path, "w");
  if (!f) return fail_ctx(ctx, CA_EINVAL, "cannot open the tuning file for writing");
  std::fprintf(f, "clipalign-autotune 2\n");
  for (const auto& kv : tune_of(ctx)) {
    const TuneEntry& e = kv.second;
    std::fprintf(f, "%d %d %.17g %.17g %.17g %.17g %.17g %lld\n", kv.first, e.path, e.us_per_kpair[0],
                 e.us_per_kpair[1], e.us_per_kpair[2], e.us_per_kpair[3], e.us_per_kpair[4], (long long)e.sample);
  }
  const bool ok = std::fclose(f) == 0;
  return ok ? CA_OK : fail_ctx(ctx, CA_EINVAL, "cannot write the tuning file");
}

extern "C" ca_status ca_autotune_load(ca_ctx* ctx, const char* path) {
  if (!ctx || !path) return CA_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return fail_ctx(ctx, CA_EINVAL, "cannot open the tuning file");
  char head[64] = {0};
  int version = 0;
  if (std::fscanf(f, "%63s %d", head, &version) != 2 || std::string(head) != "clipalign-autotune" || version != 2) {
    std::fclose(f);
    return fail_ctx(ctx, CA_EINVAL, "not a tuning file of this library");
  }
  std::map<int, TuneEntry> loaded;
  int key, chosen;
  double t0, t1, t2, t3, t4;
  long long sample;
  while (std::fscanf(f, "%d %d %lf %lf %lf %lf %lf %lld", &key, &chosen, &t0, &t1, &t2, &t3, &t4, &sample) == 8) {
    if (key < 0 || key >= N_KEYS || chosen < CA_PATH_MIXED || chosen > CA_PATH_DIRECT || chosen == CA_PATH_AUTO) {
      std::fclose(f);
      return fail_ctx(ctx, CA_EINVAL, "bad entry in the tuning file");
    }
    TuneEntry e;
    e.path = chosen;
    e.us_per_kpair[0] = t0; e.us_per_kpair[1] = t1; e.us_per_kpair[2] = t2; e.us_per_kpair[3] = t3;
    e.us_per_kpair[4] = t4;
    e.sample = sample;
    loaded[key] = e;
  }
  std::fclose(f);
  tune_of(ctx) = loaded;
  return CA_OK;
}

extern "C" ca_status ca_autotune_clear(ca_ctx* ctx) {
  if (!ctx) return CA_EINVAL;
  tune_of(ctx).clear();
  return CA_OK;
}
