// Candidate generation (ca_prune) and the clustering driver (ca_cluster):
// surprisal lazy-greedy set cover (paper Sec. 3.3, Eqs. 7-9) inside the
// coarse-to-fine closed loop (Sec. 3.1), on the host over the device results.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

#include "host_internal.h"
#include "kernels.h"

// Context and clip-set internals shared with api.hip.
struct ca_ctx;
struct ca_clipset;
namespace capriv {
ca_status fail_ctx(ca_ctx* ctx, ca_status st, const char* msg);
ca_status scratch_ctx(ca_ctx* ctx, size_t bytes, void** out);
ca_status alloc_ctx(ca_ctx* ctx, void** p, size_t bytes);
void free_ctx(ca_ctx* ctx, void* p, size_t bytes);
int device_of(const ca_ctx* ctx);
ca_run_stats* stats_of(ca_ctx* ctx);
const ca::ClipsDev& dev_of(const ca_clipset* cs);
ca_ctx* ctx_of(const ca_clipset* cs);
const std::vector<int16_t>& hN_of(const ca_clipset* cs);
const std::vector<int32_t>& hnpix_of(const ca_clipset* cs);
int64_t n_of(const ca_clipset* cs);
int maxN_of(const ca_clipset* cs);
bool mixed_ok_of(const ca_clipset* cs);
uint64_t gen_of(const ca_clipset* cs);
PruneCache* prune_cache_of(ca_ctx* ctx);
}  // namespace capriv

using namespace ca;
using namespace capriv;

namespace {

#define HIP_TRY(ctx, expr)                                                     \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) return fail_ctx((ctx), CA_EDEVICE, hipGetErrorString(e_)); \
  } while (0)

size_t aup(size_t x) { return (x + 255) & ~(size_t)255; }

// Anchor order and partner ranges for a constraint (host side, O(n log n)).
void build_ranges(const ca_clipset* cs, const ca_constraint* con, std::vector<int32_t>& order,
                  std::vector<int32_t>& hi, int64_t& screened) {
  const int64_t n = n_of(cs);
  const auto& hN = hN_of(cs);
  const auto& np = hnpix_of(cs);
  order.clear();
  hi.clear();
  screened = 0;
  for (int N : {64, 128, 256}) {
    std::vector<int32_t> ids;
    for (int64_t i = 0; i < n; ++i)
      if (hN[i] == N) ids.push_back((int32_t)i);
    if (ids.empty()) continue;
    const int64_t base = (int64_t)order.size();
    const int64_t m = (int64_t)ids.size();
    screened += m * (m - 1) / 2;
    if (con->kind == CA_COSINE) {
      // (n, id) order by a stable counting sort on n <= N^2 (ids ascend already)
      std::vector<int32_t> start((size_t)N * N + 2, 0);
      for (int32_t i : ids) ++start[(size_t)np[i] + 1];
      for (size_t v = 1; v < start.size(); ++v) start[v] += start[v - 1];
      std::vector<int32_t> sorted(ids.size());
      for (int32_t i : ids) sorted[start[(size_t)np[i]]++] = i;
      ids.swap(sorted);
      const unsigned __int128 p2 = (unsigned __int128)(con->thr_num * con->thr_num);
      const unsigned __int128 q2 = (unsigned __int128)(con->thr_den * con->thr_den);
      int64_t e = 0;
      for (int64_t a = 0; a < m; ++a) {
        // partners b > a with n_a q^2 > p^2 n_b (n_a <= n_b); monotone in b
        e = std::max(e, a + 1);
        const unsigned __int128 lhs = (unsigned __int128)np[ids[a]] * q2;
        while (e < m && lhs > p2 * (unsigned __int128)np[ids[e]]) ++e;
        hi.push_back((int32_t)(base + (np[ids[a]] > 0 ? e : a + 1)));
      }
    } else {
      for (int64_t a = 0; a < m; ++a) hi.push_back((int32_t)(base + m));
    }
    order.insert(order.end(), ids.begin(), ids.end());
  }
}

}  // namespace

// Bounds pass with a survivor bitmask (cosine on 128 x 128 clips with
// half-windows <= 16, and the edge track): the pass runs once per (clip set,
// constraint); its bitmask and counts are cached on the context, so sizing and
// writing calls share it.  Edge ranges start on 64-bit words (the edge pass
// stores whole chunk words); edge pairs are written as (smaller, larger) id.
static ca_status prune_cached_device(ca_ctx* ctx, hipStream_t s, const ca_clipset* cs, const ca_constraint* con,
                                     int64_t cap, int32_t* rep, int32_t* mem, int64_t* n_out) {
  const bool edge = con->kind == CA_EDGE;
  PruneCache* pc = prune_cache_of(ctx);
  const bool hit = pc->gen == gen_of(cs) && pc->kind == con->kind && pc->p == con->thr_num && pc->q == con->thr_den;
  // a hit (the writing call after a sizing call) reuses the device copies of
  // the anchor order, ranges and bitmask
  int64_t na = pc->na;
  char* base;
  if (!hit) {
    std::vector<int32_t> order, hi;
    int64_t screened = 0;
    build_ranges(cs, con, order, hi, screened);
    na = (int64_t)order.size();
    std::vector<int64_t> range_off(na);
    int64_t bits = 0;
    for (int64_t a = 0; a < na; ++a) {
      range_off[a] = bits;
      const int64_t len = hi[a] - a - 1;
      bits += edge ? (len + 63) / 64 * 64 : len;
    }
    const size_t b_ord = aup(4 * (size_t)na), b_rng = aup(8 * (size_t)na);
    const size_t b_mask = aup(8 * (size_t)(bits / 64 + 1));
    // transposed sliding sums (rows, columns), or box sizes and polygon counts for the edge track
    const size_t b_soa = aup(4 * 64 * (size_t)na);
    const size_t need = 2 * b_ord + 2 * b_rng + b_mask + 2 * b_soa;
    if (pc->bytes < need) {
      free_ctx(ctx, pc->dev, pc->bytes);
      pc->dev = nullptr;
      pc->bytes = 0;
      pc->gen = 0;
      ca_status st = alloc_ctx(ctx, &pc->dev, need);
      if (st) return st;
      pc->bytes = need;
    }
    base = (char*)pc->dev;
    int32_t* d_order = (int32_t*)base;
    int32_t* d_hi = (int32_t*)(base + b_ord);
    int64_t* d_roff = (int64_t*)(base + 2 * b_ord);
    int64_t* d_cnt = (int64_t*)(base + 2 * b_ord + b_rng);
    uint32_t* d_mask = (uint32_t*)(base + 2 * b_ord + 2 * b_rng);
    HIP_TRY(ctx, hipMemcpyAsync(d_order, order.data(), 4 * na, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(d_hi, hi.data(), 4 * na, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(d_roff, range_off.data(), 8 * na, hipMemcpyHostToDevice, s));
    PruneArgs pa{d_order, d_hi, na, d_cnt, nullptr, nullptr, nullptr};
    if (edge) {
      uint32_t* d_wh = (uint32_t*)(base + 2 * b_ord + 2 * b_rng + b_mask);
      int32_t* d_np = (int32_t*)(base + 2 * b_ord + 2 * b_rng + b_mask + b_soa);
      HIP_TRY(ctx, launch_edge_soa(dev_of(cs), d_order, na, d_wh, d_np, s));
      pa.soa_wh = d_wh;
      pa.soa_np = d_np;
      pa.soa_n = na;
      HIP_TRY(ctx, launch_edge_prune(dev_of(cs), pa, Threshold{con->thr_num, con->thr_den}, d_roff,
                                     (unsigned long long*)d_mask, s));
    } else {
      HIP_TRY(ctx, hipMemsetAsync(d_mask, 0, b_mask, s));
      uint32_t* d_soa = (uint32_t*)(base + 2 * b_ord + 2 * b_rng + b_mask);
      HIP_TRY(ctx, launch_prune128_soa(dev_of(cs), d_order, na, d_soa, d_soa + b_soa / 4, s));
      pa.soa_row = d_soa;
      pa.soa_col = d_soa + b_soa / 4;
      pa.soa_n = na;
      HIP_TRY(ctx, launch_prune128(dev_of(cs), dev_of(cs), pa, Threshold{con->thr_num, con->thr_den}, d_roff, d_mask,
                                   false, s));
    }
    pc->counts.assign(na, 0);
    HIP_TRY(ctx, hipMemcpyAsync(pc->counts.data(), d_cnt, 8 * na, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    pc->total = 0;
    for (int64_t a = 0; a < na; ++a) pc->total += pc->counts[a];
    pc->gen = gen_of(cs);
    pc->kind = con->kind;
    pc->p = con->thr_num;
    pc->q = con->thr_den;
    pc->na = na;
    pc->b_mask = b_mask;
    stats_of(ctx)->pairs_screened += screened;
    stats_of(ctx)->pairs_survived += pc->total;
  }
  const size_t b_ord = aup(4 * (size_t)na), b_rng = aup(8 * (size_t)na);
  base = (char*)pc->dev;
  *n_out = pc->total;
  if (!rep) return CA_OK;
  if (pc->total > cap) return fail_ctx(ctx, CA_ETRUNC, "candidate buffer too small");
  std::vector<int64_t> off(na);
  int64_t acc = 0;
  for (int64_t a = 0; a < na; ++a) {
    off[a] = acc;
    acc += pc->counts[a];
  }
  int64_t* d_off = (int64_t*)(base + 2 * b_ord + b_rng);  // reuses the count slots
  HIP_TRY(ctx, hipMemcpyAsync(d_off, off.data(), 8 * na, hipMemcpyHostToDevice, s));
  PruneArgs pa{(int32_t*)base, (int32_t*)(base + b_ord), na, nullptr, d_off, rep, mem};
  pa.order_ids = edge ? 1 : 0;
  HIP_TRY(ctx, launch_prune128(dev_of(cs), dev_of(cs), pa, Threshold{con->thr_num, con->thr_den},
                               (int64_t*)(base + 2 * b_ord), (uint32_t*)(base + 2 * b_ord + 2 * b_rng), true, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return CA_OK;
}

// Device candidate generation into caller buffers (or sizing only when rep is null).
static ca_status prune_device(ca_ctx* ctx, hipStream_t s, const ca_clipset* cs, const ca_constraint* con,
                              int64_t cap, int32_t* rep, int32_t* mem, int64_t* n_out) {
  if (con->kind == CA_EDGE || mixed_ok_of(cs)) return prune_cached_device(ctx, s, cs, con, cap, rep, mem, n_out);
  std::vector<int32_t> order, hi;
  int64_t screened = 0;
  build_ranges(cs, con, order, hi, screened);
  const int64_t na = (int64_t)order.size();
  void* sc;
  const size_t b_ord = aup(4 * (size_t)na), b_hi = aup(4 * (size_t)na), b_cnt = aup(8 * (size_t)na);
  ca_status st = scratch_ctx(ctx, b_ord + b_hi + 2 * b_cnt, &sc);
  if (st) return st;
  char* base = (char*)sc;
  int32_t* d_order = (int32_t*)base;
  int32_t* d_hi = (int32_t*)(base + b_ord);
  int64_t* d_cnt = (int64_t*)(base + b_ord + b_hi);
  int64_t* d_off = (int64_t*)(base + b_ord + b_hi + b_cnt);
  HIP_TRY(ctx, hipMemcpyAsync(d_order, order.data(), 4 * na, hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(d_hi, hi.data(), 4 * na, hipMemcpyHostToDevice, s));
  PruneArgs pa{d_order, d_hi, na, d_cnt, nullptr, nullptr, nullptr};
  const Threshold thr{con->thr_num, con->thr_den};
  HIP_TRY(ctx, launch_cosine_prune(dev_of(cs), pa, thr, maxN_of(cs), s));
  std::vector<int64_t> cnt(na), off(na);
  HIP_TRY(ctx, hipMemcpyAsync(cnt.data(), d_cnt, 8 * na, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  int64_t total = 0;
  for (int64_t a = 0; a < na; ++a) {
    off[a] = total;
    total += cnt[a];
  }
  *n_out = total;
  stats_of(ctx)->pairs_screened += screened;
  stats_of(ctx)->pairs_survived += total;
  if (!rep) return CA_OK;
  if (total > cap) return fail_ctx(ctx, CA_ETRUNC, "candidate buffer too small");
  HIP_TRY(ctx, hipMemcpyAsync(d_off, off.data(), 8 * na, hipMemcpyHostToDevice, s));
  pa.offs = d_off;
  pa.out_rep = rep;
  pa.out_mem = mem;
  HIP_TRY(ctx, launch_cosine_prune(dev_of(cs), pa, thr, maxN_of(cs), s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return CA_OK;
}

extern "C" ca_status ca_prune(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                              int64_t cap, int32_t* rep, int32_t* mem, int64_t* n_out) {
  if (!ctx) return CA_EINVAL;
  if (!cs || ctx_of(cs) != ctx || !n_out) return fail_ctx(ctx, CA_EINVAL, "bad arguments");
  if (!con || (con->kind != CA_COSINE && con->kind != CA_EDGE) || con->thr_den <= 0 ||
      con->thr_num < 0 || (con->kind == CA_COSINE && con->thr_num > con->thr_den))
    return fail_ctx(ctx, CA_EINVAL, "bad constraint");
  if (cap < 0 || (cap > 0 && (!rep || !mem))) return fail_ctx(ctx, CA_EINVAL, "bad output buffers");
  HIP_TRY(ctx, hipSetDevice(device_of(ctx)));
  return prune_device(ctx, (hipStream_t)stream, cs, con, cap, cap > 0 ? rep : nullptr, mem, n_out);
}

// ------------------------------------------------------------------ set cover

namespace {

struct Dir {
  int32_t r, m;  // representative covers member
  int32_t val;   // cosine: overlap count; edge: residual E
  bool ok;       // edge: correspondence found and re-checked
  int16_t sy, sx;
};

struct Cover {
  int64_t n;
  int kind;
  std::vector<Dir> dirs;
  const std::vector<int32_t>* npix;
  bool bit(const Dir& d, int64_t p, int64_t q) const {
    if (kind == CA_COSINE) {
      const int64_t nm = (*npix)[d.m], nr = (*npix)[d.r];
      if (nm <= 0 || nr <= 0) return false;
      const unsigned __int128 lhs = (unsigned __int128)((uint64_t)d.val * (uint64_t)d.val) *
                                    (unsigned __int128)((uint64_t)q * (uint64_t)q);
      const unsigned __int128 rhs = (unsigned __int128)((uint64_t)p * (uint64_t)p) *
                                    (unsigned __int128)((uint64_t)nm * (uint64_t)nr);
      return lhs > rhs;
    }
    return d.ok && d.val >= 0 && d.val <= p;
  }
};

// Surprisal lazy greedy on `pool` (ascending ids) with threshold (p, q).
// Returns reps in selection order and fills assign[i] for pool members.
std::vector<int32_t> lazy_greedy(const Cover& cv, const std::vector<int32_t>& pool, int64_t p, int64_t q,
                                 std::vector<int32_t>& assign) {
  const int64_t n = cv.n;
  std::vector<int32_t> pos(n, -1);
  for (size_t a = 0; a < pool.size(); ++a) pos[pool[a]] = (int32_t)a;
  const size_t P = pool.size();
  std::vector<std::vector<int32_t>> out(P);
  std::vector<int64_t> indeg(P, 0);
  for (const Dir& d : cv.dirs) {
    const int32_t a = pos[d.r], b = pos[d.m];
    if (a < 0 || b < 0 || a == b) continue;
    if (!cv.bit(d, p, q)) continue;
    out[a].push_back(b);
    indeg[b]++;
  }
  for (auto& o : out) {
    std::sort(o.begin(), o.end());
    o.erase(std::unique(o.begin(), o.end()), o.end());
  }
  // in-degree counts distinct covering nodes
  std::fill(indeg.begin(), indeg.end(), 0);
  for (size_t a = 0; a < P; ++a)
    for (int32_t b : out[a]) indeg[b]++;
  std::vector<double> S(P);
  for (size_t a = 0; a < P; ++a) S[a] = 1.0 / (double)(1 + indeg[a]);
  std::vector<char> unc(P, 1);
  auto score = [&](size_t j) {
    double t = S[j];
    for (int32_t k : out[j])
      if (unc[k]) t = t + S[k];
    return t;
  };
  struct E {
    double s;
    int32_t j;
  };
  auto less = [](const E& a, const E& b) {  // max-heap on (score, -j)
    if (a.s != b.s) return a.s < b.s;
    return a.j > b.j;
  };
  std::priority_queue<E, std::vector<E>, decltype(less)> heap(less);
  for (size_t j = 0; j < P; ++j) heap.push(E{score(j), (int32_t)j});
  std::vector<int32_t> reps;
  while (!heap.empty()) {
    E top = heap.top();
    heap.pop();
    if (!unc[top.j]) continue;
    const double sc = score(top.j);
    if (!heap.empty()) {
      const E& t2 = heap.top();
      if (sc < t2.s || (sc == t2.s && top.j > t2.j)) {
        heap.push(E{sc, top.j});
        continue;
      }
    }
    reps.push_back(pool[top.j]);
    unc[top.j] = 0;
    assign[pool[top.j]] = pool[top.j];
    for (int32_t k : out[top.j])
      if (unc[k]) {
        unc[k] = 0;
        assign[pool[k]] = pool[top.j];
      }
  }
  return reps;
}

}  // namespace

static ca_status cluster_impl(ca_ctx* ctx, hipStream_t s, const ca_clipset* cs, const ca_constraint* con,
                              int32_t path, int32_t K, int32_t* rep_of, int16_t* center_shift,
                              int64_t* n_clusters) {
  const int64_t n = n_of(cs);
  // thresholds t = 1..K (exact rationals), loosest first
  std::vector<std::pair<int64_t, int64_t>> sched;
  for (int t = 1; t <= K; ++t) {
    if (con->kind == CA_COSINE) {
      // T - (K - t) / (50 (K - 1))
      int64_t p = con->thr_num, q = con->thr_den;
      if (K > 1) {
        const int64_t num = p * 50 * (K - 1) - (int64_t)(K - t) * q;
        const int64_t den = q * 50 * (K - 1);
        const int64_t g = std::gcd(std::max<int64_t>(num, 0), den);
        p = std::max<int64_t>(num, 0) / (g ? g : 1);
        q = den / (g ? g : 1);
      }
      sched.emplace_back(p, q);
    } else {
      sched.emplace_back(con->thr_num + (K - t), 1);
    }
  }
  ca_constraint loose = *con;
  loose.thr_num = sched[0].first;
  loose.thr_den = sched[0].second;
  int64_t np = 0;
  ca_status st = prune_device(ctx, s, cs, &loose, 0, nullptr, nullptr, &np);
  if (st) return st;
  // device buffers for the candidate list and alignment outputs
  const size_t b4 = aup(4 * (size_t)std::max<int64_t>(np, 1));
  const size_t bytes = 2 * b4 + aup((size_t)np + 1) + aup(8 * (size_t)np + 8) + aup(8 * (size_t)np + 8) +
                       aup(16 * (size_t)np + 16) + b4;
  void* buf = nullptr;
  st = alloc_ctx(ctx, &buf, bytes);
  if (st) return st;
  struct Guard {
    ca_ctx* c; void* p; size_t b;
    ~Guard() { free_ctx(c, p, b); }
  } guard{ctx, buf, bytes};
  char* b = (char*)buf;
  int32_t* d_rep = (int32_t*)b; b += b4;
  int32_t* d_mem = (int32_t*)b; b += b4;
  uint8_t* d_bits = (uint8_t*)b; b += aup((size_t)np + 1);
  int16_t* d_shift = (int16_t*)b; b += aup(8 * (size_t)np + 8);
  int32_t* d_count = (int32_t*)b; b += aup(8 * (size_t)np + 8);
  double* d_score = (double*)b; b += aup(16 * (size_t)np + 16);
  uint32_t* d_flags = (uint32_t*)b;
  int64_t got = 0;
  if (np > 0) {
    st = prune_device(ctx, s, cs, &loose, np, d_rep, d_mem, &got);
    if (st) return st;
    st = ca_align_pairs(ctx, s, cs, &loose, path, np, d_rep, d_mem, d_bits, d_shift, d_count, d_score, d_flags);
    if (st) return st;
  }
  std::vector<int32_t> hrep(np), hmem(np), hcount(2 * np);
  std::vector<int16_t> hshift(4 * np);
  std::vector<uint32_t> hflags(np);
  if (np > 0) {
    HIP_TRY(ctx, hipMemcpyAsync(hrep.data(), d_rep, 4 * np, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(hmem.data(), d_mem, 4 * np, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(hcount.data(), d_count, 8 * np, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(hshift.data(), d_shift, 8 * np, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(hflags.data(), d_flags, 4 * np, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
  }
  Cover cv;
  cv.n = n;
  cv.kind = con->kind;
  cv.npix = &hnpix_of(cs);
  cv.dirs.reserve(2 * np);
  for (int64_t k = 0; k < np; ++k) {
    for (int d = 0; d < 2; ++d) {
      Dir x;
      x.r = d == 0 ? hrep[k] : hmem[k];
      x.m = d == 0 ? hmem[k] : hrep[k];
      x.val = hcount[2 * k + d];
      const uint32_t bad = d == 0 ? (CA_FLAG_NO_MATCH_FWD | CA_FLAG_RECHECK_FWD)
                                  : (CA_FLAG_NO_MATCH_REV | CA_FLAG_RECHECK_REV);
      x.ok = !(hflags[k] & bad);
      x.sy = hshift[4 * k + 2 * d];
      x.sx = hshift[4 * k + 2 * d + 1];
      cv.dirs.push_back(x);
    }
  }
  // strict relation as per-member lists of covering representatives
  const auto [ps, qs] = sched.back();
  std::vector<std::vector<int32_t>> strict_in(n);
  for (const Dir& d : cv.dirs)
    if (d.r != d.m && cv.bit(d, ps, qs)) strict_in[d.m].push_back(d.r);
  auto strict = [&](int32_t r, int32_t i) {
    if (r == i) return true;
    const auto& v = strict_in[i];
    return std::find(v.begin(), v.end(), r) != v.end();
  };
  std::vector<int32_t> pool(n), reps, rank(n, -1), assign(n, -1);
  std::iota(pool.begin(), pool.end(), 0);
  std::vector<int32_t> out_rep(n, -1);
  for (int t = 0; t < K; ++t) {
    std::vector<int32_t> remaining;
    for (int32_t i : pool) {
      int32_t best = -1;
      for (int32_t r : strict_in[i])
        if (rank[r] >= 0 && (best < 0 || rank[r] < rank[best])) best = r;
      if (best >= 0) out_rep[i] = best;
      else remaining.push_back(i);
    }
    pool.swap(remaining);
    if (pool.empty()) continue;
    std::vector<int32_t> sel = lazy_greedy(cv, pool, sched[t].first, sched[t].second, assign);
    for (int32_t r : sel) {
      rank[r] = (int32_t)reps.size();
      reps.push_back(r);
    }
    std::vector<int32_t> orphans;
    for (int32_t i : pool) {
      const int32_t r = assign[i];
      if (r == i || strict(r, i)) out_rep[i] = r;
      else orphans.push_back(i);
    }
    pool.swap(orphans);
  }
  if (!pool.empty()) return fail_ctx(ctx, CA_ESTATE, "closed loop ended with orphans");
  // centers: each member's shift relative to its representative
  std::vector<std::vector<std::pair<int32_t, int32_t>>> by_member(n);  // (rep, dir index)
  for (size_t x = 0; x < cv.dirs.size(); ++x) by_member[cv.dirs[x].m].emplace_back(cv.dirs[x].r, (int32_t)x);
  for (int64_t i = 0; i < n; ++i) {
    rep_of[i] = out_rep[i];
    int16_t sy = 0, sx = 0;
    if (out_rep[i] != i)
      for (auto& pr : by_member[i])
        if (pr.first == out_rep[i]) {
          sy = cv.dirs[pr.second].sy;
          sx = cv.dirs[pr.second].sx;
          break;
        }
    center_shift[2 * i] = sy;
    center_shift[2 * i + 1] = sx;
  }
  *n_clusters = (int64_t)reps.size();
  return CA_OK;
}

extern "C" ca_status ca_cluster(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                                int32_t path, int32_t iterations, int32_t* rep_of, int16_t* center_shift,
                                int64_t* n_clusters) {
  if (!ctx) return CA_EINVAL;
  if (!cs || ctx_of(cs) != ctx || !rep_of || !center_shift || !n_clusters)
    return fail_ctx(ctx, CA_EINVAL, "bad arguments");
  if (iterations < 1 || iterations > 64) return fail_ctx(ctx, CA_EINVAL, "iterations must be in [1, 64]");
  if (!con || (con->kind != CA_COSINE && con->kind != CA_EDGE))
    return fail_ctx(ctx, CA_EINVAL, "bad constraint");
  HIP_TRY(ctx, hipSetDevice(device_of(ctx)));
  return cluster_impl(ctx, (hipStream_t)stream, cs, con, path, iterations, rep_of, center_shift, n_clusters);
}
