// Candidate generation (ca_prune) and the clustering driver (ca_cluster):
// surprisal lazy-greedy set cover (paper Sec. 3.3, Eqs. 7-9) inside the
// coarse-to-fine closed loop (Sec. 3.1), on the host over the device results.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <functional>
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
CoverCache* cover_cache_of(ca_ctx* ctx);
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

// Device memory released at scope exit.
struct DevBuf {
  ca_ctx* c = nullptr;
  void* p = nullptr;
  size_t b = 0;
  ~DevBuf() { free_ctx(c, p, b); }
  ca_status alloc(ca_ctx* ctx, size_t bytes) {
    c = ctx;
    b = std::max<size_t>(bytes, 256);
    ca_status st = alloc_ctx(ctx, &p, b);
    if (st) b = 0;
    return st;
  }
};

// Cache key of a constraint's kind and edge set.
int64_t con_key(const ca_constraint* con) { return con->kind | ((int64_t)con->edges << 8); }

bool over_contours(const ca_constraint* con) { return con->kind == CA_EDGE && con->edges == CA_EDGES_CONTOUR; }

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
// Candidate mask held at once by the bounds pass, in bytes: a quarter of the
// free device memory (at least 1 GiB; CLIPALIGN_PRUNE_CHUNK_BYTES overrides).
// Larger masks run the pass over chunks of consecutive anchors, and the
// writing call then rebuilds each chunk's mask.
// The writing call in pieces: consecutive anchors whose candidates total at
// most `cap` pairs (cap >= the longest anchor range) are written to the start
// of (rep, mem), then fn(piece size) runs on the same stream before the next
// piece overwrites them.
struct Pieces {
  int64_t cap;
  std::function<ca_status(int64_t)> fn;
};

// End of the piece of anchors that starts at a0 (at most `cap` pairs, before
// a_end); a0 itself when one anchor alone exceeds cap.
static int64_t piece_end(const std::vector<int64_t>& counts, int64_t a0, int64_t a_end, int64_t cap) {
  int64_t a1 = a0, m = 0;
  while (a1 < a_end && m + counts[a1] <= cap) m += counts[a1++];
  return a1;
}

static int64_t prune_chunk_bytes() {
  if (const char* e = std::getenv("CLIPALIGN_PRUNE_CHUNK_BYTES")) {
    const long long v = std::atoll(e);
    if (v >= 8) return v;
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0)
    return std::max<int64_t>(1ll << 30, (int64_t)(free_b / 4));
  return 8ll << 30;
}

static ca_status prune_cached_device(ca_ctx* ctx, hipStream_t s, const ca_clipset* cs, const ca_constraint* con,
                                     int64_t cap, int32_t* rep, int32_t* mem, int64_t* n_out,
                                     const Pieces* pieces = nullptr, bool defer = false,
                                     int64_t* n_bound = nullptr) {
  const bool edge = con->kind == CA_EDGE;
  const bool topo = over_contours(con);  // polygon hashes as a third table
  const Threshold thr{con->thr_num, con->thr_den};
  PruneCache* pc = prune_cache_of(ctx);
  const bool hit = pc->gen == gen_of(cs) && pc->kind == con_key(con) && pc->p == con->thr_num && pc->q == con->thr_den;
  const bool planned = pc->plan_gen == gen_of(cs) && pc->plan_kind == con_key(con) && pc->plan_p == con->thr_num &&
                       pc->plan_q == con->thr_den;
  // a hit (the writing call after a sizing call) reuses the device copies of
  // the anchor order, ranges, partner tables and (one chunk) bitmask
  int64_t na = pc->na;
  // layout: order | hi | range_off | counts | offsets | mask (largest chunk) | partner tables
  auto b_ord_of = [](int64_t n) { return aup(4 * (size_t)n); };
  auto b_rng_of = [](int64_t n) { return aup(8 * (size_t)n); };
  auto b_soa_of = [](int64_t n) { return aup(4 * 64 * (size_t)n); };
  // edge: the box-size extremes after the polygon tables
  auto ext_of = [&](char* tables, int64_t n) { return (uint32_t*)(tables + (topo ? 3 : 2) * b_soa_of(n)); };
  // the bounds pass over anchors [cuts[c], cuts[c + 1]), mask bits from cut_bit0[c]
  auto bounds_chunk = [&](char* base, size_t b_mask, int c) -> ca_status {
    const size_t b_ord = b_ord_of(na), b_rng = b_rng_of(na), b_soa = b_soa_of(na);
    PruneArgs pa{(int32_t*)base, (int32_t*)(base + b_ord), pc->cuts[c + 1], (int64_t*)(base + 2 * b_ord + b_rng),
                 nullptr, nullptr, nullptr};
    pa.a_begin = pc->cuts[c];
    pa.mask_bit0 = pc->cut_bit0[c];
    pa.soa_n = na;
    const int64_t* d_roff = (const int64_t*)(base + 2 * b_ord);
    char* tables = base + 2 * b_ord + 3 * b_rng + b_mask;
    uint32_t* d_mask = (uint32_t*)(base + 2 * b_ord + 3 * b_rng);
    if (edge) {
      pa.soa_wh = (const uint32_t*)tables;
      pa.soa_np = (const int32_t*)(tables + b_soa);
      pa.soa_hash = topo ? (const uint32_t*)(tables + 2 * b_soa) : nullptr;
      pa.soa_ext = ext_of(tables, na);
      HIP_TRY(ctx, hipMemsetAsync(d_mask, 0, b_mask, s));
      HIP_TRY(ctx, launch_edge_prune(dev_of(cs), pa, thr, d_roff, (unsigned long long*)d_mask, s));
    } else {
      HIP_TRY(ctx, hipMemsetAsync(d_mask, 0, b_mask, s));
      pa.soa_row = (const uint32_t*)tables;
      pa.soa_col = (const uint32_t*)(tables + b_soa);
      pa.soa_grp = (const uint32_t*)(tables + 2 * b_soa);
      HIP_TRY(ctx, launch_prune128(dev_of(cs), dev_of(cs), pa, thr, d_roff, d_mask, false, s));
    }
    return CA_OK;
  };
  // the pairs of anchors [a_lo, a_hi) of mask chunk c, written in pieces to
  // the start of (rep, mem), each followed by pieces->fn; off: global offsets
  auto write_pieces = [&](char* base, int c, int64_t a_lo, int64_t a_hi, const std::vector<int64_t>& counts,
                          const std::vector<int64_t>& off) -> ca_status {
    const size_t b_ord = b_ord_of(na), b_rng = b_rng_of(na);
    int64_t* d_off = (int64_t*)(base + 2 * b_ord + 2 * b_rng);
    for (int64_t a0 = a_lo; a0 < a_hi;) {
      const int64_t a1 = pieces ? piece_end(counts, a0, a_hi, pieces->cap) : a_hi;
      if (a1 == a0) return fail_ctx(ctx, CA_EINVAL, "internal: an anchor's candidates exceed the piece size");
      PruneArgs pa{(int32_t*)base, (int32_t*)(base + b_ord), a1, nullptr, d_off, rep, mem};
      pa.a_begin = a0;
      pa.mask_bit0 = pc->cut_bit0[c];
      pa.order_ids = edge ? 1 : 0;
      pa.out_base = pieces ? off[a0] : 0;
      HIP_TRY(ctx, launch_prune128(dev_of(cs), dev_of(cs), pa, thr, (int64_t*)(base + 2 * b_ord),
                                   (uint32_t*)(base + 2 * b_ord + 3 * b_rng), true, s));
      if (pieces && off[a1] > off[a0]) {
        ca_status st = pieces->fn(off[a1] - off[a0]);
        if (st) return st;
      }
      a0 = a1;
    }
    return CA_OK;
  };
  // the counts are in: the cache is valid for this key
  auto finish = [&]() {
    pc->total = 0;
    for (int64_t a = 0; a < na; ++a) pc->total += pc->counts[a];
    pc->gen = gen_of(cs);
    pc->kind = con_key(con);
    pc->p = con->thr_num;
    pc->q = con->thr_den;
    stats_of(ctx)->pairs_screened += pc->plan_screened;
    stats_of(ctx)->pairs_survived += pc->total;
  };
  if (!hit && !planned) {
    std::vector<int32_t> order, hi;
    int64_t screened = 0;
    build_ranges(cs, con, order, hi, screened);
    na = (int64_t)order.size();
    std::vector<int64_t> range_off(na + 1);
    int64_t bits = 0;
    for (int64_t a = 0; a < na; ++a) {
      range_off[a] = bits;
      const int64_t len = hi[a] - a - 1;
      bits += edge ? (len + 63) / 64 * 64 : len;
    }
    range_off[na] = bits;
    int64_t pairs = 0;
    for (int64_t a = 0; a < na; ++a) pairs += hi[a] - a - 1;
    // anchor chunks whose mask fits the budget (at least one anchor each);
    // cosine chunks start on a 32-bit mask word, edge ranges on a 64-bit one
    const int64_t cbits = prune_chunk_bytes() * 8;
    std::vector<int64_t> cuts{0};
    for (int64_t a = 1; a < na; ++a)
      if (range_off[a + 1] - (range_off[cuts.back()] & ~(int64_t)63) > cbits) cuts.push_back(a);
    cuts.push_back(na);
    std::vector<int64_t> bit0(cuts.size() - 1);
    int64_t max_bits = 0;
    for (size_t c = 0; c + 1 < cuts.size(); ++c) {
      bit0[c] = range_off[cuts[c]] & ~(int64_t)63;
      max_bits = std::max(max_bits, range_off[cuts[c + 1]] - bit0[c]);
    }
    const size_t b_ord = b_ord_of(na), b_rng = b_rng_of(na), b_soa = b_soa_of(na);
    const size_t b_mask = aup(8 * (size_t)(max_bits / 64 + 1));
    // partner tables: cosine rows, columns and shift-group maxima; edge box
    // sizes, polygon counts (and hashes), box-size extremes
    const size_t need =
        2 * b_ord + 3 * b_rng + b_mask + (edge ? (topo ? 3 : 2) * b_soa + aup(8 * (size_t)na) : 3 * b_soa);
    pc->gen = 0;  // valid only once the counts are in
    pc->plan_gen = 0;
    if (pc->bytes < need) {
      free_ctx(ctx, pc->dev, pc->bytes);
      pc->dev = nullptr;
      pc->bytes = 0;
      ca_status st = alloc_ctx(ctx, &pc->dev, need);
      if (st) return st;
      pc->bytes = need;
    }
    char* base = (char*)pc->dev;
    int32_t* d_order = (int32_t*)base;
    HIP_TRY(ctx, hipMemcpyAsync(d_order, order.data(), 4 * na, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(base + b_ord, hi.data(), 4 * na, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(base + 2 * b_ord, range_off.data(), 8 * na, hipMemcpyHostToDevice, s));
    char* tables = base + 2 * b_ord + 3 * b_rng + b_mask;
    if (edge)
      HIP_TRY(ctx, launch_edge_soa(dev_of(cs), d_order, na, (uint32_t*)tables, (int32_t*)(tables + b_soa), s,
                                   topo ? (uint32_t*)(tables + 2 * b_soa) : nullptr, ext_of(tables, na)));
    else
      HIP_TRY(ctx, launch_prune128_soa(dev_of(cs), d_order, na, (uint32_t*)tables, (uint32_t*)(tables + b_soa),
                                       (uint32_t*)(tables + 2 * b_soa), s));
    HIP_TRY(ctx, hipStreamSynchronize(s));  // the host vectors above go out of scope
    pc->na = na;
    pc->cuts = cuts;
    pc->cut_bit0 = bit0;
    pc->b_mask = b_mask;
    pc->plan_gen = gen_of(cs);
    pc->plan_kind = con_key(con);
    pc->plan_p = con->thr_num;
    pc->plan_q = con->thr_den;
    pc->plan_screened = screened;
    pc->plan_pairs = pairs;
  }
  if (!hit) {
    const int n_chunks = (int)pc->cuts.size() - 1;
    char* base = (char*)pc->dev;
    const size_t b_ord = b_ord_of(na), b_rng = b_rng_of(na);
    if (n_chunks > 1 && defer) {
      // the caller writes in pieces next: one sweep then counts and writes
      *n_out = -1;
      if (n_bound) *n_bound = pc->plan_pairs;
      return CA_OK;
    }
    pc->counts.assign(na, 0);
    if (n_chunks > 1 && pieces && rep) {
      // one sweep: each chunk's bounds pass, its counts, then its pairs in
      // pieces while its mask is in place
      std::vector<int64_t> off(na + 1, 0);
      int64_t acc = 0;
      int64_t* d_off = (int64_t*)(base + 2 * b_ord + 2 * b_rng);
      for (int c = 0; c < n_chunks; ++c) {
        ca_status st = bounds_chunk(base, pc->b_mask, c);
        if (st) return st;
        const int64_t a_lo = pc->cuts[c], a_hi = pc->cuts[c + 1];
        HIP_TRY(ctx, hipMemcpyAsync(pc->counts.data() + a_lo, base + 2 * b_ord + b_rng + 8 * a_lo,
                                    8 * (size_t)(a_hi - a_lo), hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        for (int64_t a = a_lo; a < a_hi; ++a) {
          off[a] = acc;
          acc += pc->counts[a];
        }
        off[a_hi] = acc;
        HIP_TRY(ctx, hipMemcpyAsync(d_off + a_lo, off.data() + a_lo, 8 * (size_t)(a_hi - a_lo),
                                    hipMemcpyHostToDevice, s));
        st = write_pieces(base, c, a_lo, a_hi, pc->counts, off);
        if (st) return st;
      }
      HIP_TRY(ctx, hipStreamSynchronize(s));
      finish();
      *n_out = pc->total;
      return CA_OK;
    }
    for (int c = 0; c < n_chunks; ++c) {
      ca_status st = bounds_chunk(base, pc->b_mask, c);
      if (st) return st;
    }
    HIP_TRY(ctx, hipMemcpyAsync(pc->counts.data(), base + 2 * b_ord + b_rng, 8 * na, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    finish();
  }
  const size_t b_ord = b_ord_of(na), b_rng = b_rng_of(na);
  char* base = (char*)pc->dev;
  *n_out = pc->total;
  if (!rep) return CA_OK;
  if (!pieces && pc->total > cap) return fail_ctx(ctx, CA_ETRUNC, "candidate buffer too small");
  std::vector<int64_t> off(na + 1);
  int64_t acc = 0;
  for (int64_t a = 0; a < na; ++a) {
    off[a] = acc;
    acc += pc->counts[a];
  }
  off[na] = acc;
  int64_t* d_off = (int64_t*)(base + 2 * b_ord + 2 * b_rng);
  HIP_TRY(ctx, hipMemcpyAsync(d_off, off.data(), 8 * na, hipMemcpyHostToDevice, s));
  const int n_chunks = (int)pc->cuts.size() - 1;
  for (int c = 0; c < n_chunks; ++c) {
    // one chunk: its mask is still in place from the counting pass; more: each
    // chunk's mask is rebuilt before its pairs are written
    if (n_chunks > 1) {
      ca_status st = bounds_chunk(base, pc->b_mask, c);
      if (st) return st;
    }
    ca_status st = write_pieces(base, c, pc->cuts[c], pc->cuts[c + 1], pc->counts, off);
    if (st) return st;
  }
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return CA_OK;
}

// Device candidate generation into caller buffers (or sizing only when rep is
// null), or in pieces (rep, mem: one piece).  defer: a sizing call whose
// bounds pass would run in several chunks returns *n_out = -1 and, in
// *n_bound, an upper bound of the candidates, without running it; the
// writing call in pieces then counts and writes in one sweep.
static ca_status prune_device(ca_ctx* ctx, hipStream_t s, const ca_clipset* cs, const ca_constraint* con,
                              int64_t cap, int32_t* rep, int32_t* mem, int64_t* n_out,
                              const Pieces* pieces = nullptr, bool defer = false, int64_t* n_bound = nullptr) {
  if (con->kind == CA_EDGE || mixed_ok_of(cs))
    return prune_cached_device(ctx, s, cs, con, cap, rep, mem, n_out, pieces, defer, n_bound);
  std::vector<int32_t> order, hi;
  int64_t screened = 0;
  build_ranges(cs, con, order, hi, screened);
  const int64_t na = (int64_t)order.size();
  void* sc;
  const size_t b_ord = aup(4 * (size_t)na), b_hi = aup(4 * (size_t)na), b_cnt = aup(8 * (size_t)na);
  // pieces: the alignment between them uses the context's scratch, so the
  // anchor tables get their own allocation
  DevBuf own;
  ca_status st = pieces ? own.alloc(ctx, b_ord + b_hi + 2 * b_cnt) : scratch_ctx(ctx, b_ord + b_hi + 2 * b_cnt, &sc);
  if (st) return st;
  char* base = pieces ? (char*)own.p : (char*)sc;
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
  if (!pieces && total > cap) return fail_ctx(ctx, CA_ETRUNC, "candidate buffer too small");
  HIP_TRY(ctx, hipMemcpyAsync(d_off, off.data(), 8 * na, hipMemcpyHostToDevice, s));
  pa.offs = d_off;
  pa.out_rep = rep;
  pa.out_mem = mem;
  for (int64_t a0 = 0; a0 < na;) {
    const int64_t a1 = pieces ? piece_end(cnt, a0, na, pieces->cap) : na;
    if (a1 == a0) return fail_ctx(ctx, CA_EINVAL, "internal: an anchor's candidates exceed the piece size");
    pa.a_begin = a0;
    pa.n_anchor = a1;
    pa.out_base = pieces ? off[a0] : 0;
    HIP_TRY(ctx, launch_cosine_prune(dev_of(cs), pa, thr, maxN_of(cs), s));
    const int64_t m = (a1 < na ? off[a1] : total) - off[a0];
    if (pieces && m > 0) {
      st = pieces->fn(m);
      if (st) return st;
    }
    a0 = a1;
  }
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return CA_OK;
}

extern "C" ca_status ca_prune(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                              int64_t cap, int32_t* rep, int32_t* mem, int64_t* n_out) {
  if (!ctx) return CA_EINVAL;
  if (!cs || ctx_of(cs) != ctx || !n_out) return fail_ctx(ctx, CA_EINVAL, "bad arguments");
  if (!con || (con->kind != CA_COSINE && con->kind != CA_EDGE) || con->thr_den <= 0 ||
      con->thr_num < 0 || (con->kind == CA_COSINE && con->thr_num > con->thr_den) ||
      (con->kind == CA_COSINE && con->edges != 0) || (con->edges != CA_EDGES_BOX && con->edges != CA_EDGES_CONTOUR))
    return fail_ctx(ctx, CA_EINVAL, "bad constraint");
  if (over_contours(con) && !dev_of(cs).cstat)
    return fail_ctx(ctx, CA_ESTATE, "CA_EDGES_CONTOUR needs a clip set created with CA_CLIPS_CONTOURS");
  if (cap < 0 || (cap > 0 && (!rep || !mem))) return fail_ctx(ctx, CA_EINVAL, "bad output buffers");
  HIP_TRY(ctx, hipSetDevice(device_of(ctx)));
  return prune_device(ctx, (hipStream_t)stream, cs, con, cap, cap > 0 ? rep : nullptr, mem, n_out);
}

// ------------------------------------------------------------------ cover relation

namespace {

bool cover_hit(const CoverCache* cc, const ca_clipset* cs, const ca_constraint* con, int path) {
  return cc->gen != 0 && cc->gen == gen_of(cs) && cc->kind == con_key(con) && cc->p == con->thr_num &&
         cc->q == con->thr_den && cc->path == path;
}

}  // namespace

// Candidate pairs aligned at once by the cover relation: a list longer than
// this is aligned in pieces of at most this many pairs (at least n, so one
// anchor's partners always fit; at most 2^30, so the sort keys' pair indices
// fit).  Default: an eighth of the free device memory at 45 bytes a pair;
// CLIPALIGN_COVER_PIECE_PAIRS overrides.
static int64_t cover_piece_pairs(int64_t n) {
  int64_t v = 0;
  if (const char* e = std::getenv("CLIPALIGN_COVER_PIECE_PAIRS")) v = std::atoll(e);
  if (v <= 0) {
    size_t free_b = 0, total_b = 0;
    v = (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) ? (int64_t)(free_b / 8 / 45) : (1ll << 26);
  }
  return std::max<int64_t>(std::min<int64_t>(v, 1ll << 30), std::max<int64_t>(n, 1));
}

// Pairs with a set direction and their results, kept from the pieces of a
// long candidate list (grown as pieces arrive).
struct Kept {
  DevBuf buf;
  int64_t cap = 0;
  int32_t* rep = nullptr;
  int32_t* mem = nullptr;
  uint8_t* bits = nullptr;
  int16_t* shift = nullptr;
  int32_t* count = nullptr;
  double* score = nullptr;

  static size_t bytes(int64_t c) {
    return 2 * aup(4 * (size_t)c) + aup((size_t)c) + 2 * aup(8 * (size_t)c) + aup(16 * (size_t)c);
  }
  // capacity `want`, the first `used` entries copied over
  ca_status grow(ca_ctx* ctx, hipStream_t s, int64_t want, int64_t used) {
    DevBuf nb;
    ca_status st = nb.alloc(ctx, bytes(want));
    if (st) return st;
    char* w = (char*)nb.p;
    int32_t* n_rep = (int32_t*)w; w += aup(4 * (size_t)want);
    int32_t* n_mem = (int32_t*)w; w += aup(4 * (size_t)want);
    uint8_t* n_bits = (uint8_t*)w; w += aup((size_t)want);
    int16_t* n_shift = (int16_t*)w; w += aup(8 * (size_t)want);
    int32_t* n_count = (int32_t*)w; w += aup(8 * (size_t)want);
    double* n_score = (double*)w;
    if (used > 0) {
      HIP_TRY(ctx, hipMemcpyAsync(n_rep, rep, 4 * (size_t)used, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, hipMemcpyAsync(n_mem, mem, 4 * (size_t)used, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, hipMemcpyAsync(n_bits, bits, (size_t)used, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, hipMemcpyAsync(n_shift, shift, 8 * (size_t)used, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, hipMemcpyAsync(n_count, count, 8 * (size_t)used, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, hipMemcpyAsync(n_score, score, 16 * (size_t)used, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, hipStreamSynchronize(s));
    }
    std::swap(buf.c, nb.c);
    std::swap(buf.p, nb.p);
    std::swap(buf.b, nb.b);
    cap = want;
    rep = n_rep;
    mem = n_mem;
    bits = n_bits;
    shift = n_shift;
    count = n_count;
    score = n_score;
    return CA_OK;
  }
};

// Steps 1-5 of the compaction on np aligned pairs (both directions each):
// row counts, row pointers, keys scattered to their rows, per-row sort and
// the gather, into the cover cache's arrays.
static ca_status cover_compact(ca_ctx* ctx, hipStream_t s, CoverCache* cc, int64_t n, int64_t np,
                               const int32_t* d_rep, const int32_t* d_mem, const uint8_t* d_bits,
                               const int16_t* d_shift, const int32_t* d_count, const double* d_score) {
  if (np >= (1ll << 31))
    return fail_ctx(ctx, CA_EUNSUPPORTED, "cover relation from 2^31 or more candidate pairs with a set direction");
  DevBuf rows;
  ca_status st = rows.alloc(ctx, 2 * aup(8 * (size_t)n));
  if (st) return st;
  unsigned long long* d_rowcnt = (unsigned long long*)rows.p;
  unsigned long long* d_fill = (unsigned long long*)((char*)rows.p + aup(8 * (size_t)n));
  HIP_TRY(ctx, launch_zero_u64(d_rowcnt, n, s));
  HIP_TRY(ctx, launch_cover_count(np, d_rep, d_mem, d_bits, d_rowcnt, s));
  std::vector<int64_t> cnt(n);
  HIP_TRY(ctx, hipMemcpyAsync(cnt.data(), d_rowcnt, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  std::vector<int64_t> row_ptr(n + 1, 0);
  std::vector<int32_t> small_rows, large_rows;
  int64_t longest = 0;
  for (int64_t r = 0; r < n; ++r) {
    row_ptr[r + 1] = row_ptr[r] + cnt[r];
    if (cnt[r] > 64) large_rows.push_back((int32_t)r);
    else if (cnt[r] > 1) small_rows.push_back((int32_t)r);
    longest = std::max(longest, cnt[r]);
  }
  const int64_t nnz = row_ptr[n];
  // the cache's arrays
  const size_t c_rp = aup(8 * (size_t)(n + 1)), c_col = aup(4 * (size_t)nnz), c_sh = aup(4 * (size_t)nnz),
               c_val = aup(4 * (size_t)nnz), c_sc = aup(8 * (size_t)nnz);
  const size_t c_bytes = c_rp + c_col + c_sh + c_val + c_sc;
  st = alloc_ctx(ctx, &cc->dev, c_bytes);
  if (st) return st;
  cc->bytes = c_bytes;
  char* c = (char*)cc->dev;
  cc->row_ptr = (int64_t*)c; c += c_rp;
  cc->col = (int32_t*)c; c += c_col;
  cc->shift = (int16_t*)c; c += c_sh;
  cc->value = (int32_t*)c; c += c_val;
  cc->score = (double*)c;
  HIP_TRY(ctx, hipMemcpyAsync(cc->row_ptr, row_ptr.data(), 8 * (size_t)(n + 1), hipMemcpyHostToDevice, s));
  if (nnz > 0) {
    // keys, merge space for rows above the LDS sort, and the row lists
    const size_t k_keys = aup(8 * (size_t)nnz), k_tmp = longest > 4096 ? k_keys : 0,
                 k_small = aup(4 * small_rows.size()), k_large = aup(4 * large_rows.size());
    DevBuf kb;
    st = kb.alloc(ctx, k_keys + k_tmp + k_small + k_large);
    if (st) return st;
    char* k = (char*)kb.p;
    uint64_t* d_keys = (uint64_t*)k;
    uint64_t* d_tmp = k_tmp ? (uint64_t*)(k + k_keys) : nullptr;
    int32_t* d_small = (int32_t*)(k + k_keys + k_tmp);
    int32_t* d_large = (int32_t*)(k + k_keys + k_tmp + k_small);
    if (!small_rows.empty())
      HIP_TRY(ctx, hipMemcpyAsync(d_small, small_rows.data(), 4 * small_rows.size(), hipMemcpyHostToDevice, s));
    if (!large_rows.empty())
      HIP_TRY(ctx, hipMemcpyAsync(d_large, large_rows.data(), 4 * large_rows.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, launch_zero_u64(d_fill, n, s));
    HIP_TRY(ctx, launch_cover_scatter(np, d_rep, d_mem, d_bits, cc->row_ptr, d_fill, d_keys, s));
    HIP_TRY(ctx, launch_cover_sort(d_small, (int64_t)small_rows.size(), d_large, (int64_t)large_rows.size(),
                                   cc->row_ptr, d_keys, d_tmp, s));
    HIP_TRY(ctx, launch_cover_gather(nnz, d_keys, d_shift, d_count, d_score, cc->col, cc->shift, cc->value,
                                     cc->score, s));
  }
  HIP_TRY(ctx, hipStreamSynchronize(s));
  cc->n = n;
  cc->nnz = nnz;
  cc->h_row_ptr.swap(row_ptr);
  stats_of(ctx)->cover_nnz = nnz;
  return CA_OK;
}

// The cover relation of `con` on the clip set (Sec. 3.1 stage 2): candidate
// pairs from the safe bounds, both directions aligned with `path` (cosine)
// or the edge track, and the set directions compacted on the device into a
// CSR sorted by (representative, member), kept in the context's cache.  A
// candidate list longer than the piece size is written, aligned and reduced
// to its pairs with a set direction piece by piece, so its per-pair results
// never exist all at once.
static ca_status cover_build(ca_ctx* ctx, hipStream_t s, const ca_clipset* cs, const ca_constraint* con, int path,
                             CoverCache** out) {
  CoverCache* cc = cover_cache_of(ctx);
  const int pth = con->kind == CA_COSINE ? path : -1;
  *out = cc;
  if (cover_hit(cc, cs, con, pth)) return CA_OK;
  // the stale relation's memory goes before the new one is built
  free_ctx(ctx, cc->dev, cc->bytes);
  cc->dev = nullptr;
  cc->bytes = 0;
  cc->gen = 0;
  const int64_t n = n_of(cs);
  int64_t np = 0, bound = 0;
  ca_status st = prune_device(ctx, s, cs, con, 0, nullptr, nullptr, &np, nullptr, true, &bound);
  if (st) return st;
  // np < 0: the bounds pass runs in chunks and is left to the piece sweep;
  // no piece needs to hold more than the bound of the candidates
  const int64_t piece =
      np >= 0 ? cover_piece_pairs(n) : std::min(cover_piece_pairs(n), std::max<int64_t>(bound, 1));
  if (np >= 0 && np <= piece) {
    // candidate pairs and their results
    const size_t b4 = aup(4 * (size_t)np), b_bits = aup((size_t)np), b_sh = aup(8 * (size_t)np),
                 b_cnt = aup(8 * (size_t)np), b_sc = aup(16 * (size_t)np);
    DevBuf work;
    st = work.alloc(ctx, 3 * b4 + b_bits + b_sh + b_cnt + b_sc);
    if (st) return st;
    char* w = (char*)work.p;
    int32_t* d_rep = (int32_t*)w; w += b4;
    int32_t* d_mem = (int32_t*)w; w += b4;
    uint32_t* d_flags = (uint32_t*)w; w += b4;
    uint8_t* d_bits = (uint8_t*)w; w += b_bits;
    int16_t* d_shift = (int16_t*)w; w += b_sh;
    int32_t* d_count = (int32_t*)w; w += b_cnt;
    double* d_score = (double*)w;
    if (np > 0) {
      int64_t got = 0;
      st = prune_device(ctx, s, cs, con, np, d_rep, d_mem, &got);
      if (st) return st;
      st = ca_align_pairs(ctx, s, cs, con, path, np, d_rep, d_mem, d_bits, d_shift, d_count, d_score, d_flags);
      if (st) return st;
    }
    st = cover_compact(ctx, s, cc, n, np, d_rep, d_mem, d_bits, d_shift, d_count, d_score);
  } else {
    Kept kept;
    int64_t n_kept = 0;
    {
      const size_t p4 = aup(4 * (size_t)piece), p_bits = aup((size_t)piece), p8 = aup(8 * (size_t)piece),
                   p_sc = aup(16 * (size_t)piece);
      DevBuf work;
      st = work.alloc(ctx, 3 * p4 + p_bits + 2 * p8 + p_sc + 256);
      if (st) return st;
      char* w = (char*)work.p;
      int32_t* p_rep = (int32_t*)w; w += p4;
      int32_t* p_mem = (int32_t*)w; w += p4;
      uint32_t* p_flags = (uint32_t*)w; w += p4;
      uint8_t* p_bitv = (uint8_t*)w; w += p_bits;
      int16_t* p_shift = (int16_t*)w; w += p8;
      int32_t* p_count = (int32_t*)w; w += p8;
      double* p_score = (double*)w; w += p_sc;
      unsigned long long* d_ctr = (unsigned long long*)w;  // [0] kept in the piece, [1] next slot
      HIP_TRY(ctx, launch_zero_u64(d_ctr, 2, s));
      Pieces pcs{piece, [&](int64_t m) -> ca_status {
        ca_status e = ca_align_pairs(ctx, s, cs, con, path, m, p_rep, p_mem, p_bitv, p_shift, p_count, p_score,
                                     p_flags);
        if (e) return e;
        HIP_TRY(ctx, launch_zero_u64(d_ctr, 1, s));
        HIP_TRY(ctx, launch_cover_keep_count(m, p_bitv, d_ctr, s));
        unsigned long long c = 0;
        HIP_TRY(ctx, hipMemcpyAsync(&c, d_ctr, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        if (c == 0) return CA_OK;
        if (n_kept + (int64_t)c >= (1ll << 31))
          return fail_ctx(ctx, CA_EUNSUPPORTED,
                          "cover relation from 2^31 or more candidate pairs with a set direction");
        if (n_kept + (int64_t)c > kept.cap) {
          e = kept.grow(ctx, s, std::max(n_kept + (int64_t)c, kept.cap + kept.cap / 2), n_kept);
          if (e) return e;
        }
        HIP_TRY(ctx, launch_cover_keep(m, p_rep, p_mem, p_bitv, p_shift, p_count, p_score, d_ctr + 1, kept.rep,
                                       kept.mem, kept.bits, kept.shift, kept.count, kept.score, s));
        n_kept += (int64_t)c;
        return CA_OK;
      }};
      int64_t got = 0;
      st = prune_device(ctx, s, cs, con, 0, p_rep, p_mem, &got, &pcs);
      if (st) return st;
    }
    st = cover_compact(ctx, s, cc, n, n_kept, kept.rep, kept.mem, kept.bits, kept.shift, kept.count, kept.score);
  }
  if (st) return st;
  cc->gen = gen_of(cs);
  cc->kind = con_key(con);
  cc->p = con->thr_num;
  cc->q = con->thr_den;
  cc->path = pth;
  return CA_OK;
}

// Cosine paths the cover relation and the clustering accept (every one but
// the switched-off direct path).
static bool cover_path_ok(int32_t path) {
  return (path >= CA_PATH_MIXED && path <= CA_PATH_AUTO) || path == CA_PATH_XCORR || path == CA_PATH_XYSEP;
}

static bool valid_con(const ca_constraint* con) {
  if (!con) return false;
  if (con->kind == CA_COSINE)
    return con->edges == 0 && con->thr_num >= 0 && con->thr_den > 0 && con->thr_num <= con->thr_den &&
           con->thr_den <= (1 << 24);
  if (con->kind == CA_EDGE)
    return (con->edges == CA_EDGES_BOX || con->edges == CA_EDGES_CONTOUR) && con->thr_num >= 0 &&
           con->thr_den == 1 && con->thr_num < (1 << 20);
  return false;
}

// CA_EDGES_CONTOUR reads the contour tables of the clip set.
static ca_status contours_ok(ca_ctx* ctx, const ca_clipset* cs, const ca_constraint* con) {
  if (over_contours(con) && !dev_of(cs).cstat)
    return fail_ctx(ctx, CA_ESTATE, "CA_EDGES_CONTOUR needs a clip set created with CA_CLIPS_CONTOURS");
  return CA_OK;
}

extern "C" ca_status ca_cover(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                              int32_t path, int64_t cap, int64_t* row_ptr, int32_t* col, int16_t* shift,
                              int32_t* value, double* score, int64_t* nnz) {
  if (!ctx) return CA_EINVAL;
  if (!cs || ctx_of(cs) != ctx || !nnz || cap < 0) return fail_ctx(ctx, CA_EINVAL, "bad arguments");
  if (!valid_con(con)) return fail_ctx(ctx, CA_EINVAL, "bad constraint");
  if (contours_ok(ctx, cs, con)) return CA_ESTATE;
  if (con->kind == CA_COSINE && !cover_path_ok(path))
    return fail_ctx(ctx, CA_EINVAL, "cover path must be CA_PATH_MIXED, CA_PATH_FP32, CA_PATH_FP64, CA_PATH_AUTO, CA_PATH_XCORR or CA_PATH_XYSEP");
  HIP_TRY(ctx, hipSetDevice(device_of(ctx)));
  hipStream_t s = (hipStream_t)stream;
  CoverCache* cc = nullptr;
  ca_status st = cover_build(ctx, s, cs, con, path, &cc);
  if (st) return st;
  *nnz = cc->nnz;
  if (!row_ptr) return CA_OK;
  if (cc->nnz > cap) return fail_ctx(ctx, CA_ETRUNC, "cover buffers smaller than the relation (see *nnz)");
  const int64_t n = cc->n, z = cc->nnz;
  HIP_TRY(ctx, hipMemcpyAsync(row_ptr, cc->row_ptr, 8 * (size_t)(n + 1), hipMemcpyDeviceToDevice, s));
  if (z > 0) {
    if (col) HIP_TRY(ctx, hipMemcpyAsync(col, cc->col, 4 * (size_t)z, hipMemcpyDeviceToDevice, s));
    if (shift) HIP_TRY(ctx, hipMemcpyAsync(shift, cc->shift, 4 * (size_t)z, hipMemcpyDeviceToDevice, s));
    if (value) HIP_TRY(ctx, hipMemcpyAsync(value, cc->value, 4 * (size_t)z, hipMemcpyDeviceToDevice, s));
    if (score) HIP_TRY(ctx, hipMemcpyAsync(score, cc->score, 8 * (size_t)z, hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return CA_OK;
}

extern "C" ca_status ca_cover_dense(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                                    int32_t path, uint64_t* bits) {
  if (!ctx) return CA_EINVAL;
  if (!cs || ctx_of(cs) != ctx || !bits) return fail_ctx(ctx, CA_EINVAL, "bad arguments");
  if (!valid_con(con)) return fail_ctx(ctx, CA_EINVAL, "bad constraint");
  if (contours_ok(ctx, cs, con)) return CA_ESTATE;
  if (con->kind == CA_COSINE && !cover_path_ok(path))
    return fail_ctx(ctx, CA_EINVAL, "cover path must be CA_PATH_MIXED, CA_PATH_FP32, CA_PATH_FP64, CA_PATH_AUTO, CA_PATH_XCORR or CA_PATH_XYSEP");
  if (n_of(cs) > CA_COVER_DENSE_MAX) return fail_ctx(ctx, CA_EUNSUPPORTED, "dense cover matrix above 65,536 clips");
  HIP_TRY(ctx, hipSetDevice(device_of(ctx)));
  hipStream_t s = (hipStream_t)stream;
  CoverCache* cc = nullptr;
  ca_status st = cover_build(ctx, s, cs, con, path, &cc);
  if (st) return st;
  const int64_t n = cc->n, words = (n + 63) / 64;
  HIP_TRY(ctx, launch_zero_u64((unsigned long long*)bits, n * words, s));
  HIP_TRY(ctx, launch_cover_dense(n, words, cc->row_ptr, cc->col, (unsigned long long*)bits, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return CA_OK;
}

// Center verification of an assignment (host arrays) on the device.
static ca_status verify_centers(ca_ctx* ctx, hipStream_t s, const ca_clipset* cs, const ca_constraint* con,
                                const int32_t* rep_of, const int16_t* center_shift, int64_t* n_viol,
                                int64_t* first_viol) {
  const int64_t n = n_of(cs);
  int64_t viol = 0, first = -1;
  auto note = [&](int64_t i) {
    ++viol;
    if (first < 0 || i < first) first = i;
  };
  std::vector<int32_t> mem, rep;
  std::vector<int16_t> sh;
  std::vector<int64_t> who;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t r = rep_of[i];
    if (r < 0 || r >= n) { note(i); continue; }
    if (r == i) {
      if (center_shift[2 * i] != 0 || center_shift[2 * i + 1] != 0) note(i);
      continue;
    }
    if (rep_of[r] != r) { note(i); continue; }  // a representative represents itself
    mem.push_back((int32_t)i);
    rep.push_back(r);
    sh.push_back(center_shift[2 * i]);
    sh.push_back(center_shift[2 * i + 1]);
    who.push_back(i);
  }
  const int64_t m = (int64_t)mem.size();
  if (m > 0) {
    DevBuf buf;
    const size_t b4 = aup(4 * (size_t)m);
    ca_status st = buf.alloc(ctx, 3 * b4 + 256);
    if (st) return st;
    char* p = (char*)buf.p;
    int32_t* d_mem = (int32_t*)p;
    int32_t* d_rep = (int32_t*)(p + b4);
    int16_t* d_sh = (int16_t*)(p + 2 * b4);
    unsigned long long* d_out = (unsigned long long*)(p + 3 * b4);
    HIP_TRY(ctx, hipMemcpyAsync(d_mem, mem.data(), 4 * (size_t)m, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(d_rep, rep.data(), 4 * (size_t)m, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(d_sh, sh.data(), 4 * (size_t)m, hipMemcpyHostToDevice, s));
    const unsigned long long init[2] = {0ull, ~0ull};
    HIP_TRY(ctx, hipMemcpyAsync(d_out, init, sizeof(init), hipMemcpyHostToDevice, s));
    const Threshold thr{con->thr_num, con->thr_den};
    if (con->kind == CA_COSINE)
      HIP_TRY(ctx, launch_verify_cosine(dev_of(cs), m, d_mem, d_rep, d_sh, thr, d_out, d_out + 1, s));
    else
      HIP_TRY(ctx, launch_verify_edge(dev_of(cs), m, d_mem, d_rep, d_sh, thr, d_out, d_out + 1, s,
                                      over_contours(con)));
    unsigned long long h[2];
    HIP_TRY(ctx, hipMemcpyAsync(h, d_out, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    viol += (int64_t)h[0];
    if (h[0] > 0) {
      const int64_t i = who[(size_t)h[1]];
      if (first < 0 || i < first) first = i;
    }
  }
  ca_run_stats* rs = stats_of(ctx);
  rs->members_verified += m;
  rs->center_violations += viol;
  *n_viol = viol;
  if (first_viol) *first_viol = first;
  return CA_OK;
}

extern "C" ca_status ca_verify_centers(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                                       const int32_t* rep_of, const int16_t* center_shift, int64_t* n_violations,
                                       int64_t* first_violation) {
  if (!ctx) return CA_EINVAL;
  if (!cs || ctx_of(cs) != ctx || !rep_of || !center_shift || !n_violations)
    return fail_ctx(ctx, CA_EINVAL, "bad arguments");
  if (!valid_con(con)) return fail_ctx(ctx, CA_EINVAL, "bad constraint");
  if (contours_ok(ctx, cs, con)) return CA_ESTATE;
  HIP_TRY(ctx, hipSetDevice(device_of(ctx)));
  return verify_centers(ctx, (hipStream_t)stream, cs, con, rep_of, center_shift, n_violations, first_violation);
}

// ------------------------------------------------------------------ set cover

namespace {

// The cover relation on the host: CSR rows of representatives, entries that
// pass the loosest threshold; the bit at any stricter threshold is decided
// from the stored count (cosine) or residual (edge).
struct Cover {
  int64_t n;
  int kind;
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col, value;
  std::vector<int16_t> shift;
  const std::vector<int32_t>* npix;
  bool bit(int64_t r, int64_t e, int64_t p, int64_t q) const {
    if (kind == CA_COSINE) {
      const int64_t nm = (*npix)[col[e]], nr = (*npix)[r];
      if (nm <= 0 || nr <= 0) return false;
      const uint64_t c = (uint64_t)value[e];
      const unsigned __int128 lhs = (unsigned __int128)(c * c) * (unsigned __int128)((uint64_t)q * (uint64_t)q);
      const unsigned __int128 rhs = (unsigned __int128)((uint64_t)p * (uint64_t)p) *
                                    (unsigned __int128)((uint64_t)nm * (uint64_t)nr);
      return lhs > rhs;
    }
    return value[e] >= 0 && value[e] <= p;
  }
};

// Surprisal lazy greedy on `pool` (ascending ids) with threshold (p, q).
// Returns reps in selection order and fills assign[i] for pool members.
std::vector<int32_t> lazy_greedy(const Cover& cv, const std::vector<int32_t>& pool, int64_t p, int64_t q,
                                 std::vector<int32_t>& pos, std::vector<int32_t>& assign) {
  for (size_t a = 0; a < pool.size(); ++a) pos[pool[a]] = (int32_t)a;
  const size_t P = pool.size();
  // out-neighbours within the pool; rows list members in ascending id, and
  // positions ascend with ids, so each list is sorted and duplicate-free
  std::vector<std::vector<int32_t>> out(P);
  std::vector<int64_t> indeg(P, 0);
  for (size_t a = 0; a < P; ++a) {
    const int64_t r = pool[a];
    for (int64_t e = cv.row_ptr[r]; e < cv.row_ptr[r + 1]; ++e) {
      const int32_t b = pos[cv.col[e]];
      if (b < 0 || !cv.bit(r, e, p, q)) continue;
      out[a].push_back(b);
      indeg[b]++;
    }
  }
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
  for (int32_t i : pool) pos[i] = -1;
  return reps;
}

}  // namespace

// relax_num / relax_den: the cosine schedule's total relaxation (tau_t =
// T - relax (K - t) / (K - 1)), or the edge schedule's step in pixels
// (tau_t = T + relax_num (K - t)).
static ca_status cluster_impl(ca_ctx* ctx, hipStream_t s, const ca_clipset* cs, const ca_constraint* con,
                              int32_t path, int32_t K, int64_t relax_num, int64_t relax_den, int32_t* rep_of,
                              int16_t* center_shift, int64_t* n_clusters) {
  const int64_t n = n_of(cs);
  // thresholds t = 1..K (exact rationals), loosest first
  std::vector<std::pair<int64_t, int64_t>> sched;
  for (int t = 1; t <= K; ++t) {
    if (con->kind == CA_COSINE) {
      // p/q - (a/b) (K - t)/(K - 1) = (p b (K - 1) - a q (K - t)) / (q b (K - 1))
      int64_t p = con->thr_num, q = con->thr_den;
      if (K > 1) {
        const int64_t num = p * relax_den * (K - 1) - relax_num * q * (int64_t)(K - t);
        const int64_t den = q * relax_den * (K - 1);
        const int64_t g = std::gcd(std::max<int64_t>(num, 0), den);
        p = std::max<int64_t>(num, 0) / (g ? g : 1);
        q = den / (g ? g : 1);
      }
      sched.emplace_back(p, q);
    } else {
      sched.emplace_back(con->thr_num + relax_num * (K - t), 1);
    }
  }
  ca_constraint loose = *con;
  loose.thr_num = sched[0].first;
  loose.thr_den = sched[0].second;
  // the relation at the loosest threshold, compacted on the device; the host
  // holds O(n + nnz)
  CoverCache* cc = nullptr;
  ca_status st = cover_build(ctx, s, cs, &loose, path, &cc);
  if (st) return st;
  Cover cv;
  cv.n = n;
  cv.kind = con->kind;
  cv.npix = &hnpix_of(cs);
  cv.row_ptr = cc->h_row_ptr;
  const int64_t nnz = cc->nnz;
  cv.col.resize(nnz);
  cv.value.resize(nnz);
  cv.shift.resize(2 * nnz);
  if (nnz > 0) {
    HIP_TRY(ctx, hipMemcpyAsync(cv.col.data(), cc->col, 4 * (size_t)nnz, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(cv.value.data(), cc->value, 4 * (size_t)nnz, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(cv.shift.data(), cc->shift, 4 * (size_t)nnz, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
  }
  // strict relation as per-member lists of covering representatives
  const auto [ps, qs] = sched.back();
  std::vector<int64_t> in_ptr(n + 1, 0);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t e = cv.row_ptr[r]; e < cv.row_ptr[r + 1]; ++e)
      if (cv.bit(r, e, ps, qs)) in_ptr[cv.col[e] + 1]++;
  for (int64_t i = 0; i < n; ++i) in_ptr[i + 1] += in_ptr[i];
  std::vector<int32_t> strict_in(in_ptr[n]);
  {
    std::vector<int64_t> cur(in_ptr.begin(), in_ptr.end() - 1);
    for (int64_t r = 0; r < n; ++r)
      for (int64_t e = cv.row_ptr[r]; e < cv.row_ptr[r + 1]; ++e)
        if (cv.bit(r, e, ps, qs)) strict_in[cur[cv.col[e]]++] = (int32_t)r;
  }
  // strict bit of (r covers i), r != i: binary search of i in row r
  auto find = [&](int32_t r, int32_t i) -> int64_t {
    const auto b = cv.col.begin() + cv.row_ptr[r], e = cv.col.begin() + cv.row_ptr[r + 1];
    const auto it = std::lower_bound(b, e, i);
    return (it != e && *it == i) ? (int64_t)(it - cv.col.begin()) : -1;
  };
  auto strict = [&](int32_t r, int32_t i) {
    if (r == i) return true;
    const int64_t e = find(r, i);
    return e >= 0 && cv.bit(r, e, ps, qs);
  };
  std::vector<int32_t> pool(n), reps, rank(n, -1), assign(n, -1), pos(n, -1);
  std::iota(pool.begin(), pool.end(), 0);
  std::vector<int32_t> out_rep(n, -1);
  for (int t = 0; t < K; ++t) {
    // re-attach to the first representative (selection order) covering strictly
    std::vector<int32_t> remaining;
    for (int32_t i : pool) {
      int32_t best = -1;
      for (int64_t x = in_ptr[i]; x < in_ptr[i + 1]; ++x) {
        const int32_t r = strict_in[x];
        if (rank[r] >= 0 && (best < 0 || rank[r] < rank[best])) best = r;
      }
      if (best >= 0) out_rep[i] = best;
      else remaining.push_back(i);
    }
    pool.swap(remaining);
    if (pool.empty()) continue;
    std::vector<int32_t> sel = lazy_greedy(cv, pool, sched[t].first, sched[t].second, pos, assign);
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
  for (int64_t i = 0; i < n; ++i) {
    rep_of[i] = out_rep[i];
    int16_t sy = 0, sx = 0;
    if (out_rep[i] != i) {
      const int64_t e = find(out_rep[i], (int32_t)i);
      if (e < 0) return fail_ctx(ctx, CA_ESTATE, "member without a cover entry to its representative");
      sy = cv.shift[2 * e];
      sx = cv.shift[2 * e + 1];
    }
    center_shift[2 * i] = sy;
    center_shift[2 * i + 1] = sx;
  }
  *n_clusters = (int64_t)reps.size();
  // every member satisfies the strict constraint at its center (recomputed
  // on the device from the clips' rasters, exact integer arithmetic)
  int64_t viol = 0, first = -1;
  st = verify_centers(ctx, s, cs, con, rep_of, center_shift, &viol, &first);
  if (st) return st;
  if (viol > 0)
    return fail_ctx(ctx, CA_ESTATE, ("center verification failed for " + std::to_string(viol) +
                                     " clips (first: " + std::to_string(first) + ")").c_str());
  return CA_OK;
}

extern "C" ca_status ca_cluster(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                                int32_t path, int32_t iterations, int32_t* rep_of, int16_t* center_shift,
                                int64_t* n_clusters) {
  if (!ctx) return CA_EINVAL;
  if (!cs || ctx_of(cs) != ctx || !rep_of || !center_shift || !n_clusters)
    return fail_ctx(ctx, CA_EINVAL, "bad arguments");
  if (iterations < 1 || iterations > 64) return fail_ctx(ctx, CA_EINVAL, "iterations must be in [1, 64]");
  if (!valid_con(con)) return fail_ctx(ctx, CA_EINVAL, "bad constraint");
  if (contours_ok(ctx, cs, con)) return CA_ESTATE;
  HIP_TRY(ctx, hipSetDevice(device_of(ctx)));
  return cluster_impl(ctx, (hipStream_t)stream, cs, con, path, iterations, con->kind == CA_COSINE ? 2 : 1,
                      con->kind == CA_COSINE ? 100 : 1, rep_of, center_shift, n_clusters);
}

extern "C" ca_status ca_cluster_schedule(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                                         int32_t path, int32_t iterations, int64_t relax_num, int64_t relax_den,
                                         int32_t* rep_of, int16_t* center_shift, int64_t* n_clusters) {
  if (!ctx) return CA_EINVAL;
  if (!cs || ctx_of(cs) != ctx || !rep_of || !center_shift || !n_clusters)
    return fail_ctx(ctx, CA_EINVAL, "bad arguments");
  if (iterations < 1 || iterations > 64) return fail_ctx(ctx, CA_EINVAL, "iterations must be in [1, 64]");
  if (!valid_con(con)) return fail_ctx(ctx, CA_EINVAL, "bad constraint");
  if (contours_ok(ctx, cs, con)) return CA_ESTATE;
  if (con->kind == CA_COSINE) {
    // 0 <= relax < T, exact; kept small enough for 64-bit products
    if (relax_num < 0 || relax_den <= 0 || relax_den > (1 << 24) ||
        (__int128)relax_num * con->thr_den >= (__int128)con->thr_num * relax_den)
      return fail_ctx(ctx, CA_EINVAL, "cosine relaxation must satisfy 0 <= relax_num/relax_den < thr_num/thr_den");
  } else if (relax_num < 0 || relax_num > 1024 || relax_den != 1) {
    return fail_ctx(ctx, CA_EINVAL, "edge relaxation is relax_num pixels per step (0..1024) with relax_den = 1");
  }
  HIP_TRY(ctx, hipSetDevice(device_of(ctx)));
  return cluster_impl(ctx, (hipStream_t)stream, cs, con, path, iterations, relax_num, relax_den, rep_of, center_shift,
                      n_clusters);
}
