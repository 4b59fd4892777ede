// Serving: continuous batching of request batches against a device-resident
// library of cluster representatives (the cosine track of paper Sec. 3.2.1
// applied as in the refinement step of Sec. 3.1: a new pattern is aligned to
// fixed representatives and accepted by the strict threshold).
//
// A server owns `slots` workers, each with its own library context, HIP
// stream (default priority) and host thread.  Requests are admitted while
// their estimated device footprint fits the server's HBM budget; an admitted
// request waits for a free slot, and requests on different slots overlap on
// the device.  A request's pipeline, all on its slot's stream:
//   1. rasterise, pack and transform the batch (ca_clips_create);
//   2. candidates: for every batch clip the library range allowed by the area
//      bound (library ordered by pixel count, range by binary search), then
//      the signature bounds on the GPU (bipartite prune128);
//   3. mixed-precision alignment of every candidate (member = batch clip,
//      representative = library clip) with FP64 re-decision of near ties;
//   4. per batch clip the best covering representative: highest score, ties
//      to the lowest representative id; unmatched clips report -1.
// The result of a clip depends only on the clip and the library, never on
// which other requests share the device.
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host_internal.h"
#include "kernels.h"

struct ca_ctx;
struct ca_clipset;
namespace capriv {
ca_status fail_ctx(ca_ctx* ctx, ca_status st, const char* msg);
int device_of(const ca_ctx* ctx);
const ca::ClipsDev& dev_of(const ca_clipset* cs);
ca_ctx* ctx_of(const ca_clipset* cs);
const std::vector<int32_t>& hnpix_of(const ca_clipset* cs);
int64_t n_of(const ca_clipset* cs);
bool mixed_ok_of(const ca_clipset* cs);
ca_status align_cosine_sets(ca_ctx* ctx, const ca_clipset* crs, const ca_clipset* cms, hipStream_t s,
                            ca::Threshold thr, int path, const ca::PairIO& io, bool checked = false,
                            int direct_n = 0, int bucket_w = 1 << 20);
ca_status clips_create_in(ca_ctx* ctx, void* stream, int64_t n, const int64_t* rect_ptr, const int32_t* rects,
                          const int16_t* raster_n, const int16_t* marker_w, uint32_t flags, DevArena* arena,
                          ca_clipset** out);
bool has_fp32_of(const ca_clipset* cs);
bool has_fp64_of(const ca_clipset* cs);
int64_t check_sample_of(const ca_ctx* ctx);
}  // namespace capriv

using namespace ca;
using namespace capriv;

namespace {

struct Request {
  uint64_t id = 0;
  int64_t n = 0;
  std::vector<int64_t> rect_ptr;
  std::vector<int32_t> rects;
  std::vector<int16_t> raster_n, marker_w;
  uint64_t est_bytes = 0;
  int state = 0;  // 0 queued, 1 running, 2 done, 3 failed
  ca_status status = CA_OK;
  std::string error;
  std::vector<int32_t> best_rep;
  std::vector<int16_t> shift;
  std::vector<double> score;
  std::vector<uint8_t> matched;
  int64_t candidates = 0;
};

// Per-request device footprint estimate: the batch clip set (bits, tables,
// runs, FP16 + FP64 spectra at 128 x 128, FP32 spectra too when the library
// keeps them) and up to 4096 candidates per clip with their outputs and prune
// scratch.  It also sizes the slot's arena.
uint64_t estimate_bytes(int64_t n, bool fp32) {
  return (uint64_t)n * (200000ull + (fp32 ? 70000ull : 0ull) + 4096ull * 64ull) + (1ull << 20);
}

}  // namespace

struct ca_server {
  ca_ctx* owner = nullptr;
  const ca_clipset* lib = nullptr;
  ca_constraint con{};
  uint64_t budget = 0;
  uint64_t inflight = 0;
  std::vector<int32_t> lib_order;  // library ids by (n, id)
  std::vector<int32_t> lib_n;      // their pixel counts
  int32_t* d_order = nullptr;
  uint32_t* d_soa = nullptr;       // transposed library sliding sums: rows, columns (64 x n each), then
                                   // their shift-group maxima (64 x n)
  std::vector<ca_ctx*> slot_ctx;
  std::vector<hipStream_t> slot_stream;
  std::vector<capriv::DevArena> slot_arena;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> reqs;
  uint64_t next_id = 1;
  bool stop = false;
  int64_t done_requests = 0, done_pairs = 0;
  std::vector<ca_run_stats> slot_stats;  // each slot context's statistics after its last request
  std::string err;
};

namespace {

ca_status srv_fail(ca_server* srv, ca_status st, const std::string& msg) {
  std::lock_guard<std::mutex> g(srv->mu);
  srv->err = msg;
  return st;
}

#define RUN_HIP(expr)                                                  \
  do {                                                                 \
    hipError_t e_ = (expr);                                            \
    if (e_ != hipSuccess) {                                            \
      req->status = CA_EDEVICE;                                        \
      req->error = std::string(#expr ": ") + hipGetErrorString(e_);    \
      goto cleanup;                                                    \
    }                                                                  \
  } while (0)

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// Carve from the slot arena, else allocate (the caller frees what it allocated).
hipError_t slot_alloc(capriv::DevArena& ar, void** p, size_t bytes, std::vector<void*>& extra) {
  const size_t at = al(ar.used);
  if (at + bytes <= ar.cap) {
    *p = ar.base + at;
    ar.used = at + bytes;
    return hipSuccess;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) extra.push_back(*p);
  return e;
}

void run_request(ca_server* srv, int slot, Request* req) {
  ca_ctx* ctx = srv->slot_ctx[slot];
  hipStream_t s = srv->slot_stream[slot];
  capriv::DevArena& arena = srv->slot_arena[slot];
  std::vector<void*> extra;  // allocations beyond the arena (rare)
  ca_clipset* rc = nullptr;
  void* buf = nullptr;
  const int64_t n = req->n;
  const int64_t p = srv->con.thr_num, q = srv->con.thr_den;
  std::vector<int32_t> lo(n), hi(n), anchors(n);
  std::vector<int64_t> roff(n), cnt, off;
  int64_t bits = 0, total = 0;
  std::vector<char> h_out;  // the pairs' result arrays, as laid out on the device
  const int32_t *h_rep = nullptr, *h_mem = nullptr;
  const uint8_t* h_bits = nullptr;
  const int16_t* h_shift = nullptr;
  const double* h_score = nullptr;
  // grow the slot's arena (only when a larger request than any before arrives)
  {
    const size_t want = (size_t)req->est_bytes;
    if (arena.cap < want) {
      if (arena.base) (void)hipFree(arena.base);
      arena.base = nullptr;
      arena.cap = 0;
      if (hipMalloc((void**)&arena.base, want) == hipSuccess) arena.cap = want;
    }
    arena.used = 0;
  }
  req->status = clips_create_in(ctx, s, n, req->rect_ptr.data(), req->rects.empty() ? nullptr : req->rects.data(),
                                req->raster_n.data(), req->marker_w.data(),
                                (has_fp32_of(srv->lib) ? CA_CLIPS_FP32 : 0u) |
                                    (has_fp64_of(srv->lib) ? 0u : CA_CLIPS_NO_FP64),
                                &arena, &rc);
  if (req->status != CA_OK) {
    req->error = ca_last_error(ctx);
    goto cleanup;
  }
  {
    // area-bound ranges in the library order (exact integer comparisons)
    const auto& np = hnpix_of(rc);
    const unsigned __int128 p2 = (unsigned __int128)(p * p), q2 = (unsigned __int128)(q * q);
    for (int64_t i = 0; i < n; ++i) {
      anchors[i] = (int32_t)i;
      const uint64_t ni = (uint64_t)np[i];
      auto first_true = [&](auto pred) {
        int64_t a = 0, b = (int64_t)srv->lib_n.size();
        while (a < b) {
          const int64_t m = (a + b) / 2;
          if (pred((uint64_t)srv->lib_n[m])) b = m;
          else a = m + 1;
        }
        return a;
      };
      // partners need n_b q^2 > p^2 n_i (smaller side) and n_i q^2 > p^2 n_b (larger side)
      int64_t l = first_true([&](uint64_t nb) { return (unsigned __int128)nb * q2 > p2 * ni; });
      int64_t h = first_true([&](uint64_t nb) { return !((unsigned __int128)ni * q2 > p2 * nb); });
      if (ni == 0 || h < l) h = l;
      lo[i] = (int32_t)l;
      hi[i] = (int32_t)h;
      roff[i] = bits;
      bits += h - l;
    }
  }
  {
    // a batch has few anchors and each a long library range: split the ranges
    // into segments of 64-partner chunks, about 2048 segments in all; counts
    // and write offsets are kept per (anchor, segment)
    int64_t longest = 0;
    for (int64_t i = 0; i < n; ++i) longest = std::max<int64_t>(longest, (int64_t)hi[i] - lo[i]);
    const int64_t seg = std::min<int64_t>(4096, std::max<int64_t>(64, (bits / 2048 + 63) / 64 * 64));
    const int64_t n_seg = std::max<int64_t>(1, (longest + seg - 1) / seg);
    const int64_t ns = n * n_seg;
    const size_t b_a = al(4 * (size_t)n), b_r = al(8 * (size_t)n), b_s = al(8 * (size_t)ns),
                 b_m = al(4 * (size_t)(bits / 32 + 1));
    RUN_HIP(slot_alloc(arena, &buf, 3 * b_a + b_r + 2 * b_s + b_m, extra));
    // the four range tables go over in one copy, laid out as on the device
    std::vector<char> stage(3 * b_a + b_r);
    std::memcpy(stage.data(), anchors.data(), 4 * n);
    std::memcpy(stage.data() + b_a, lo.data(), 4 * n);
    std::memcpy(stage.data() + 2 * b_a, hi.data(), 4 * n);
    std::memcpy(stage.data() + 3 * b_a, roff.data(), 8 * n);
    char* c = (char*)buf;
    int32_t* d_anchor = (int32_t*)c; c += b_a;
    int32_t* d_lo = (int32_t*)c; c += b_a;
    int32_t* d_hi = (int32_t*)c; c += b_a;
    int64_t* d_roff = (int64_t*)c; c += b_r;
    int64_t* d_cnt = (int64_t*)c; c += b_s;
    int64_t* d_off = (int64_t*)c; c += b_s;
    uint32_t* d_mask = (uint32_t*)c;
    RUN_HIP(hipMemcpyAsync(buf, stage.data(), stage.size(), hipMemcpyHostToDevice, s));
    RUN_HIP(hipMemsetAsync(d_mask, 0, b_m, s));
    // pairs are written as (batch clip, library clip): each batch clip's
    // candidates are consecutive, so the alignment kernel stages that clip once
    // as the fixed side and streams the library clips; direction 1 of a pair
    // is then the batch clip aligned to the library representative
    PruneArgs pa{srv->d_order, d_hi, n, d_cnt, nullptr, nullptr, nullptr, d_anchor, d_lo};
    const int64_t nl = (int64_t)srv->lib_order.size();
    pa.soa_row = srv->d_soa;
    pa.soa_col = srv->d_soa + 64 * nl;
    pa.soa_grp = srv->d_soa + 128 * nl;
    pa.soa_n = nl;
    pa.seg = (int)seg;
    pa.n_seg = (int)n_seg;
    const Threshold thr{p, q};
    RUN_HIP(launch_prune128(dev_of(rc), dev_of(srv->lib), pa, thr, d_roff, d_mask, false, s));
    cnt.resize(ns);
    off.resize(ns);
    RUN_HIP(hipMemcpyAsync(cnt.data(), d_cnt, 8 * ns, hipMemcpyDeviceToHost, s));
    RUN_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < ns; ++i) {
      off[i] = total;
      total += cnt[i];
    }
    req->candidates = total;
    if (total > 0) {
      void* out = nullptr;
      const size_t o4 = al(4 * (size_t)total), o1 = al((size_t)total), o8 = al(8 * (size_t)total),
                   o16 = al(16 * (size_t)total);
      RUN_HIP(slot_alloc(arena, &out, 2 * o4 + o1 + o8 + o8 + o16 + o4, extra));
      char* o = (char*)out;
      int32_t* d_rep = (int32_t*)o; o += o4;
      int32_t* d_mem = (int32_t*)o; o += o4;
      uint8_t* d_bits = (uint8_t*)o; o += o1;
      int16_t* d_shift = (int16_t*)o; o += o8;
      int32_t* d_count = (int32_t*)o; o += o8;
      double* d_score = (double*)o; o += o16;
      uint32_t* d_flags = (uint32_t*)o;
      RUN_HIP(hipMemcpyAsync(d_off, off.data(), 8 * ns, hipMemcpyHostToDevice, s));
      PruneArgs pw = pa;
      pw.counts = nullptr;
      pw.offs = d_off;
      pw.out_rep = d_rep;
      pw.out_mem = d_mem;
      hipError_t e = launch_prune128(dev_of(rc), dev_of(srv->lib), pw, thr, d_roff, d_mask, true, s);
      if (e == hipSuccess) {
        PairIO io{total, d_rep, d_mem, d_bits, d_shift, d_count, d_score, d_flags};
        req->status = align_cosine_sets(ctx, rc, srv->lib, s, thr, CA_PATH_MIXED, io);
        if (req->status != CA_OK) req->error = ca_last_error(ctx);
      } else {
        req->status = CA_EDEVICE;
        req->error = hipGetErrorString(e);
      }
      if (req->status == CA_OK) {
        // the result arrays (rep .. score) are contiguous: one copy back
        h_out.resize(2 * o4 + o1 + 2 * o8 + o16);
        hipError_t e1 = hipMemcpyAsync(h_out.data(), out, h_out.size(), hipMemcpyDeviceToHost, s);
        if (e1 == hipSuccess) e1 = hipStreamSynchronize(s);
        if (e1 != hipSuccess) {
          req->status = CA_EDEVICE;
          req->error = hipGetErrorString(e1);
        }
        h_rep = (const int32_t*)h_out.data();
        h_mem = (const int32_t*)(h_out.data() + o4);
        h_bits = (const uint8_t*)(h_out.data() + 2 * o4);
        h_shift = (const int16_t*)(h_out.data() + 2 * o4 + o1);
        h_score = (const double*)(h_out.data() + 2 * o4 + o1 + 2 * o8);
      }
      if (req->status != CA_OK) goto cleanup;
    }
  }
  // best covering representative per batch clip: pair k = (batch clip h_rep[k],
  // library clip h_mem[k]); direction 1 aligns the batch clip to the library clip
  req->best_rep.assign(n, -1);
  req->shift.assign(2 * n, 0);
  req->score.assign(n, 0.0);
  req->matched.assign(n, 0);
  for (int64_t k = 0; k < total; ++k) {
    if (!(h_bits[k] & 2)) continue;
    const int32_t i = h_rep[k], r = h_mem[k];
    const double sc = h_score[2 * k + 1];
    if (!req->matched[i] || sc > req->score[i] || (sc == req->score[i] && r < req->best_rep[i])) {
      req->matched[i] = 1;
      req->best_rep[i] = r;
      req->score[i] = sc;
      req->shift[2 * i] = h_shift[4 * k + 2];
      req->shift[2 * i + 1] = h_shift[4 * k + 3];
    }
  }
cleanup:
  if (rc) ca_clips_destroy(rc);
  for (void* x : extra) (void)hipFree(x);
}

void worker_main(ca_server* srv, int slot) {
  (void)hipSetDevice(device_of(srv->owner));
  for (;;) {
    Request* req = nullptr;
    {
      std::unique_lock<std::mutex> g(srv->mu);
      srv->cv_work.wait(g, [&] { return srv->stop || !srv->queue.empty(); });
      if (srv->stop && srv->queue.empty()) return;
      req = srv->queue.front();
      srv->queue.pop_front();
      req->state = 1;
    }
    run_request(srv, slot, req);
    ca_run_stats snap{};
    (void)ca_get_stats(srv->slot_ctx[slot], &snap);  // this worker is the slot context's only user
    {
      std::lock_guard<std::mutex> g(srv->mu);
      srv->slot_stats[slot] = snap;
      req->state = req->status == CA_OK ? 2 : 3;
      srv->inflight -= req->est_bytes;
      srv->done_requests += 1;
      srv->done_pairs += req->candidates;
    }
    srv->cv_done.notify_all();
  }
}

}  // namespace

extern "C" ca_status ca_server_create(ca_ctx* ctx, const ca_clipset* library, const ca_constraint* con,
                                      int32_t slots, uint64_t hbm_budget_bytes, ca_server** out) {
  if (!ctx) return CA_EINVAL;
  if (!library || ctx_of(library) != ctx || !con || !out || slots < 1 || slots > 32)
    return fail_ctx(ctx, CA_EINVAL, "bad server arguments");
  if (con->kind != CA_COSINE || con->edges != 0 || con->thr_den <= 0 || con->thr_num < 0 || con->thr_num > con->thr_den)
    return fail_ctx(ctx, CA_EUNSUPPORTED, "serving supports the cosine constraint");
  if (!mixed_ok_of(library))
    return fail_ctx(ctx, CA_EUNSUPPORTED, "serving needs a 128 x 128 library with half-windows <= 16");
  if (hipSetDevice(device_of(ctx)) != hipSuccess) return fail_ctx(ctx, CA_EDEVICE, "hipSetDevice failed");
  ca_server* srv = new ca_server();
  srv->owner = ctx;
  srv->lib = library;
  srv->con = *con;
  srv->budget = hbm_budget_bytes;
  const auto& np = hnpix_of(library);
  srv->lib_order.resize(n_of(library));
  for (int64_t i = 0; i < n_of(library); ++i) srv->lib_order[i] = (int32_t)i;
  std::sort(srv->lib_order.begin(), srv->lib_order.end(),
            [&](int32_t a, int32_t b) { return np[a] != np[b] ? np[a] < np[b] : a < b; });
  srv->lib_n.resize(srv->lib_order.size());
  for (size_t k = 0; k < srv->lib_order.size(); ++k) srv->lib_n[k] = np[srv->lib_order[k]];
  const int64_t nl = (int64_t)srv->lib_order.size();
  const size_t b_ord = (4 * (size_t)nl + 4 + 255) & ~(size_t)255;
  if (hipMalloc((void**)&srv->d_order, b_ord + 3 * 256 * (size_t)nl) != hipSuccess ||
      hipMemcpy(srv->d_order, srv->lib_order.data(), 4 * (size_t)nl, hipMemcpyHostToDevice) != hipSuccess ||
      (srv->d_soa = (uint32_t*)((char*)srv->d_order + b_ord),
       launch_prune128_soa(dev_of(library), srv->d_order, nl, srv->d_soa, srv->d_soa + 64 * nl,
                           srv->d_soa + 128 * nl, nullptr)) != hipSuccess ||
      hipStreamSynchronize(nullptr) != hipSuccess) {
    if (srv->d_order) (void)hipFree(srv->d_order);
    delete srv;
    return fail_ctx(ctx, CA_ENOMEM, "server library order upload failed");
  }
  // slot contexts check a small sample of decided pairs per request in FP64
  // (at most 128, none if the server's context checks none), so the check
  // adds little to a request's latency
  const int64_t chk = check_sample_of(ctx);
  ca_config cfg{device_of(ctx), chk <= 0 ? -1 : (int32_t)std::min<int64_t>(chk, 128), 0};
  for (int sl = 0; sl < slots; ++sl) {
    ca_ctx* sc = nullptr;
    hipStream_t st = nullptr;
    if (ca_create(&cfg, &sc) != CA_OK || hipStreamCreate(&st) != hipSuccess) {
      if (sc) ca_destroy(sc);
      for (size_t k = 0; k < srv->slot_ctx.size(); ++k) {
        ca_destroy(srv->slot_ctx[k]);
        (void)hipStreamDestroy(srv->slot_stream[k]);
      }
      (void)hipFree(srv->d_order);
      delete srv;
      return fail_ctx(ctx, CA_EDEVICE, "server slot set-up failed");
    }
    srv->slot_ctx.push_back(sc);
    srv->slot_stats.emplace_back();
    srv->slot_stream.push_back(st);
    srv->slot_arena.emplace_back();
  }
  for (int sl = 0; sl < slots; ++sl) srv->workers.emplace_back(worker_main, srv, sl);
  *out = srv;
  return CA_OK;
}

extern "C" ca_status ca_server_destroy(ca_server* srv) {
  if (!srv) return CA_EINVAL;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto& t : srv->workers) t.join();
  for (size_t k = 0; k < srv->slot_ctx.size(); ++k) {
    ca_destroy(srv->slot_ctx[k]);
    (void)hipStreamDestroy(srv->slot_stream[k]);
    if (srv->slot_arena[k].base) (void)hipFree(srv->slot_arena[k].base);
  }
  (void)hipFree(srv->d_order);
  for (auto& kv : srv->reqs) delete kv.second;
  delete srv;
  return CA_OK;
}

extern "C" ca_status ca_server_submit(ca_server* srv, int64_t n, const int64_t* rect_ptr, const int32_t* rects,
                                      const int16_t* raster_n, const int16_t* marker_w, uint64_t* req_id) {
  if (!srv) return CA_EINVAL;
  if (n <= 0 || n > (1 << 24) || !rect_ptr || !raster_n || !marker_w || !req_id)
    return srv_fail(srv, CA_EINVAL, "bad request arguments");
  if (rect_ptr[0] != 0) return srv_fail(srv, CA_EINVAL, "rect_ptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i) {
    if (rect_ptr[i + 1] < rect_ptr[i]) return srv_fail(srv, CA_EINVAL, "rect_ptr must be non-decreasing");
    if (raster_n[i] != 128 || marker_w[i] < 0 || marker_w[i] > 16)
      return srv_fail(srv, CA_EUNSUPPORTED, "requests need 128 x 128 clips with half-windows <= 16");
  }
  if (rect_ptr[n] > 0 && !rects) return srv_fail(srv, CA_EINVAL, "null rects");
  Request* req = new Request();
  req->n = n;
  req->est_bytes = estimate_bytes(n, has_fp32_of(srv->lib));
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->budget && srv->inflight + req->est_bytes > srv->budget) {
      srv->err = "admission refused: HBM budget in use";
      delete req;
      return CA_EBUSY;
    }
    srv->inflight += req->est_bytes;
  }
  req->rect_ptr.assign(rect_ptr, rect_ptr + n + 1);
  if (rect_ptr[n] > 0) req->rects.assign(rects, rects + 4 * rect_ptr[n]);
  req->raster_n.assign(raster_n, raster_n + n);
  req->marker_w.assign(marker_w, marker_w + n);
  {
    std::lock_guard<std::mutex> g(srv->mu);
    req->id = srv->next_id++;
    srv->reqs[req->id] = req;
    srv->queue.push_back(req);
  }
  srv->cv_work.notify_one();
  *req_id = req->id;
  return CA_OK;
}

extern "C" ca_status ca_server_poll(ca_server* srv, uint64_t req_id, int32_t* best_rep, int16_t* shift,
                                    double* score, uint8_t* matched, int32_t* done) {
  if (!srv || !done) return CA_EINVAL;
  Request* req = nullptr;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    auto it = srv->reqs.find(req_id);
    if (it == srv->reqs.end()) {
      srv->err = "unknown request id";
      return CA_EINVAL;
    }
    req = it->second;
    if (req->state < 2) {
      *done = 0;
      return CA_OK;
    }
    srv->reqs.erase(it);
  }
  *done = 1;
  ca_status st = req->status;
  if (st == CA_OK) {
    if (best_rep) std::memcpy(best_rep, req->best_rep.data(), 4 * req->n);
    if (shift) std::memcpy(shift, req->shift.data(), 4 * req->n);
    if (score) std::memcpy(score, req->score.data(), 8 * req->n);
    if (matched) std::memcpy(matched, req->matched.data(), req->n);
  } else {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->err = req->error;
  }
  delete req;
  return st;
}

extern "C" ca_status ca_server_wait(ca_server* srv, uint64_t req_id, int32_t timeout_ms) {
  if (!srv) return CA_EINVAL;
  std::unique_lock<std::mutex> g(srv->mu);
  auto ready = [&] {
    auto it = srv->reqs.find(req_id);
    return it == srv->reqs.end() || it->second->state >= 2;
  };
  if (timeout_ms < 0) srv->cv_done.wait(g, ready);
  else if (!srv->cv_done.wait_for(g, std::chrono::milliseconds(timeout_ms), ready)) return CA_EBUSY;
  return CA_OK;
}

extern "C" ca_status ca_server_stats(ca_server* srv, int64_t* requests_done, int64_t* candidate_pairs,
                                     uint64_t* inflight_bytes) {
  if (!srv) return CA_EINVAL;
  std::lock_guard<std::mutex> g(srv->mu);
  if (requests_done) *requests_done = srv->done_requests;
  if (candidate_pairs) *candidate_pairs = srv->done_pairs;
  if (inflight_bytes) *inflight_bytes = srv->inflight;
  return CA_OK;
}

extern "C" ca_status ca_server_run_stats(ca_server* srv, ca_run_stats* out) {
  if (!srv || !out) return CA_EINVAL;
  std::lock_guard<std::mutex> g(srv->mu);
  ca_run_stats t{};
  bool first = true;
  for (const ca_run_stats& a : srv->slot_stats) {
    if (first) {
      t = a;  // bands and other constants
      first = false;
      continue;
    }
    t.pairs_aligned += a.pairs_aligned;
    t.pairs_rescored += a.pairs_rescored;
    t.pairs_edge += a.pairs_edge;
    t.pairs_screened += a.pairs_screened;
    t.pairs_survived += a.pairs_survived;
    t.n_main_launch += a.n_main_launch;
    t.t_main_ms += a.t_main_ms;
    t.main_alg_bytes += a.main_alg_bytes;
    t.max_surface_err = std::max(t.max_surface_err, a.max_surface_err);
    t.max_peak_err_sqrt = std::max(t.max_peak_err_sqrt, a.max_peak_err_sqrt);
    t.groups_exact += a.groups_exact;
    t.pairs_full_fp64 += a.pairs_full_fp64;
    t.cover_nnz += a.cover_nnz;
    t.members_verified += a.members_verified;
    t.center_violations += a.center_violations;
    t.check_pairs += a.check_pairs;
    t.check_changed += a.check_changed;
    t.check_peak_err_sqrt = std::max(t.check_peak_err_sqrt, a.check_peak_err_sqrt);
    t.check_band_frac = std::max(t.check_band_frac, a.check_band_frac);
  }
  *out = t;
  return CA_OK;
}

extern "C" const char* ca_server_last_error(ca_server* srv) {
  if (!srv) return "";
  std::lock_guard<std::mutex> g(srv->mu);
  return srv->err.c_str();
}
