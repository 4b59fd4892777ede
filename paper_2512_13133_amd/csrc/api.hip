// Host runtime behind the C ABI in include/clipalign.h: contexts, device
// clip sets, pair alignment dispatch with the FP64 re-decision queue,
// candidate generation, and the set cover + closed loop on the host.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "host_internal.h"
#include "kernels.h"

using namespace ca;

// Bands under which a low-precision window peak is re-decided in FP64.  A band
// must exceed twice the path's worst surface error plus the tie tolerance.
// FP32: normalised surface units.  Mixed and direct (FP16 data): the error of
// K r grows like sqrt(K_hi), so the band is a coefficient of sqrt(K_hi) in
// units of K r.  With the split of T the worst error seen is 0.0065 sqrt(K_hi)
// (1.5M emulated workload candidate pairs and the worst of all 17.2M), so
// 0.03 covers twice it with a factor 2.3.
static constexpr double BAND_FP32 = 1e-5;
static constexpr double BAND_MIXED = 0.03;
static constexpr double BAND_DIRECT = 0.03;
// The general MFMA kernel's surface error in these units grows with the raster
// size (the FP16 twiddle roundings add up coherently along one axis, about
// sqrt(N)): the FP64 check of decided 256 x 256 pairs saw peak errors up to
// 0.019 sqrt(K_hi), so rasters above 128 take a band proportional to N.
static double band_mixed(int N) { return N > 128 ? BAND_MIXED * N / 128.0 : BAND_MIXED; }
// The direct-correlation kernel is built but not launched: its first GPU run
// ended in a memory-aperture fault whose cause is not yet identified, so the
// path reports CA_EUNSUPPORTED until it is.
static constexpr bool DIRECT_ENABLED = false;

struct ca_ctx {
  int device = 0;
  uint64_t budget = 0;
  int64_t check_sample = 1024;  // decided pairs per mixed call checked in FP64
  uint64_t used = 0;
  std::string err;
  ca_run_stats stats{};
  int live_clipsets = 0;
  float2* tw32 = nullptr;   // exp(-2 pi i m / 256), m < 128
  double2* tw64 = nullptr;
  // reusable per-call scratch
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  // on-demand FP64 spectra of sets without them: remap tables, then spectra
  void* fp64_tab = nullptr;
  size_t fp64_tab_bytes = 0;
  void* fp64_spec = nullptr;
  size_t fp64_spec_bytes = 0;
  // MFMA fragment tables of the mixed path (raster 128)
  void* mf_b1 = nullptr;
  void* mf_a2 = nullptr;
  // MFMA fragment tables of the mixed path for other raster sizes and windows,
  // by (raster code, window blocks): b1 then a2 in one allocation, made on first use
  void* gen_tab[3][6] = {};
  // HIP events bracketing the main alignment kernel
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  capriv::PruneCache prune_cache;
  capriv::CoverCache cover_cache;
  uint64_t next_gen = 1;
  std::map<int, capriv::TuneEntry> tune;  // autotuner choices by bucket key
};

struct ca_clipset {
  ca_ctx* ctx = nullptr;
  int64_t n = 0;
  int flags = 0;
  ClipsDev d{};
  std::vector<std::pair<void*, size_t>> owned;  // allocations freed by ca_clips_destroy
  capriv::DevArena* arena = nullptr;             // region the set was carved from (not owned)
  std::vector<int16_t> hN, hw;
  std::vector<int32_t> hnpix, hnpoly;
  int maxN = 0, minN = 1 << 30, Lmax = 0;
  bool mixed_ok = false;  // every clip is 128 x 128 with half-window <= 16
  int wmax = 0;           // largest half-window
  bool direct_ok = false; // whitened images kept, rasters <= 256, half-windows <= 7
  uint64_t gen = 0;       // unique per clip set within its context
};

static thread_local std::string g_create_err;
static constexpr int64_t CHECK_MAX = 4096;  // decided pairs checked in FP64 per call, at most
static hipError_t noalloc_setup(int device);  // allocation-free work array, per device

namespace {

ca_status fail(ca_ctx* ctx, ca_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  else g_create_err = msg;
  return st;
}

#define HIP_OR_FAIL(ctx, expr)                                                        \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail((ctx), CA_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

ca_status dev_alloc(ca_ctx* ctx, void** p, size_t bytes, std::vector<void*>* owner) {
  *p = nullptr;
  if (bytes == 0) return CA_OK;
  if (ctx->budget && ctx->used + bytes > ctx->budget)
    return fail(ctx, CA_ENOMEM, "allocation of " + std::to_string(bytes) + " bytes exceeds the HBM budget");
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(ctx, CA_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  ctx->used += bytes;
  if (owner) owner->push_back(*p);
  return CA_OK;
}

// Allocation for a clip set: carved from its arena when it has one and the
// request fits, else a device allocation the set owns.
ca_status cs_alloc(ca_ctx* ctx, ca_clipset* cs, void** p, size_t bytes) {
  if (bytes == 0) {
    *p = nullptr;
    return CA_OK;
  }
  if (cs->arena) {
    const size_t at = (cs->arena->used + 255) & ~(size_t)255;
    if (at + bytes <= cs->arena->cap) {
      *p = cs->arena->base + at;
      cs->arena->used = at + bytes;
      return CA_OK;
    }
  }
  std::vector<void*> tmp;
  ca_status st = dev_alloc(ctx, p, bytes, &tmp);
  if (st == CA_OK) cs->owned.emplace_back(*p, bytes);
  return st;
}

// Per-call scratch, grown on demand and kept on the context.
// Grow-only device buffer kept on the context.
ca_status grow_buffer(ca_ctx* ctx, void** buf, size_t* have, size_t bytes) {
  if (*have < bytes) {
    if (*buf) {
      (void)hipFree(*buf);
      ctx->used -= *have;
      *buf = nullptr;
      *have = 0;
    }
    const size_t want = std::max(bytes, (size_t)1 << 20);
    ca_status st = dev_alloc(ctx, buf, want, nullptr);
    if (st != CA_OK) return st;
    *have = want;
  }
  return CA_OK;
}

ca_status scratch(ca_ctx* ctx, size_t bytes, void** out) {
  if (ctx->scratch_bytes < bytes) {
    if (ctx->scratch) {
      (void)hipFree(ctx->scratch);
      ctx->used -= ctx->scratch_bytes;
      ctx->scratch = nullptr;
      ctx->scratch_bytes = 0;
    }
    size_t want = std::max(bytes, (size_t)1 << 20);
    ca_status st = dev_alloc(ctx, &ctx->scratch, want, nullptr);
    if (st != CA_OK) return st;
    ctx->scratch_bytes = want;
  }
  *out = ctx->scratch;
  return CA_OK;
}

int axis_len(int w, int N) { return (2 * w + 1 <= N) ? 2 * w + 1 : N; }

constexpr size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

bool valid_constraint(const ca_constraint* c) {
  if (!c) return false;
  if (c->kind == CA_COSINE) return c->edges == 0 && c->thr_num >= 0 && c->thr_den > 0 && c->thr_num <= c->thr_den &&
                                   c->thr_den <= (1 << 24);
  if (c->kind == CA_EDGE)
    return (c->edges == CA_EDGES_BOX || c->edges == CA_EDGES_CONTOUR) && c->thr_num >= 0 && c->thr_den == 1 &&
           c->thr_num < (1 << 20);
  return false;
}

}  // namespace

extern "C" {

ca_status ca_create(const ca_config* cfg, ca_ctx** out) {
  if (!cfg || !out) return fail(nullptr, CA_EINVAL, "null argument");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
    return fail(nullptr, CA_EDEVICE, "no HIP device visible");
  if (cfg->device < 0 || cfg->device >= ndev) return fail(nullptr, CA_EINVAL, "bad device ordinal");
  if (hipSetDevice(cfg->device) != hipSuccess) return fail(nullptr, CA_EDEVICE, "hipSetDevice failed");
  ca_ctx* ctx = new ca_ctx();
  ctx->device = cfg->device;
  ctx->budget = cfg->hbm_budget_bytes;
  ctx->check_sample = cfg->check_sample == 0 ? 1024 : (cfg->check_sample < 0 ? 0 : std::min<int64_t>(cfg->check_sample, CHECK_MAX));
  ctx->stats.tie_band_mixed = BAND_MIXED;
  ctx->stats.tie_band_fp32 = BAND_FP32;
  ctx->stats.tie_band_direct = BAND_DIRECT;
  std::vector<float2> t32(128);
  std::vector<double2> t64(128);
  for (int m = 0; m < 128; ++m) {
    const double a = -2.0 * M_PI * (double)m / 256.0;
    t64[m] = make_double2(std::cos(a), std::sin(a));
    t32[m] = make_float2((float)t64[m].x, (float)t64[m].y);
  }
  void* p32 = nullptr;
  void* p64 = nullptr;
  if (dev_alloc(ctx, &p32, sizeof(float2) * 128, nullptr) != CA_OK ||
      dev_alloc(ctx, &p64, sizeof(double2) * 128, nullptr) != CA_OK) {
    g_create_err = ctx->err;
    delete ctx;
    return CA_ENOMEM;
  }
  ctx->tw32 = (float2*)p32;
  ctx->tw64 = (double2*)p64;
  if (hipMemcpy(p32, t32.data(), sizeof(float2) * 128, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p64, t64.data(), sizeof(double2) * 128, hipMemcpyHostToDevice) != hipSuccess) {
    g_create_err = "twiddle upload failed";
    (void)hipFree(p32);
    (void)hipFree(p64);
    delete ctx;
    return CA_EDEVICE;
  }
  {
    std::vector<_Float16> b1(4 * 3 * 64 * 8), a2(8 * 3 * 64 * 8);
    build_mfma128_tables(b1.data(), a2.data());
    if (dev_alloc(ctx, &ctx->mf_b1, b1.size() * 2, nullptr) != CA_OK ||
        dev_alloc(ctx, &ctx->mf_a2, a2.size() * 2, nullptr) != CA_OK ||
        hipMemcpy(ctx->mf_b1, b1.data(), b1.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->mf_a2, a2.data(), a2.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
        hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess) {
      g_create_err = "context set-up failed";
      return CA_EDEVICE;
    }
  }
  {
    const hipError_t e = noalloc_setup(cfg->device);
    if (e != hipSuccess) {
      g_create_err = std::string("hipGetSymbolAddress of the allocation-free work array: ") + hipGetErrorString(e);
      return CA_EDEVICE;
    }
  }
  *out = ctx;
  return CA_OK;
}

ca_status ca_destroy(ca_ctx* ctx) {
  if (!ctx) return CA_EINVAL;
  if (ctx->live_clipsets) return fail(ctx, CA_ESTATE, "clip sets still alive on this context");
  (void)hipSetDevice(ctx->device);
  (void)hipFree(ctx->tw32);
  (void)hipFree(ctx->tw64);
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  if (ctx->fp64_tab) (void)hipFree(ctx->fp64_tab);
  if (ctx->fp64_spec) (void)hipFree(ctx->fp64_spec);
  if (ctx->mf_b1) (void)hipFree(ctx->mf_b1);
  if (ctx->mf_a2) (void)hipFree(ctx->mf_a2);
  for (auto& row : ctx->gen_tab)
    for (void* t : row)
      if (t) (void)hipFree(t);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->prune_cache.dev) (void)hipFree(ctx->prune_cache.dev);
  if (ctx->cover_cache.dev) (void)hipFree(ctx->cover_cache.dev);
  delete ctx;
  return CA_OK;
}

const char* ca_last_error(const ca_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

ca_status ca_get_stats(const ca_ctx* ctx, ca_run_stats* out) {
  if (!ctx || !out) return CA_EINVAL;
  *out = ctx->stats;
  return CA_OK;
}

ca_status ca_reset_stats(ca_ctx* ctx) {
  if (!ctx) return CA_EINVAL;
  ctx->stats = ca_run_stats{};
  ctx->stats.tie_band_mixed = BAND_MIXED;
  ctx->stats.tie_band_fp32 = BAND_FP32;
  ctx->stats.tie_band_direct = BAND_DIRECT;
  return CA_OK;
}

ca_status ca_clips_destroy(ca_clipset* cs) {
  if (!cs) return CA_EINVAL;
  (void)hipSetDevice(cs->ctx->device);
  if (cs->ctx->prune_cache.gen == cs->gen) cs->ctx->prune_cache.gen = 0;
  if (cs->ctx->cover_cache.gen == cs->gen) cs->ctx->cover_cache.gen = 0;
  for (auto& pb : cs->owned) {
    (void)hipFree(pb.first);
    cs->ctx->used -= pb.second;
  }
  cs->ctx->live_clipsets--;
  delete cs;
  return CA_OK;
}

ca_status ca_clips_count(const ca_clipset* cs, int64_t* n) {
  if (!cs || !n) return CA_EINVAL;
  *n = cs->n;
  return CA_OK;
}

static ca_status clips_create_impl(ca_ctx* ctx, void* stream, int64_t n, const int64_t* rect_ptr,
                                   const int32_t* rects, const int16_t* raster_n, const int16_t* marker_w,
                                   int32_t flags, capriv::DevArena* arena, ca_clipset** out) {
  if (!ctx) return CA_EINVAL;
  if (!out || !rect_ptr || !raster_n || !marker_w || n <= 0 || n > (1ll << 31) - 1)
    return fail(ctx, CA_EINVAL, "bad clip-set arguments");
  *out = nullptr;
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const bool on_dev = flags & CA_CLIPS_DEVICE_PTRS;
  std::vector<int64_t> hptr(n + 1);
  std::vector<int16_t> hN(n), hw(n);
  auto fetch = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (on_dev) return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
    std::memcpy(dst, src, bytes);
    return hipSuccess;
  };
  HIP_OR_FAIL(ctx, fetch(hptr.data(), rect_ptr, sizeof(int64_t) * (n + 1)));
  HIP_OR_FAIL(ctx, fetch(hN.data(), raster_n, sizeof(int16_t) * n));
  HIP_OR_FAIL(ctx, fetch(hw.data(), marker_w, sizeof(int16_t) * n));
  if (hptr[0] != 0) return fail(ctx, CA_EINVAL, "rect_ptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i) {
    if (hptr[i + 1] < hptr[i]) return fail(ctx, CA_EINVAL, "rect_ptr must be non-decreasing");
    if (hN[i] != 64 && hN[i] != 128 && hN[i] != 256)
      return fail(ctx, CA_EINVAL, "raster size must be 64, 128 or 256 (clip " + std::to_string(i) + ")");
    if (hw[i] < 0) return fail(ctx, CA_EINVAL, "marker half-window must be >= 0");
    if (axis_len(hw[i], hN[i]) > MAX_AXIS)
      return fail(ctx, CA_EUNSUPPORTED, "half-window above 32 px on a raster larger than 64");
  }
  const int64_t m = hptr[n];
  if (m > 0 && !rects) return fail(ctx, CA_EINVAL, "null rects");
  const bool no_fp64 = (flags & CA_CLIPS_NO_FP64) != 0;
  if (no_fp64) {
    if (flags & CA_CLIPS_IMAGE) return fail(ctx, CA_EUNSUPPORTED, "CA_CLIPS_NO_FP64 with CA_CLIPS_IMAGE");
    for (int64_t i = 0; i < n; ++i)
      if (hN[i] != 128) return fail(ctx, CA_EUNSUPPORTED, "CA_CLIPS_NO_FP64 needs 128 x 128 clips");
  }

  ca_clipset* cs = new ca_clipset();
  cs->ctx = ctx;
  cs->gen = ctx->next_gen++;
  cs->arena = arena;
  cs->n = n;
  cs->flags = no_fp64 ? flags : (flags | CA_CLIPS_FP64);  // FP64 spectra back the re-decision pass
  cs->hN = hN;
  cs->hw = hw;
  ctx->live_clipsets++;
  auto bail = [&](ca_status st) {
    ca_clips_destroy(cs);
    return st;
  };
  std::vector<int64_t> bits_off(n), sig_off(n), rowptr_off(n), spec_off(n), img_off(n);
  int64_t nb = 0, ns = 0, nr = 0, nsp = 0, nimg = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int N = hN[i];
    bits_off[i] = nb; nb += (int64_t)N * N / 64;
    sig_off[i] = ns; ns += N;
    rowptr_off[i] = nr; nr += N + 1;
    spec_off[i] = nsp; nsp += (int64_t)N * (N / 2 + 1);
    img_off[i] = nimg; nimg += (int64_t)N * N;
    cs->maxN = std::max(cs->maxN, N);
    cs->minN = std::min(cs->minN, N);
    cs->Lmax = std::max(cs->Lmax, axis_len(hw[i], N));
  }
  cs->mixed_ok = true;
  for (int64_t i = 0; i < n; ++i) {
    if (hN[i] != 128 || hw[i] > 16) cs->mixed_ok = false;
    cs->wmax = std::max<int>(cs->wmax, hw[i]);
  }
  const bool image = (flags & CA_CLIPS_IMAGE) != 0;
  cs->direct_ok = image;
  for (int64_t i = 0; i < n; ++i)
    if (hw[i] > 7) cs->direct_ok = false;
  void* p;
  ca_status st;
#define ALLOC(field, type, count)                                              \
  do {                                                                         \
    st = cs_alloc(ctx, cs, &p, sizeof(type) * (size_t)(count));                \
    if (st != CA_OK) return bail(st);                                          \
    cs->d.field = (type*)p;                                                    \
  } while (0)
  int16_t *dN, *dw;
  int64_t *dbo, *dso, *dro, *dspo, *drun_off;
  st = cs_alloc(ctx, cs, &p, sizeof(int16_t) * n); if (st) return bail(st); dN = (int16_t*)p;
  st = cs_alloc(ctx, cs, &p, sizeof(int16_t) * n); if (st) return bail(st); dw = (int16_t*)p;
  st = cs_alloc(ctx, cs, &p, sizeof(int64_t) * n); if (st) return bail(st); dbo = (int64_t*)p;
  st = cs_alloc(ctx, cs, &p, sizeof(int64_t) * n); if (st) return bail(st); dso = (int64_t*)p;
  st = cs_alloc(ctx, cs, &p, sizeof(int64_t) * n); if (st) return bail(st); dro = (int64_t*)p;
  st = cs_alloc(ctx, cs, &p, sizeof(int64_t) * n); if (st) return bail(st); dspo = (int64_t*)p;
  st = cs_alloc(ctx, cs, &p, sizeof(int64_t) * n); if (st) return bail(st); drun_off = (int64_t*)p;
  cs->d.n = n;
  cs->d.N = dN; cs->d.w = dw; cs->d.bits_off = dbo; cs->d.sig_off = dso;
  cs->d.rowptr_off = dro; cs->d.spec_off = dspo; cs->d.run_off = drun_off;
  ALLOC(bits, uint64_t, nb);
  ALLOC(npix, int32_t, n);
  ALLOC(rowsum, uint16_t, ns);
  ALLOC(colsum, uint16_t, ns);
  ALLOC(winrow, uint16_t, ns);
  ALLOC(wincol, uint16_t, ns);
  ALLOC(nruns, int32_t, n);
  ALLOC(npoly, int32_t, n);
  ALLOC(boxes, int16_t, n * MAX_POLY * 4);
  ALLOC(gbox, int16_t, n * 4);
  ALLOC(run_rowptr, uint16_t, nr);
  ALLOC(zero_bins, int32_t, n);
  ALLOC(spec16, __half2, nsp);
  if (flags & CA_CLIPS_FP32) ALLOC(spec32, float2, nsp);
  if (!no_fp64) ALLOC(spec64, double2, nsp);
  if (image) {
    int64_t* dio;
    st = cs_alloc(ctx, cs, &p, sizeof(int64_t) * n); if (st) return bail(st); dio = (int64_t*)p;
    cs->d.img_off = dio;
    ALLOC(img16, __half, nimg);
    HIP_OR_FAIL(ctx, hipMemcpyAsync(dio, img_off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
  }
  HIP_OR_FAIL(ctx, hipMemcpyAsync(dN, hN.data(), sizeof(int16_t) * n, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(dw, hw.data(), sizeof(int16_t) * n, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(dbo, bits_off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(dso, sig_off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(dro, rowptr_off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(dspo, spec_off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(ctx, hipMemsetAsync(cs->d.zero_bins, 0, sizeof(int32_t) * n, s));
  // inputs on the device
  const int64_t* d_ptr = rect_ptr;
  const int32_t* d_rects = rects;
  if (!on_dev) {  // inputs copied into the set's own memory (kept with the set)
    st = cs_alloc(ctx, cs, &p, sizeof(int64_t) * (n + 1)); if (st) return bail(st);
    d_ptr = (const int64_t*)p;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(p, rect_ptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
    if (m > 0) {
      st = cs_alloc(ctx, cs, &p, sizeof(int32_t) * 4 * m); if (st) return bail(st);
      d_rects = (const int32_t*)p;
      HIP_OR_FAIL(ctx, hipMemcpyAsync(p, rects, sizeof(int32_t) * 4 * m, hipMemcpyHostToDevice, s));
    }
  }
  HIP_OR_FAIL(ctx, launch_pack(d_ptr, d_rects, cs->d, n, s));
  std::vector<int32_t> nruns(n);
  HIP_OR_FAIL(ctx, hipMemcpyAsync(nruns.data(), cs->d.nruns, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  std::vector<int64_t> run_off(n);
  int64_t total_runs = 0;
  for (int64_t i = 0; i < n; ++i) {
    run_off[i] = total_runs;
    if (nruns[i] <= MAX_RUNS) total_runs += nruns[i];
  }
  ALLOC(runs, uint32_t, std::max<int64_t>(total_runs, 1));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(drun_off, run_off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(ctx, launch_label(cs->d, n, s));
  if (flags & CA_CLIPS_CONTOURS) {
    // contours: edges per clip, their offsets (host scan), then the walk
    ALLOC(cstat, int32_t, n);
    ALLOC(cpoly, uint16_t, n * (MAX_POLY + 1));
    ALLOC(chash, uint32_t, n * MAX_POLY);
    HIP_OR_FAIL(ctx, launch_contour_count(cs->d, cs->d.cstat, s));
    std::vector<int32_t> ne(n);
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ne.data(), cs->d.cstat, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
    std::vector<int64_t> eoff(n);
    int64_t total_edges = 0;
    for (int64_t i = 0; i < n; ++i) {
      eoff[i] = total_edges;
      total_edges += std::max(ne[i], 0);
    }
    int64_t* deo;
    st = cs_alloc(ctx, cs, &p, sizeof(int64_t) * n); if (st) return bail(st); deo = (int64_t*)p;
    cs->d.cedge_off = deo;
    ALLOC(cedges, uint16_t, std::max<int64_t>(total_edges, 1));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(deo, eoff.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
    HIP_OR_FAIL(ctx, launch_contour_trace(cs->d, cs->maxN, s));
  }
  // spectra per raster size, in batches through an FP64 scratch
  for (int N : {64, 128, 256}) {
    std::vector<int64_t> ids;
    for (int64_t i = 0; i < n; ++i)
      if (hN[i] == N) ids.push_back(i);
    if (ids.empty()) continue;
    if (N == 128 && !image) {
      // whole transform per workgroup, no scratch: one launch for all clips
      void* sc;
      st = scratch(ctx, align_up(sizeof(int64_t) * ids.size()), &sc);
      if (st) return bail(st);
      HIP_OR_FAIL(ctx, hipMemcpyAsync(sc, ids.data(), sizeof(int64_t) * ids.size(), hipMemcpyHostToDevice, s));
      HIP_OR_FAIL(ctx, launch_spectrum128(cs->d, (const int64_t*)sc, (int64_t)ids.size(), ctx->tw64, s));
      HIP_OR_FAIL(ctx, hipStreamSynchronize(s));  // scratch reuse
      continue;
    }
    const size_t per = (size_t)N * (N / 2 + 1) * sizeof(double2);
    const int64_t batch = std::max<int64_t>(1, std::min<int64_t>((int64_t)ids.size(), (512ll << 20) / (int64_t)per));
    void* sc;
    st = scratch(ctx, align_up(per * batch) + align_up(sizeof(int64_t) * batch), &sc);
    if (st) return bail(st);
    double2* sbuf = (double2*)sc;
    int64_t* dids = (int64_t*)((char*)sc + align_up(per * batch));
    for (int64_t b0 = 0; b0 < (int64_t)ids.size(); b0 += batch) {
      const int64_t nb2 = std::min<int64_t>(batch, (int64_t)ids.size() - b0);
      HIP_OR_FAIL(ctx, hipMemcpyAsync(dids, ids.data() + b0, sizeof(int64_t) * nb2, hipMemcpyHostToDevice, s));
      HIP_OR_FAIL(ctx, launch_spectrum(cs->d, dids, nb2, N, sbuf, ctx->tw64, s));
      if (image) HIP_OR_FAIL(ctx, launch_image(cs->d, dids, nb2, N, sbuf, ctx->tw64, s));
      HIP_OR_FAIL(ctx, hipStreamSynchronize(s));  // scratch reuse
    }
  }
  cs->hnpix.resize(n);
  cs->hnpoly.resize(n);
  HIP_OR_FAIL(ctx, hipMemcpyAsync(cs->hnpix.data(), cs->d.npix, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(cs->hnpoly.data(), cs->d.npoly, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
#undef ALLOC
  *out = cs;
  return CA_OK;
}

ca_status ca_clips_create(ca_ctx* ctx, void* stream, int64_t n, const int64_t* rect_ptr,
                          const int32_t* rects, const int16_t* raster_n, const int16_t* marker_w,
                          int32_t flags, ca_clipset** out) {
  return clips_create_impl(ctx, stream, n, rect_ptr, rects, raster_n, marker_w, flags, nullptr, out);
}

ca_status ca_clips_inspect(const ca_clipset* cs, int64_t i, uint64_t* bits, int32_t* n_pix,
                           uint16_t* rowsum, uint16_t* colsum, int32_t* n_poly, int16_t* boxes,
                           int32_t* zero_bins, float* spec16) {
  if (!cs) return CA_EINVAL;
  ca_ctx* ctx = cs->ctx;
  if (i < 0 || i >= cs->n) return fail(ctx, CA_EINVAL, "clip id out of range");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  const int N = cs->hN[i];
  std::vector<int64_t> off(4);
  HIP_OR_FAIL(ctx, hipMemcpy(&off[0], cs->d.bits_off + i, 8, hipMemcpyDeviceToHost));
  HIP_OR_FAIL(ctx, hipMemcpy(&off[1], cs->d.sig_off + i, 8, hipMemcpyDeviceToHost));
  HIP_OR_FAIL(ctx, hipMemcpy(&off[2], cs->d.spec_off + i, 8, hipMemcpyDeviceToHost));
  if (bits) HIP_OR_FAIL(ctx, hipMemcpy(bits, cs->d.bits + off[0], (size_t)N * N / 8, hipMemcpyDeviceToHost));
  if (n_pix) HIP_OR_FAIL(ctx, hipMemcpy(n_pix, cs->d.npix + i, 4, hipMemcpyDeviceToHost));
  if (rowsum) HIP_OR_FAIL(ctx, hipMemcpy(rowsum, cs->d.rowsum + off[1], 2 * N, hipMemcpyDeviceToHost));
  if (colsum) HIP_OR_FAIL(ctx, hipMemcpy(colsum, cs->d.colsum + off[1], 2 * N, hipMemcpyDeviceToHost));
  if (n_poly) HIP_OR_FAIL(ctx, hipMemcpy(n_poly, cs->d.npoly + i, 4, hipMemcpyDeviceToHost));
  if (boxes) HIP_OR_FAIL(ctx, hipMemcpy(boxes, cs->d.boxes + (size_t)i * MAX_POLY * 4, MAX_POLY * 8, hipMemcpyDeviceToHost));
  if (zero_bins) HIP_OR_FAIL(ctx, hipMemcpy(zero_bins, cs->d.zero_bins + i, 4, hipMemcpyDeviceToHost));
  if (spec16) {
    const int H = N / 2;
    std::vector<__half2> h((size_t)N * (H + 1));
    HIP_OR_FAIL(ctx, hipMemcpy(h.data(), cs->d.spec16 + off[2], sizeof(__half2) * h.size(), hipMemcpyDeviceToHost));
    for (int u = 0; u < N; ++u)
      for (int v = 0; v <= H; ++v) {
        const __half2 x = (v < H) ? h[(size_t)u * H + v] : h[(size_t)N * H + u];
        spec16[((size_t)u * (H + 1) + v) * 2 + 0] = __half2float(__low2half(x));
        spec16[((size_t)u * (H + 1) + v) * 2 + 1] = __half2float(__high2half(x));
      }
  }
  return CA_OK;
}

ca_status ca_clips_image(const ca_clipset* cs, int64_t i, float* img) {
  if (!cs || !img) return CA_EINVAL;
  ca_ctx* ctx = cs->ctx;
  if (i < 0 || i >= cs->n) return fail(ctx, CA_EINVAL, "clip id out of range");
  if (!cs->d.img16) return fail(ctx, CA_ESTATE, "clip set created without CA_CLIPS_IMAGE");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  const int N = cs->hN[i];
  int64_t off = 0;
  HIP_OR_FAIL(ctx, hipMemcpy(&off, cs->d.img_off + i, 8, hipMemcpyDeviceToHost));
  std::vector<__half> h((size_t)N * N);
  HIP_OR_FAIL(ctx, hipMemcpy(h.data(), cs->d.img16 + off, sizeof(__half) * h.size(), hipMemcpyDeviceToHost));
  for (size_t t = 0; t < h.size(); ++t) img[t] = __half2float(h[t]);
  return CA_OK;
}

ca_status ca_clips_spectrum(const ca_clipset* cs, int64_t i, int32_t precision, double* out) {
  if (!cs || !out) return CA_EINVAL;
  ca_ctx* ctx = cs->ctx;
  if (i < 0 || i >= cs->n) return fail(ctx, CA_EINVAL, "clip id out of range");
  if (precision != 16 && precision != 32 && precision != 64) return fail(ctx, CA_EINVAL, "precision 16, 32 or 64");
  if (precision == 32 && !cs->d.spec32) return fail(ctx, CA_ESTATE, "clip set created without CA_CLIPS_FP32");
  if (precision == 64 && !cs->d.spec64) return fail(ctx, CA_ESTATE, "clip set without FP64 spectra");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  const int N = cs->hN[i], H = N / 2 + 1;
  int64_t off = 0;
  HIP_OR_FAIL(ctx, hipMemcpy(&off, cs->d.spec_off + i, 8, hipMemcpyDeviceToHost));
  const size_t nb = (size_t)N * H;
  if (precision == 64) {
    HIP_OR_FAIL(ctx, hipMemcpy(out, cs->d.spec64 + off, sizeof(double2) * nb, hipMemcpyDeviceToHost));
  } else if (precision == 32) {
    std::vector<float2> h(nb);
    HIP_OR_FAIL(ctx, hipMemcpy(h.data(), cs->d.spec32 + off, sizeof(float2) * nb, hipMemcpyDeviceToHost));
    for (size_t t = 0; t < nb; ++t) {
      out[2 * t] = h[t].x;
      out[2 * t + 1] = h[t].y;
    }
  } else {
    // FP16 layout: [u][v < N/2], then the Nyquist column [u]
    std::vector<__half2> h(nb);
    HIP_OR_FAIL(ctx, hipMemcpy(h.data(), cs->d.spec16 + off, sizeof(__half2) * nb, hipMemcpyDeviceToHost));
    for (int u = 0; u < N; ++u)
      for (int v = 0; v < H; ++v) {
        const __half2 z = v < N / 2 ? h[(size_t)u * (N / 2) + v] : h[(size_t)N * (N / 2) + u];
        out[2 * ((size_t)u * H + v)] = __low2float(z);
        out[2 * ((size_t)u * H + v) + 1] = __high2float(z);
      }
  }
  return CA_OK;
}

ca_status ca_clips_contours(const ca_clipset* cs, int64_t i, int32_t* n_edges, uint16_t* edges, int64_t cap,
                            uint16_t* poly_ptr, uint32_t* hashes) {
  if (!cs) return CA_EINVAL;
  ca_ctx* ctx = cs->ctx;
  if (i < 0 || i >= cs->n) return fail(ctx, CA_EINVAL, "clip id out of range");
  if (!cs->d.cstat) return fail(ctx, CA_ESTATE, "clip set created without CA_CLIPS_CONTOURS");
  if (cap < 0) return fail(ctx, CA_EINVAL, "negative capacity");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  int32_t ne = 0;
  int64_t off = 0;
  HIP_OR_FAIL(ctx, hipMemcpy(&ne, cs->d.cstat + i, 4, hipMemcpyDeviceToHost));
  HIP_OR_FAIL(ctx, hipMemcpy(&off, cs->d.cedge_off + i, 8, hipMemcpyDeviceToHost));
  if (n_edges) *n_edges = ne;
  if (poly_ptr)
    HIP_OR_FAIL(ctx, hipMemcpy(poly_ptr, cs->d.cpoly + i * (MAX_POLY + 1), 2 * (MAX_POLY + 1), hipMemcpyDeviceToHost));
  if (hashes) HIP_OR_FAIL(ctx, hipMemcpy(hashes, cs->d.chash + i * MAX_POLY, 4 * MAX_POLY, hipMemcpyDeviceToHost));
  if (edges && ne > 0) {
    if (cap < ne) return fail(ctx, CA_ETRUNC, "edge buffer too small");
    HIP_OR_FAIL(ctx, hipMemcpy(edges, cs->d.cedges + off, 2 * (size_t)ne, hipMemcpyDeviceToHost));
  }
  return CA_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ alignment

namespace {

// flag: a device word for the result (null: the context's scratch), cleared
// here by a kernel.
ca_status validate_pairs(ca_ctx* ctx, const ca_clipset* crs, const ca_clipset* cms, hipStream_t s,
                         int64_t n_pairs, const int32_t* rep, const int32_t* mem, int need_poly,
                         unsigned long long* flag = nullptr) {
  if (!flag) {
    void* sc;
    ca_status st = scratch(ctx, 256, &sc);
    if (st) return st;
    flag = (unsigned long long*)sc;
  }
  int* bad = (int*)flag;
  HIP_OR_FAIL(ctx, launch_zero_u64(flag, 1, s));
  HIP_OR_FAIL(ctx, launch_validate(crs->d, cms->d, n_pairs, rep, mem, need_poly, bad, s));
  int hbad = 0;
  HIP_OR_FAIL(ctx, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  if (hbad & 1) return fail(ctx, CA_EINVAL, "pair list has an out-of-range id or unequal raster sizes");
  if (hbad & 2) return fail(ctx, CA_EUNSUPPORTED, "edge track on a clip with more than 64 polygons");
  if (hbad & 4)
    return fail(ctx, CA_EUNSUPPORTED, "full-edge track on a clip with more than 4,096 boundary edges");
  return CA_OK;
}

// Algorithmic bytes of the FP32 per-pair kernel: both FP32 half-spectra and both bit rasters.
double io_bytes_fp32(int maxN, int64_t n) {
  const double N = maxN;
  return (double)n * (2.0 * N * (N / 2 + 1) * 8.0 + 2.0 * N * N / 8.0);
}

struct FftPlan {
  int CH, LINES;
  size_t smem;
};

FftPlan plan_fft(int N, int L, int scalar_bytes) {
  const size_t budget = 150 * 1024;
  FftPlan p;
  p.LINES = N <= 64 ? 16 : 8;  // at least 512 butterflies between barriers
  const size_t c = 2 * (size_t)scalar_bytes;
  const size_t fixed = (size_t)p.LINES * N * c + (size_t)L * L * scalar_bytes;
  int ch = (int)((budget - fixed) / ((size_t)N * c));
  p.CH = std::max(1, std::min(L, ch));
  p.smem = pcm_fft_smem(scalar_bytes, N, p.CH, p.LINES, L);
  return p;
}

}  // namespace

// Queue storage of the low-precision paths for n pairs: need[n], list[n],
// r1_low[2n], 32 counters (0 queued pairs, 1 max error bits, 2 candidate
// groups, 3 candidate shifts, 4 tile counter, 5 error ratio bits, 8 groups
// left by the FP32 screen, 10 checked decided pairs, 11 / 12 their peak error
// bits (as 1 / 5), 13 their changed answers, rest spare), candidate groups,
// their shifts, the groups left by the screen, and the list and saved results
// of the decided pairs checked in FP64 (at most CHECK_MAX a call).
struct QueueMem {
  RescoreQueue q;
  CandQueue cq;
  CandQueue exact;  // groups the FP32 screen leaves to the FP64 pass (cq's shifts)
  unsigned long long* counters;
  RescoreQueue check;  // the sample of decided pairs: q's need and r1_low, its own list and counters
  SampleSave* check_saved;
  int32_t* sel;              // pairs a queue-free first pass leaves undecided (batched kernel)
  unsigned long long* n_sel;
};
static constexpr size_t queue_bytes(int64_t n) {
  const int64_t cap_g = n / 4 + 65536, cap_s = 16 * cap_g;
  return align_up(n) + 2 * align_up(8 * (size_t)n) + 256 + 2 * align_up(sizeof(CandGroup) * (size_t)cap_g) +
         align_up(2 * (size_t)cap_s) + align_up(8 * (size_t)CHECK_MAX) + align_up(sizeof(SampleSave) * (size_t)CHECK_MAX) +
         align_up(4 * (size_t)n);
}
static QueueMem queue_carve(char* base, int64_t n) {
  const int64_t cap_g = n / 4 + 65536, cap_s = 16 * cap_g;
  const size_t b_need = align_up(n), b_list = align_up(8 * (size_t)n), b_r1 = align_up(8 * (size_t)n);
  const size_t b_cnt = 256, b_grp = align_up(sizeof(CandGroup) * (size_t)cap_g);
  QueueMem m;
  m.q.need = (uint8_t*)base;
  m.q.list = (int64_t*)(base + b_need);
  m.q.r1_low = (float*)(base + b_need + b_list);
  m.counters = (unsigned long long*)(base + b_need + b_list + b_r1);
  m.q.len = m.counters;
  m.q.peak_err_bits = m.counters + 1;
  m.q.peak_ratio_bits = m.counters + 5;
  m.cq.n_groups = m.counters + 2;
  m.cq.n_shifts = m.counters + 3;
  m.cq.groups = (CandGroup*)(base + b_need + b_list + b_r1 + b_cnt);
  m.cq.shifts = (int16_t*)(base + b_need + b_list + b_r1 + b_cnt + b_grp);
  m.cq.cap_groups = cap_g;
  m.cq.cap_shifts = cap_s;
  m.exact = m.cq;
  m.exact.groups = (CandGroup*)(base + b_need + b_list + b_r1 + b_cnt + b_grp + align_up(2 * (size_t)cap_s));
  m.exact.n_groups = m.counters + 8;
  m.exact.n_shifts = nullptr;
  char* chk = base + b_need + b_list + b_r1 + b_cnt + 2 * b_grp + align_up(2 * (size_t)cap_s);
  m.check = m.q;
  m.check.list = (int64_t*)chk;
  m.check.len = m.counters + 10;
  m.check.peak_err_bits = m.counters + 11;
  m.check.peak_ratio_bits = m.counters + 12;
  m.check_saved = (SampleSave*)(chk + align_up(8 * (size_t)CHECK_MAX));
  m.sel = (int32_t*)(chk + align_up(8 * (size_t)CHECK_MAX) + align_up(sizeof(SampleSave) * (size_t)CHECK_MAX));
  m.n_sel = m.counters + 6;
  return m;
}

// Allocation-free alignment (ca_align_pairs_noalloc): the queue of up to
// CA_NOALLOC_MAX_PAIRS pairs and a validation word live in one static device
// array, which each device holds from the library's first use on it until the
// process ends.  Host code never names the array in a kernel argument or a
// copy: it uses the device address taken once per device at context creation.
static constexpr size_t NOALLOC_QUEUE_BYTES = queue_bytes(CA_NOALLOC_MAX_PAIRS);
static constexpr size_t NOALLOC_BYTES = NOALLOC_QUEUE_BYTES + 256;
static __device__ __align__(256) char g_noalloc_scratch[NOALLOC_BYTES];
static constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_noalloc_mu;
static char* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// With `device` current: look up the array's address on it (once per device).
static hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_noalloc_scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_noalloc_ptr[device] = (char*)p;
  return hipSuccess;
}

static char* noalloc_base(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  return g_noalloc_ptr[device];
}

// The device sequence of a low-precision path (CA_PATH_FP32 or CA_PATH_MIXED):
// counters cleared by a kernel, the main surface kernel (bracketed by the
// context's events when `events`), then the FP64 re-decision sized on the
// device.  No host synchronisation, so it can be captured in a graph.
// The fragment tables of the general MFMA kernel for (N, NB), built on the
// host in FP64 and uploaded on first use (a few hundred KB at most).
static ca_status ensure_gen_tables(ca_ctx* ctx, int N, int NB) {
  void*& t = ctx->gen_tab[N == 64 ? 0 : (N == 128 ? 1 : 2)][NB];
  if (t) return CA_OK;
  std::vector<_Float16> tab(mfma_gen_table_halves(N, NB));
  build_mfma_gen_tables(N, NB, tab.data(), tab.data() + (size_t)(N / 32) * NB * 64 * 8);
  void* p = nullptr;
  ca_status st = dev_alloc(ctx, &p, tab.size() * 2, nullptr);
  if (st) return st;
  const hipError_t e = hipMemcpy(p, tab.data(), tab.size() * 2, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(p);
    ctx->used -= tab.size() * 2;
    return fail(ctx, CA_EDEVICE, std::string("fragment table upload: ") + hipGetErrorString(e));
  }
  t = p;
  return CA_OK;
}

// Decided pairs of an n-pair mixed call checked on the full FP64 surface: the
// context's check_sample, at most one pair in 256 of the call (so that small
// calls and graph replays stay cheap), none when switched off.
static int64_t check_count(const ca_ctx* ctx, int64_t n) {
  return ctx->check_sample > 0 ? std::min<int64_t>(ctx->check_sample, std::max<int64_t>(1, n / 256)) : 0;
}

// gen_nb > 0: CA_PATH_MIXED runs the general MFMA kernel on raster maxN with
// gen_nb x gen_nb window blocks (0: the 128 x 128 kernel for half-windows <= 16).
// check_n > 0: after the re-decision, up to check_n decided pairs are checked
// against the full FP64 surface (QueueMem::check).
static hipError_t enqueue_cosine(ca_ctx* ctx, const ClipsDev& cr, const ClipsDev& cm, int maxN, int Lmax, int path,
                                 Threshold thr, const PairIO& io, const QueueMem& m, hipStream_t s, bool events,
                                 int direct_n = 0, bool fp64_pass = true, int gen_nb = 0, int64_t check_n = 0) {
  const int64_t n = io.n_pairs;
  hipError_t e = launch_zero_u64(m.counters, 32, s);
  if (e != hipSuccess) return e;
  if (events && (e = hipEventRecord(ctx->ev0, s)) != hipSuccess) return e;
  if (path == CA_PATH_FP32) {
    FftPlan pl = plan_fft(maxN, Lmax, 4);
    e = launch_pcm_fft32(cr, cm, io, nullptr, n, MODE_LOW, thr, BAND_FP32, ctx->tw32, pl.CH, pl.LINES, Lmax, maxN,
                         m.q, s);
  } else if (path == CA_PATH_DIRECT) {
    e = launch_pcm_direct(cr, cm, io, direct_n, thr, (float)BAND_DIRECT, m.q, m.cq, nullptr, m.counters + 4, s);
  } else if (gen_nb > 0) {
    const _Float16* tab = (const _Float16*)ctx->gen_tab[maxN == 64 ? 0 : (maxN == 128 ? 1 : 2)][gen_nb];
    if (!tab) return hipErrorNotInitialized;  // made by ensure_gen_tables before any launch
    e = launch_pcm_mfma_gen(maxN, gen_nb, cr, cm, io, thr, (float)band_mixed(maxN), m.q, m.cq, tab,
                            tab + (size_t)(maxN / 32) * gen_nb * 64 * 8, m.counters + 4, m.sel, m.n_sel, s);
  } else {
    e = launch_pcm_mfma128(cr, cm, io, thr, (float)BAND_MIXED, m.q, m.cq, ctx->mf_b1, ctx->mf_a2, nullptr,
                           m.counters + 4, s);
  }
  if (e != hipSuccess) return e;
  if (events && (e = hipEventRecord(ctx->ev1, s)) != hipSuccess) return e;
  if (!fp64_pass) {
    // sets without FP64 spectra: only the FP32 screen here; the rest runs on
    // demand once the host knows which clips it needs
    if (cr.spec32 && cm.spec32)
      return launch_rescore_screen(cr, cm, io, thr, m.cq, m.exact, ctx->tw64, m.q.peak_err_bits,
                                   m.q.peak_ratio_bits, m.q.r1_low, s);
    return hipSuccess;
  }
  // FP64 re-decision: the candidate groups, then the full FP64 surface of the
  // pairs queued for it
  e = launch_rescore_candidates(cr, cm, io, thr, m.cq, m.exact, ctx->tw64, m.q.peak_err_bits, m.q.peak_ratio_bits,
                                m.q.r1_low, s);
  if (e != hipSuccess) return e;
  FftPlan pl = plan_fft(maxN, Lmax, 8);
  e = launch_pcm_fft64(cr, cm, io, m.q.list, n, MODE_RESCORE, thr, 0.0, ctx->tw64, pl.CH, pl.LINES, Lmax, maxN, m.q,
                       s, m.q.len);
  if (e != hipSuccess || check_n <= 0) return e;
  const int64_t cn = std::min(check_n, std::min(n, CHECK_MAX));
  e = launch_sample_pick(n, cn, io, m.q.need, m.check.list, m.check.len, m.check_saved, s);
  if (e == hipSuccess)
    e = launch_pcm_fft64(cr, cm, io, m.check.list, cn, MODE_RESCORE, thr, 0.0, ctx->tw64, pl.CH, pl.LINES, Lmax, maxN,
                         m.check, s, m.check.len);
  if (e == hipSuccess)
    e = launch_sample_compare(cn, m.check.list, m.check.len, m.check_saved, io, m.q.need, m.counters + 13, s);
  return e;
}

// FP64 re-decision for clip sets without stored FP64 spectra: after the main
// kernel (and the FP32 screen) the groups and pairs still to re-decide are
// known; their clips are collected on the device (each once, in a per-set
// table mapping clip -> slot), their FP64 spectra computed into a buffer on
// the context, and the FP64 passes run on views whose FP64 spectra and offsets
// point there.  h: the queue counters already read back.
static ca_status fp64_on_demand(ca_ctx* ctx, const ca_clipset* crs, const ca_clipset* cms, hipStream_t s,
                                Threshold thr, const PairIO& io, const QueueMem& qm, const unsigned long long* h,
                                int maxN, int Lmax) {
  const ClipsDev& cr = crs->d;
  const ClipsDev& cm = cms->d;
  const bool screened = cr.spec32 && cm.spec32;
  const CandQueue& groups = screened ? qm.exact : qm.cq;
  const int64_t n_groups = std::min<int64_t>((int64_t)(screened ? h[8] : h[2]), groups.cap_groups);
  const int64_t n_full = (int64_t)h[0];
  if (n_groups == 0 && n_full == 0) return CA_OK;
  const bool same = crs == cms;
  const int64_t nr = crs->n, nm = same ? 0 : cms->n;
  const size_t b_r = align_up(8 * (size_t)nr), b_m = align_up(8 * (size_t)nm);
  ca_status st = grow_buffer(ctx, &ctx->fp64_tab, &ctx->fp64_tab_bytes, 2 * b_r + 2 * b_m + 256);
  if (st) return st;
  char* t = (char*)ctx->fp64_tab;
  int64_t* remap_r = (int64_t*)t;
  int64_t* ids_r = (int64_t*)(t + b_r);
  int64_t* remap_m = same ? remap_r : (int64_t*)(t + 2 * b_r);
  int64_t* ids_m = same ? ids_r : (int64_t*)(t + 2 * b_r + b_m);
  unsigned long long* cnt = (unsigned long long*)(t + 2 * b_r + 2 * b_m);
  constexpr int64_t PER = 128 * 65;  // FP64 half-spectrum of a 128 x 128 clip, in double2
  HIP_OR_FAIL(ctx, hipMemsetAsync(remap_r, 0xff, 8 * (size_t)nr, s));
  if (!same) HIP_OR_FAIL(ctx, hipMemsetAsync(remap_m, 0xff, 8 * (size_t)nm, s));
  HIP_OR_FAIL(ctx, launch_zero_u64(cnt, 2, s));
  HIP_OR_FAIL(ctx, launch_mark_fp64(io, groups.groups, n_groups, qm.q.list, n_full, remap_r, ids_r, cnt, remap_m,
                                    ids_m, same ? cnt : cnt + 1, PER, s));
  unsigned long long hc[2] = {0, 0};
  HIP_OR_FAIL(ctx, hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  const int64_t kr = (int64_t)hc[0], km = same ? 0 : (int64_t)hc[1];
  st = grow_buffer(ctx, &ctx->fp64_spec, &ctx->fp64_spec_bytes, sizeof(double2) * (size_t)PER * (size_t)(kr + km));
  if (st) return st;
  double2* spec_r = (double2*)ctx->fp64_spec;
  double2* spec_m = same ? spec_r : spec_r + PER * kr;
  // views for the spectrum writes (FP64 only, at the remapped offsets) and for the FP64 passes
  auto write_view = [](ClipsDev v, double2* spec, const int64_t* remap) {
    v.spec16 = nullptr;
    v.spec32 = nullptr;
    v.spec64 = spec;
    v.spec_off = remap;
    v.zero_bins = nullptr;
    return v;
  };
  auto read_view = [](ClipsDev v, double2* spec, const int64_t* remap) {
    v.spec64 = spec;
    v.spec_off = remap;
    return v;
  };
  HIP_OR_FAIL(ctx, launch_spectrum128(write_view(cr, spec_r, remap_r), ids_r, kr, ctx->tw64, s));
  if (!same) HIP_OR_FAIL(ctx, launch_spectrum128(write_view(cm, spec_m, remap_m), ids_m, km, ctx->tw64, s));
  const ClipsDev vr = read_view(cr, spec_r, remap_r), vm = read_view(cm, spec_m, remap_m);
  HIP_OR_FAIL(ctx, launch_rescore_exact(vr, vm, io, thr, groups, ctx->tw64, qm.q.peak_err_bits, qm.q.peak_ratio_bits,
                                        qm.q.r1_low, s));
  FftPlan pl = plan_fft(maxN, Lmax, 8);
  HIP_OR_FAIL(ctx, launch_pcm_fft64(vr, vm, io, qm.q.list, io.n_pairs, MODE_RESCORE, thr, 0.0, ctx->tw64, pl.CH,
                                    pl.LINES, Lmax, maxN, qm.q, s, qm.q.len));
  return CA_OK;
}

// Cosine alignment of a device pair list with the chosen path (no validation).
// `checked`: the caller guarantees that every pair suits the path (the
// autotuner's buckets), so the set-wide shape tests of CA_PATH_MIXED and
// CA_PATH_DIRECT are skipped; `direct_n` then names the bucket's raster size
// and `bucket_w` bounds its half-windows, so the per-pair FFT kernels are
// planned (LDS per workgroup) for the bucket rather than for the whole set.
// `qmem`: queue memory of at least queue_bytes(n) bytes supplied by the caller
// (null: the context's scratch, grown on demand).
static ca_status align_cosine(ca_ctx* ctx, const ca_clipset* crs, const ca_clipset* cms, hipStream_t s,
                              Threshold thr, int path, const PairIO& io, bool checked = false, int direct_n = 0,
                              int bucket_w = 1 << 20, char* qmem = nullptr) {
  int maxN = std::max(crs->maxN, cms->maxN), Lmax = std::max(crs->Lmax, cms->Lmax);
  if (checked && direct_n > 0) {
    maxN = direct_n;
    Lmax = std::min(Lmax, axis_len(bucket_w, direct_n));
  }
  const ClipsDev& cr = crs->d;
  const ClipsDev& cm = cms->d;
  const int64_t n = io.n_pairs;
  const RescoreQueue none{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (path == CA_PATH_XYSEP) {
    if (crs != cms) return fail(ctx, CA_EUNSUPPORTED, "CA_PATH_XYSEP aligns pairs within one clip set");
    HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev0, s));
    HIP_OR_FAIL(ctx, launch_xysep(cr, io, thr, s));
    HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev1, s));
    HIP_OR_FAIL(ctx, hipEventSynchronize(ctx->ev1));
    float ms = 0.f;
    HIP_OR_FAIL(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->stats.t_main_ms += ms;
    ctx->stats.n_main_launch += 1;
    ctx->stats.pairs_aligned += n;
    return CA_OK;
  }
  const bool on_demand = !cr.spec64 || !cm.spec64;
  if (on_demand && path != CA_PATH_MIXED && path != CA_PATH_FP32)
    return fail(ctx, CA_EUNSUPPORTED, "this path needs FP64 spectra (clip set made with CA_CLIPS_NO_FP64)");
  if (path == CA_PATH_FP64) {
    FftPlan pl = plan_fft(maxN, Lmax, 8);
    HIP_OR_FAIL(ctx, launch_pcm_fft64(cr, cm, io, nullptr, n, MODE_EXACT, thr, 0.0, ctx->tw64, pl.CH,
                                      pl.LINES, Lmax, maxN, none, s));
    ctx->stats.pairs_aligned += n;
    return CA_OK;
  }
  if (path == CA_PATH_XCORR) {
    if (maxN > 128 || Lmax > 33)
      return fail(ctx, CA_EUNSUPPORTED, "CA_PATH_XCORR needs rasters of 64 or 128 and half-windows <= 16");
    HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev0, s));
    for (int N : {64, 128})
      if (std::min(crs->minN, cms->minN) <= N && N <= maxN) HIP_OR_FAIL(ctx, launch_xcorr(cr, cm, io, N, thr, s));
    HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev1, s));
    HIP_OR_FAIL(ctx, hipEventSynchronize(ctx->ev1));
    float ms = 0.f;
    HIP_OR_FAIL(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->stats.t_main_ms += ms;
    ctx->stats.n_main_launch += 1;
    ctx->stats.pairs_aligned += n;
    return CA_OK;
  }
  if (path == CA_PATH_FP32 && (!cr.spec32 || !cm.spec32))
    return fail(ctx, CA_ESTATE, "CA_PATH_FP32 needs a clip set created with CA_CLIPS_FP32");
  // CA_PATH_MIXED: the 128 x 128 kernel for half-windows <= 16, else the
  // general kernel with enough window blocks for the largest half-window
  int gen_nb = 0;
  if (path == CA_PATH_MIXED) {
    int N = maxN, wb = std::max(crs->wmax, cms->wmax);
    if (checked && direct_n > 0) {
      N = direct_n;
      wb = bucket_w;
    } else if (!(crs->mixed_ok && cms->mixed_ok) &&
               (crs->minN != crs->maxN || cms->minN != cms->maxN || crs->maxN != cms->maxN)) {
      return fail(ctx, CA_EUNSUPPORTED, "CA_PATH_MIXED needs clip sets of one raster size (CA_PATH_AUTO mixes sizes)");
    }
    if (N > 64) wb = std::min(wb, 32);
    if (!(N == 128 && wb <= 16)) {
      gen_nb = mfma_gen_blocks(N, wb);
      if (gen_nb <= 0) return fail(ctx, CA_EUNSUPPORTED, "CA_PATH_MIXED: half-window above 32");
      maxN = N;
      ca_status st = ensure_gen_tables(ctx, N, gen_nb);
      if (st) return st;
    }
  }
  if (path == CA_PATH_DIRECT) {
    if (!DIRECT_ENABLED) return fail(ctx, CA_EUNSUPPORTED, "CA_PATH_DIRECT is switched off in this library");
    if (!cr.img16 || !cm.img16) return fail(ctx, CA_ESTATE, "CA_PATH_DIRECT needs clip sets made with CA_CLIPS_IMAGE");
    if (!checked) {
      if (!crs->direct_ok || !cms->direct_ok || crs->minN != maxN || cms->minN != maxN)
        return fail(ctx, CA_EUNSUPPORTED, "CA_PATH_DIRECT needs one raster size and half-windows <= 7");
      direct_n = maxN;
    }
    if (direct_n != 64 && direct_n != 128 && direct_n != 256)
      return fail(ctx, CA_EINVAL, "CA_PATH_DIRECT raster size");
  }
  void* sc = qmem;
  ca_status st = CA_OK;
  if (!sc && (st = scratch(ctx, queue_bytes(n), &sc)) != CA_OK) return st;
  const QueueMem qm = queue_carve((char*)sc, n);
  unsigned long long* counters = qm.counters;
  const int64_t cap_g = qm.cq.cap_groups;
  const int64_t check_n = (path == CA_PATH_MIXED && !on_demand) ? check_count(ctx, n) : 0;
  HIP_OR_FAIL(ctx, enqueue_cosine(ctx, cr, cm, maxN, Lmax, path, thr, io, qm, s, true, direct_n, !on_demand, gen_nb,
                                  check_n));
  unsigned long long h[14] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  HIP_OR_FAIL(ctx, hipMemcpyAsync(h, counters, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  if (on_demand) {
    st = fp64_on_demand(ctx, crs, cms, s, thr, io, qm, h, maxN, Lmax);
    if (st) return st;
    // the FP64 passes raised the error maxima
    HIP_OR_FAIL(ctx, hipMemcpyAsync(h, counters, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  }
  {
    float ms = 0.f;
    HIP_OR_FAIL(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->stats.t_main_ms += ms;
    ctx->stats.n_main_launch += 1;
    if (path == CA_PATH_MIXED)  // the member's FP16 half-spectrum and bit raster per pair
      ctx->stats.main_alg_bytes += (double)n * (4.0 * maxN * (maxN / 2 + 1) + maxN * maxN / 8.0);
    else if (path == CA_PATH_DIRECT) ctx->stats.main_alg_bytes += (double)n * (2.0 * direct_n * direct_n + direct_n * direct_n / 8.0);
    else ctx->stats.main_alg_bytes += io_bytes_fp32(maxN, n);
  }
  const int64_t n_groups = std::min<int64_t>((int64_t)h[2], cap_g);
  if (n_groups > 0 || h[0] > 0) {
    double err;
    std::memcpy(&err, &h[1], 8);
    ctx->stats.max_surface_err = std::max(ctx->stats.max_surface_err, err);
    std::memcpy(&err, &h[5], 8);
    ctx->stats.max_peak_err_sqrt = std::max(ctx->stats.max_peak_err_sqrt, err);
  }
  if (check_n > 0) {
    ctx->stats.check_pairs += (int64_t)h[10];
    ctx->stats.check_changed += (int64_t)h[13];
    double err;
    std::memcpy(&err, &h[12], 8);
    if (h[10] > 0) {
      ctx->stats.check_peak_err_sqrt = std::max(ctx->stats.check_peak_err_sqrt, err);
      const double band = gen_nb > 0 ? band_mixed(maxN) : BAND_MIXED;
      ctx->stats.check_band_frac = std::max(ctx->stats.check_band_frac, err / band);
    }
  }
  ctx->stats.pairs_aligned += n;
  ctx->stats.pairs_rescored += n_groups + (int64_t)h[0];
  ctx->stats.groups_exact += (cr.spec32 && cm.spec32) ? (int64_t)h[8] : n_groups;
  ctx->stats.pairs_full_fp64 += (int64_t)h[0];
  return CA_OK;
}

namespace capriv {
ca_status clips_create_in(ca_ctx* ctx, void* stream, int64_t n, const int64_t* rect_ptr, const int32_t* rects,
                          const int16_t* raster_n, const int16_t* marker_w, uint32_t flags, DevArena* arena,
                          ca_clipset** out) {
  return clips_create_impl(ctx, stream, n, rect_ptr, rects, raster_n, marker_w, flags, arena, out);
}
ca_status align_cosine_sets(ca_ctx* ctx, const ca_clipset* crs, const ca_clipset* cms, hipStream_t s,
                            Threshold thr, int path, const PairIO& io, bool checked, int direct_n, int bucket_w) {
  return align_cosine(ctx, crs, cms, s, thr, path, io, checked, direct_n, bucket_w);
}
}  // namespace capriv

namespace capriv {
// Bucketed, autotuned alignment (api_auto.hip).
ca_status align_auto(ca_ctx* ctx, const ca_clipset* cs, hipStream_t s, Threshold thr, const PairIO& io);
}  // namespace capriv

extern "C" ca_status ca_align_pairs(ca_ctx* ctx, void* stream, const ca_clipset* cs,
                                    const ca_constraint* con, int32_t path, int64_t n_pairs,
                                    const int32_t* rep, const int32_t* mem, uint8_t* bits,
                                    int16_t* shift, int32_t* count, double* score, uint32_t* flags) {
  if (!ctx) return CA_EINVAL;
  if (!cs || cs->ctx != ctx) return fail(ctx, CA_EINVAL, "clip set of another context");
  if (!valid_constraint(con)) return fail(ctx, CA_EINVAL, "bad constraint");
  if (n_pairs < 0) return fail(ctx, CA_EINVAL, "negative pair count");
  if (n_pairs == 0) return CA_OK;
  if (!rep || !mem || !bits || !shift || !count || !score || !flags)
    return fail(ctx, CA_EINVAL, "null output or pair pointer");
  if (n_pairs > (1ll << 31) - 1) return fail(ctx, CA_EINVAL, "pair list longer than 2^31 - 1");
  if (path < CA_PATH_MIXED || path > CA_PATH_XYSEP) return fail(ctx, CA_EINVAL, "bad path");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const bool contour = con->kind == CA_EDGE && con->edges == CA_EDGES_CONTOUR;
  if (contour && !cs->d.cstat)
    return fail(ctx, CA_ESTATE, "CA_EDGES_CONTOUR needs a clip set created with CA_CLIPS_CONTOURS");
  ca_status st = validate_pairs(ctx, cs, cs, s, n_pairs, rep, mem, con->kind == CA_EDGE ? (contour ? 2 : 1) : 0);
  if (st) return st;
  PairIO io{n_pairs, rep, mem, bits, shift, count, score, flags};
  if (con->kind == CA_EDGE) {
    HIP_OR_FAIL(ctx, hipMemsetAsync(score, 0, sizeof(double) * 2 * n_pairs, s));
    if (contour) HIP_OR_FAIL(ctx, launch_edge_contour(cs->d, io, Threshold{con->thr_num, 1}, s));
    else HIP_OR_FAIL(ctx, launch_edge(cs->d, io, Threshold{con->thr_num, 1}, s));
    ctx->stats.pairs_edge += n_pairs;
    return CA_OK;
  }
  if (path == CA_PATH_AUTO) {
    if (!cs->d.spec64)
      return fail(ctx, CA_EUNSUPPORTED, "CA_PATH_AUTO verifies against FP64 spectra (clip set made with CA_CLIPS_NO_FP64)");
    return capriv::align_auto(ctx, cs, s, Threshold{con->thr_num, con->thr_den}, io);
  }
  return align_cosine(ctx, cs, cs, s, Threshold{con->thr_num, con->thr_den}, path, io);
}

extern "C" ca_status ca_align_pairs_noalloc(ca_ctx* ctx, void* stream, const ca_clipset* cs,
                                            const ca_constraint* con, int32_t path, int64_t n_pairs,
                                            const int32_t* rep, const int32_t* mem, uint8_t* bits,
                                            int16_t* shift, int32_t* count, double* score, uint32_t* flags) {
  if (!ctx) return CA_EINVAL;
  if (!cs || cs->ctx != ctx) return fail(ctx, CA_EINVAL, "clip set of another context");
  if (!valid_constraint(con)) return fail(ctx, CA_EINVAL, "bad constraint");
  if (n_pairs < 0) return fail(ctx, CA_EINVAL, "negative pair count");
  if (n_pairs > CA_NOALLOC_MAX_PAIRS)
    return fail(ctx, CA_EINVAL, "ca_align_pairs_noalloc takes at most CA_NOALLOC_MAX_PAIRS (1,048,576) pairs; got " +
                                    std::to_string(n_pairs));
  if (n_pairs == 0) return CA_OK;
  if (!rep || !mem || !bits || !shift || !count || !score || !flags)
    return fail(ctx, CA_EINVAL, "null output or pair pointer");
  const bool cosine = con->kind == CA_COSINE;
  const bool contour = con->kind == CA_EDGE && con->edges == CA_EDGES_CONTOUR;
  if (contour && !cs->d.cstat)
    return fail(ctx, CA_ESTATE, "CA_EDGES_CONTOUR needs a clip set created with CA_CLIPS_CONTOURS");
  if (cosine) {
    if (path != CA_PATH_MIXED && path != CA_PATH_FP32)
      return fail(ctx, CA_EUNSUPPORTED, "ca_align_pairs_noalloc runs CA_PATH_MIXED or CA_PATH_FP32");
    if (!cs->d.spec64)
      return fail(ctx, CA_EUNSUPPORTED, "ca_align_pairs_noalloc needs stored FP64 spectra (no CA_CLIPS_NO_FP64)");
    if (path == CA_PATH_MIXED && !cs->mixed_ok)
      return fail(ctx, CA_EUNSUPPORTED, "CA_PATH_MIXED needs 128 x 128 clips with half-windows <= 16");
    if (path == CA_PATH_FP32 && !cs->d.spec32)
      return fail(ctx, CA_ESTATE, "CA_PATH_FP32 needs a clip set created with CA_CLIPS_FP32");
  }
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  char* base = noalloc_base(ctx->device);
  if (!base) return fail(ctx, CA_ESTATE, "allocation-free work array not set up on this device");
  hipStream_t s = (hipStream_t)stream;
  ca_status st = validate_pairs(ctx, cs, cs, s, n_pairs, rep, mem, cosine ? 0 : (contour ? 2 : 1),
                                (unsigned long long*)(base + NOALLOC_QUEUE_BYTES));
  if (st) return st;
  PairIO io{n_pairs, rep, mem, bits, shift, count, score, flags};
  if (!cosine) {
    HIP_OR_FAIL(ctx, launch_zero_u64((unsigned long long*)score, 2 * n_pairs, s));
    if (contour) HIP_OR_FAIL(ctx, launch_edge_contour(cs->d, io, Threshold{con->thr_num, 1}, s));
    else HIP_OR_FAIL(ctx, launch_edge(cs->d, io, Threshold{con->thr_num, 1}, s));
    ctx->stats.pairs_edge += n_pairs;
    return CA_OK;
  }
  return align_cosine(ctx, cs, cs, s, Threshold{con->thr_num, con->thr_den}, path, io, false, 0, 1 << 20, base);
}

// ---- captured alignment ------------------------------------------------------

struct ca_graph {
  ca_ctx* ctx = nullptr;
  int64_t n = 0;
  void* mem = nullptr;
  size_t bytes = 0;
  unsigned long long* n_bad = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" ca_status ca_graph_destroy(ca_graph* g) {
  if (!g) return CA_EINVAL;
  (void)hipSetDevice(g->ctx->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->mem) {
    (void)hipFree(g->mem);
    g->ctx->used -= g->bytes;
  }
  delete g;
  return CA_OK;
}

extern "C" ca_status ca_graph_create(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                                     int64_t n_pairs, const int32_t* rep, const int32_t* mem, uint8_t* bits,
                                     int16_t* shift, int32_t* count, double* score, uint32_t* flags,
                                     ca_graph** out) {
  if (!ctx) return CA_EINVAL;
  if (!out || !cs || cs->ctx != ctx) return fail(ctx, CA_EINVAL, "bad arguments");
  if (!valid_constraint(con) || con->kind != CA_COSINE) return fail(ctx, CA_EINVAL, "graphs capture the cosine track");
  if (!cs->d.spec64)
    return fail(ctx, CA_EUNSUPPORTED, "a captured sequence needs stored FP64 spectra (clip set made with CA_CLIPS_NO_FP64)");
  if (n_pairs <= 0 || n_pairs > (1ll << 31) - 1) return fail(ctx, CA_EINVAL, "bad pair count");
  if (!rep || !mem || !bits || !shift || !count || !score || !flags)
    return fail(ctx, CA_EINVAL, "null output or pair pointer");
  if (!cs->mixed_ok)
    return fail(ctx, CA_EUNSUPPORTED, "graphs capture CA_PATH_MIXED: 128 x 128 clips with half-windows <= 16");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = n_pairs;
  ca_graph* g = new ca_graph();
  g->ctx = ctx;
  g->n = n;
  const size_t b_q = queue_bytes(n), b_ids = align_up(4 * (size_t)n), b_bad = align_up(n);
  g->bytes = b_q + 2 * b_ids + b_bad + 256;
  ca_status st = dev_alloc(ctx, &g->mem, g->bytes, nullptr);
  if (st) {
    g->bytes = 0;
    ca_graph_destroy(g);
    return st;
  }
  char* p = (char*)g->mem;
  const QueueMem qm = queue_carve(p, n);
  int32_t* p_rep = (int32_t*)(p + b_q);
  int32_t* p_mem = (int32_t*)(p + b_q + b_ids);
  uint8_t* bad = (uint8_t*)(p + b_q + 2 * b_ids);
  g->n_bad = (unsigned long long*)(p + b_q + 2 * b_ids + b_bad);
  const PairIO io{n, p_rep, p_mem, bits, shift, count, score, flags};
  const Threshold thr{con->thr_num, con->thr_den};
  auto sequence = [&](hipStream_t q) -> hipError_t {
    hipError_t e = launch_zero_u64(g->n_bad, 1, q);
    if (e == hipSuccess) e = launch_sanitize_pairs(n, rep, mem, cs->n, cs->n, p_rep, p_mem, bad, g->n_bad, q);
    if (e == hipSuccess)
      e = enqueue_cosine(ctx, cs->d, cs->d, cs->maxN, cs->Lmax, CA_PATH_MIXED, thr, io, qm, q, false, 0, true, 0,
                         check_count(ctx, n));
    if (e == hipSuccess) e = launch_reject_pairs(n, bad, io, q);
    return e;
  };
  // one eager run first (function attributes, first-use set-up), then the
  // capture on a private stream (the caller's may be the legacy null stream,
  // which cannot be captured)
  hipError_t e = sequence(s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipStream_t cap = nullptr;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t ec = sequence(cap);
    const hipError_t ee = hipStreamEndCapture(cap, &g->graph);
    e = ec != hipSuccess ? ec : ee;
  }
  if (cap) (void)hipStreamDestroy(cap);
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    ca_graph_destroy(g);
    return fail(ctx, CA_EDEVICE, hipGetErrorString(e));
  }
  *out = g;
  return CA_OK;
}

extern "C" ca_status ca_graph_launch(ca_graph* g, void* stream) {
  if (!g) return CA_EINVAL;
  HIP_OR_FAIL(g->ctx, hipSetDevice(g->ctx->device));
  HIP_OR_FAIL(g->ctx, hipGraphLaunch(g->exec, (hipStream_t)stream));
  return CA_OK;
}

extern "C" ca_status ca_graph_invalid(ca_graph* g, void* stream, int64_t* n_invalid) {
  if (!g || !n_invalid) return CA_EINVAL;
  HIP_OR_FAIL(g->ctx, hipSetDevice(g->ctx->device));
  unsigned long long h = 0;
  HIP_OR_FAIL(g->ctx, hipMemcpyAsync(&h, g->n_bad, sizeof(h), hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_OR_FAIL(g->ctx, hipStreamSynchronize((hipStream_t)stream));
  *n_invalid = (int64_t)h;
  return CA_OK;
}

// Accessors used by api_cluster.hip.
namespace capriv {
ca_status fail_ctx(ca_ctx* ctx, ca_status st, const char* msg) { return fail(ctx, st, msg); }
ca_status scratch_ctx(ca_ctx* ctx, size_t bytes, void** out) { return scratch(ctx, bytes, out); }
ca_status alloc_ctx(ca_ctx* ctx, void** p, size_t bytes) { return dev_alloc(ctx, p, bytes, nullptr); }
void free_ctx(ca_ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  ctx->used -= bytes;
}
int device_of(const ca_ctx* ctx) { return ctx->device; }
int64_t check_sample_of(const ca_ctx* ctx) { return ctx->check_sample; }
void set_check_sample(ca_ctx* ctx, int64_t v) { ctx->check_sample = v; }
ca_run_stats* stats_of(ca_ctx* ctx) { return &ctx->stats; }
const ca::ClipsDev& dev_of(const ca_clipset* cs) { return cs->d; }
ca_ctx* ctx_of(const ca_clipset* cs) { return cs->ctx; }
const std::vector<int16_t>& hN_of(const ca_clipset* cs) { return cs->hN; }
const std::vector<int32_t>& hnpix_of(const ca_clipset* cs) { return cs->hnpix; }
int64_t n_of(const ca_clipset* cs) { return cs->n; }
int maxN_of(const ca_clipset* cs) { return cs->maxN; }
bool mixed_ok_of(const ca_clipset* cs) { return cs->mixed_ok; }
bool has_fp32_of(const ca_clipset* cs) { return cs->d.spec32 != nullptr; }
bool has_fp64_of(const ca_clipset* cs) { return cs->d.spec64 != nullptr; }
bool has_image_of(const ca_clipset* cs) { return DIRECT_ENABLED && cs->d.img16 != nullptr; }
const std::vector<int16_t>& hw_of(const ca_clipset* cs) { return cs->hw; }
std::map<int, TuneEntry>& tune_of(ca_ctx* ctx) { return ctx->tune; }
void set_stats(ca_ctx* ctx, const ca_run_stats& st) { ctx->stats = st; }
uint64_t gen_of(const ca_clipset* cs) { return cs->gen; }
PruneCache* prune_cache_of(ca_ctx* ctx) { return &ctx->prune_cache; }
CoverCache* cover_cache_of(ca_ctx* ctx) { return &ctx->cover_cache; }
}  // namespace capriv

extern "C" ca_status ca_surface(ca_ctx* ctx, void* stream, const ca_clipset* cs, int32_t path,
                                int64_t n_pairs, const int32_t* rep, const int32_t* mem, float* surf) {
  if (!ctx) return CA_EINVAL;
  if (!cs || cs->ctx != ctx || n_pairs < 0 || (n_pairs > 0 && (!rep || !mem || !surf)))
    return fail(ctx, CA_EINVAL, "bad arguments");
  const bool direct = DIRECT_ENABLED && path == CA_PATH_DIRECT && cs->direct_ok && cs->minN == cs->maxN;
  if (!direct && (path != CA_PATH_MIXED || !cs->mixed_ok))
    return fail(ctx, CA_EUNSUPPORTED, "surface access is provided for CA_PATH_MIXED and CA_PATH_DIRECT on the sets they accept");
  if (n_pairs == 0) return CA_OK;
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  ca_status st = validate_pairs(ctx, cs, cs, s, n_pairs, rep, mem, false);
  if (st) return st;
  const size_t n = (size_t)n_pairs;
  const size_t b_bits = align_up(n), b_shift = align_up(8 * n), b_cnt = align_up(8 * n), b_sc = align_up(16 * n),
               b_fl = align_up(4 * n), b_need = align_up(n), b_list = align_up(8 * n), b_r1 = align_up(8 * n);
  void* sc;
  st = scratch(ctx, b_bits + b_shift + b_cnt + b_sc + b_fl + b_need + b_list + b_r1 + 512, &sc);
  if (st) return st;
  char* p = (char*)sc;
  PairIO io{n_pairs, rep, mem, (uint8_t*)p, (int16_t*)(p + b_bits), (int32_t*)(p + b_bits + b_shift),
            (double*)(p + b_bits + b_shift + b_cnt), (uint32_t*)(p + b_bits + b_shift + b_cnt + b_sc)};
  p += b_bits + b_shift + b_cnt + b_sc + b_fl;
  RescoreQueue q;
  q.need = (uint8_t*)p;
  q.list = (int64_t*)(p + b_need);
  q.r1_low = (float*)(p + b_need + b_list);
  q.len = (unsigned long long*)(p + b_need + b_list + b_r1);
  q.peak_err_bits = q.len + 1;
  q.peak_ratio_bits = q.len + 5;
  HIP_OR_FAIL(ctx, hipMemsetAsync(q.len, 0, 32, s));
  CandQueue cq{nullptr, nullptr, q.len + 2, q.len + 3, 0, 0};
  if (direct)
    HIP_OR_FAIL(ctx, launch_pcm_direct(cs->d, cs->d, io, cs->maxN, Threshold{1, 1}, (float)BAND_DIRECT, q, cq, surf,
                                       q.len + 4, s));
  else
    HIP_OR_FAIL(ctx, launch_pcm_mfma128(cs->d, cs->d, io, Threshold{1, 1}, (float)BAND_MIXED, q, cq, ctx->mf_b1,
                                        ctx->mf_a2, surf, q.len + 4, s));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  return CA_OK;
}
