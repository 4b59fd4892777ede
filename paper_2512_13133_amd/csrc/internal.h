// Library-internal declarations shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/clipalign.h"

namespace ca {

// Tie tolerance of the peak (shifts within TAU of the window maximum are tied)
// and the whitening cut |F| > EPS, both in the units of the paper's Eqs. 4-5
// as read in the library's documentation.
constexpr double TAU = 1e-9;
constexpr double EPS = 1e-2;
constexpr int MAX_POLY = 64;       // polygons per clip kept for the edge track
constexpr int MAX_RUNS = 4096;     // row runs per clip handled by the labeller
constexpr int MAX_AXIS = 65;       // window positions per axis (half-window <= 32)
constexpr int MAX_EDGES = 4096;    // boundary edges per clip kept for the full-edge track

// Device-resident clip set.  Per-clip arrays are indexed by clip id; pools are
// addressed through per-clip offsets that depend only on the raster size.
struct ClipsDev {
  int64_t n;
  const int16_t* N;          // [n] raster size
  const int16_t* w;          // [n] marker half-window
  const int64_t* bits_off;   // [n] word offset into bits (N*N/64 words)
  uint64_t* bits;
  int32_t* npix;             // [n]
  const int64_t* sig_off;    // [n] element offset into rowsum/colsum (N each)
  uint16_t* rowsum;
  uint16_t* colsum;
  uint16_t* winrow;          // sum of rowsum over rows t .. t+7 (mod N), N each
  uint16_t* wincol;          // same for columns
  int32_t* nruns;            // [n] total runs
  int32_t* npoly;            // [n] polygon count, -1 over the cap
  int16_t* boxes;            // [n][MAX_POLY][4] (x0, x1, y0, y1)
  int16_t* gbox;             // [n][4] global bounding box (zeros if empty)
  const int64_t* rowptr_off; // [n] offset into run_rowptr (N+1 each)
  uint16_t* run_rowptr;      // per clip: first run of each row, relative
  const int64_t* run_off;    // [n] offset into runs
  uint32_t* runs;            // x0 | x1 << 9 | label << 18 (label 0..63)
  int32_t* zero_bins;        // [n] full-grid bins with |F| <= EPS
  const int64_t* spec_off;   // [n] offset in bins: N*(N/2+1) per clip
  __half2* spec16;           // per clip: [u][v < N/2] then Nyquist column [u]
  float2* spec32;            // per clip: [u][v <= N/2] (optional)
  double2* spec64;           // per clip: [u][v <= N/2] (optional)
  const int64_t* img_off;    // [n] element offset into img16 (N*N each), or null
  __half* img16;             // per clip: whitened image N * IDFT2(W), row-major (optional)
  // Polygon contours (sets made with CA_CLIPS_CONTOURS; null otherwise).  The
  // edges of a clip list polygon 0, 1, ... in turn, each polygon its outer
  // contour and then its holes, each contour from the start of its least
  // rotation: coordinate (y of E/W edges, x of S/N edges) | direction
  // (E 0, S 1, W 2, N 3) << 9 | first edge of a contour << 11.
  int32_t* cstat;            // [n] edges of the clip, or -1 without contour data
  const int64_t* cedge_off;  // [n] offset into cedges
  uint16_t* cedges;
  uint16_t* cpoly;           // [n][MAX_POLY + 1] first edge of each polygon (relative), then the total
  uint32_t* chash;           // [n][MAX_POLY] polygon hash (FNV-1a 64 over the codes, low 32 bits)
};

// Per-call alignment problem in device-visible form.
struct PairIO {
  int64_t n_pairs;
  const int32_t* rep;
  const int32_t* mem;
  uint8_t* bits;
  int16_t* shift;   // [n][2][2]
  int32_t* count;   // [n][2]
  double* score;    // [n][2]
  uint32_t* flags;  // [n]
};

struct Threshold {
  int64_t p, q;  // cosine: p/q ; edge: p px (q = 1)
};

// Surface modes of the per-pair FFT kernel.
enum { MODE_LOW = 0, MODE_EXACT = 1, MODE_RESCORE = 2 };

// Queue of pair directions whose low-precision peak is too close to call.
struct RescoreQueue {
  uint8_t* need;                      // [n_pairs] directions queued for FP64 (bit d)
  int64_t* list;                      // queued pair ids
  unsigned long long* len;            // number of queued pairs
  float* r1_low;                      // [n_pairs][2] low-precision normalised peak value
  unsigned long long* peak_err_bits;  // max |r1_low - r1_fp64| as double bits (both K r / K_hi)
  unsigned long long* peak_ratio_bits = nullptr;  // the same difference in K r units / sqrt(K_hi)
};

// Near-tie candidates of a queued direction: the window shifts whose
// low-precision value lies within the band of the maximum.
constexpr int MAX_CAND = 64;
struct CandGroup {
  int64_t pair;    // pair id
  int64_t offset;  // first candidate in CandQueue::shifts
  int32_t dir;     // direction 0 or 1; 2: both (equal windows, candidates in forward shifts)
  int32_t count;   // candidates (0: group unused)
};
struct CandQueue {
  CandGroup* groups;
  int16_t* shifts;                  // (dy << 8) | (dx & 0xff)
  unsigned long long* n_groups;
  unsigned long long* n_shifts;
  int64_t cap_groups, cap_shifts;
};

// A decided pair's low-precision result, kept while the FP64 check of a
// sample of decided pairs recomputes it.
struct SampleSave {
  int16_t shift[4];
  int32_t count[2];
  uint32_t flags;
  uint8_t bits;
};

// Candidate generation: anchors, their partner ranges and the output list.
// Within one clip set the anchors are the positions of `order` and each
// anchor's partners start right after it; between two sets (a request batch
// against a library) `anchor_ids` and `lo` give the anchors and range starts.
struct PruneArgs {
  const int32_t* order;  // partner clip ids, grouped by raster size (cosine: by (n, id) within a size)
  const int32_t* hi;     // [n_anchor] exclusive end of each anchor's partner range in `order`
  int64_t n_anchor;
  int64_t* counts;       // [n_anchor] survivors (count pass)
  const int64_t* offs;   // [n_anchor] write offsets (write pass), or null
  int32_t* out_rep;
  int32_t* out_mem;
  const int32_t* anchor_ids = nullptr;  // [n_anchor] anchor clip ids (null: order[a])
  const int32_t* lo = nullptr;          // [n_anchor] start of each range in `order` (null: a + 1)
  int order_ids = 0;                    // write each pair as (smaller id, larger id)
  // a launch over anchors [a_begin, n_anchor) whose mask buffer starts at bit
  // mask_bit0 of the range offsets (the bounds pass in anchor chunks)
  int64_t a_begin = 0;
  int64_t mask_bit0 = 0;
  // subtracted from every write offset, so a piece of anchors [a_begin,
  // n_anchor) lands at the start of its own output buffer
  int64_t out_base = 0;
  // partner sliding sums transposed (packed row pair q of the partner at
  // position b of `order` at [q * soa_n + b]), so a wave's 64 partners read
  // one contiguous run per pair; null: read each partner's own row
  const uint32_t* soa_row = nullptr;
  const uint32_t* soa_col = nullptr;
  int64_t soa_n = 0;
  // the partners' shift-group maxima of the sliding sums (32 rows a
  // dimension, rows then columns, stride soa_n); null: no group stage
  const uint32_t* soa_grp = nullptr;
  // edge track: polygon box sizes (w | h << 16 of polygon q of the partner at
  // position b at [q * soa_n + b]) and polygon counts by position
  const uint32_t* soa_wh = nullptr;
  const int32_t* soa_np = nullptr;
  // edge track over full boundary edges: polygon hashes in the layout of
  // soa_wh, and polygons match only with equal hashes (null: box track)
  const uint32_t* soa_hash = nullptr;
  // edge track: the extremes of each partner's polygon box sizes, (min w |
  // max w << 16) at [b] and (min h | max h << 16) at [soa_n + b]
  const uint32_t* soa_ext = nullptr;
  int seg = 0;      // partners per workgroup (0: one workgroup per anchor range; > 0: n_seg
                    // segments per anchor, counts and offs indexed [a * n_seg + segment])
  int n_seg = 1;
};

}  // namespace ca
