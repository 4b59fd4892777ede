/* clipalign.h -- C ABI of the MI355X clip-alignment library.
 *
 * Batched pairwise optimal alignment and scoring of rasterised layout clips:
 * the hot path of the optimal-alignment clustering framework (arXiv
 * 2512.13133).  Inputs follow the paper's problem statement (Sec. 2.1-2.3):
 * clips given as Manhattan rectangles in their marker-centred window, the
 * marker half-window that bounds each clip's center shift, and a constraint
 * type with its threshold.  Outputs are the cover bits, the optimal integer
 * shifts (the member's center offset from its marker center) and scores, and,
 * from ca_cluster, the partition with its centers.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns ca_status (0 = CA_OK, < 0 = error).  No C++ exception,
 *   longjmp or abort crosses the ABI.  On error ca_last_error() returns a
 *   message that stays valid until the next call on the same context.
 * - Handles (ca_ctx, ca_clipset, ca_server) are owned by the library and freed
 *   only by their *_destroy call.  Every output buffer is owned by the caller.
 * - "Device pointer" means memory on the context's GPU (hipMalloc or a torch
 *   CUDA tensor); "host pointer" means ordinary host memory.  Each argument
 *   states which it accepts.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Asynchronous calls enqueue work on it and return; outputs are valid once
 *   that stream has reached the call's last operation.  Calls that return
 *   host-side results synchronise the stream before returning.
 * - A ca_ctx is used from one thread at a time; ca_server_submit and
 *   ca_server_poll may be called from any thread.
 * - A shift is (dy, dx) in pixels: the member's displacement relative to its
 *   representative, taken circularly on the N x N grid for the cosine track
 *   and linearly for the edge track.
 */
#ifndef CLIPALIGN_H
#define CLIPALIGN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CA_OK = 0,
  CA_EINVAL = -1,       /* malformed argument (null pointer, bad size, bad id) */
  CA_ENOMEM = -2,       /* device allocation failed or over the HBM budget */
  CA_EDEVICE = -3,      /* a HIP runtime call failed */
  CA_EBUSY = -4,        /* admission refused for now; retry later */
  CA_ETRUNC = -5,       /* caller buffer too small; required size written back */
  CA_ESTATE = -6,       /* call not valid in the object's current state */
  CA_EUNSUPPORTED = -7  /* input outside the library's supported envelope */
} ca_status;

typedef struct ca_ctx ca_ctx;
typedef struct ca_clipset ca_clipset;
typedef struct ca_server ca_server;

/* Context configuration.  device: HIP device ordinal.  hbm_budget_bytes: cap
 * on the library's own device allocations (0 = no cap); allocations that would
 * exceed it fail with CA_ENOMEM instead of exhausting HBM.
 * check_sample: pairs per CA_PATH_MIXED alignment call that the low-precision
 * pass decided (no FP64 re-decision) and that are nevertheless re-evaluated on
 * the full FP64 surface, as a run-time check of the decision band: 0 = 1,024,
 * negative = none, at most 4,096 and at most one pair in 256 of the call
 * (spread evenly over the call's pairs, the same pairs for equal pair
 * counts; the autotuner's timing runs check none).  A checked pair whose answer changes keeps the
 * FP64 answer and is counted in ca_run_stats.check_changed. */
typedef struct {
  int32_t device;
  int32_t check_sample;
  uint64_t hbm_budget_bytes;
} ca_config;

/* Constraint (paper Sec. 2.2).  CA_COSINE: Eq. 2, cosine strictly greater than
 * thr_num/thr_den (an exact rational, e.g. 19/20).  CA_EDGE: Sec. 2.2.2,
 * residual edge displacement at most thr_num pixels (thr_den must be 1).
 * edges (CA_EDGE only; 0 for CA_COSINE) names the corresponding edges of two
 * matched polygons:
 *   CA_EDGES_BOX: the four sides of the polygons' bounding boxes;
 *   CA_EDGES_CONTOUR: every edge of the polygon boundaries (Sec. 2.2.2 read
 *     over the full boundary).  A polygon's boundary is traced into closed
 *     contours with the polygon on the right (image coordinates, y down; a
 *     contour turns right where two of its pixels meet only diagonally); an
 *     edge is a maximal straight run.  Each contour starts at the least
 *     rotation of its direction codes (E 0, S 1, W 2, N 3; unique, since the
 *     sequence of a closed contour has no shorter period), the outer contour
 *     first, then the holes in raster order of their first vertex.  Two
 *     matched polygons correspond only if these code sequences are equal
 *     (else the direction has no correspondence: count -1, shift T0,
 *     CA_FLAG_NO_MATCH_*); then edge k corresponds to edge k, vertical edges
 *     displaced along x and horizontal ones along y.  Needs a clip set made
 *     with CA_CLIPS_CONTOURS (CA_ESTATE otherwise); pairs with a clip of more
 *     than 4,096 boundary edges return CA_EUNSUPPORTED.  The candidate
 *     generation (ca_prune) adds the topological hash: every polygon of the
 *     fewer side must find a polygon of the other side with the same hash
 *     (FNV-1a over its code sequences, see ca_clips_contours) as well as
 *     box sizes within 2 thr_num. */
enum { CA_COSINE = 1, CA_EDGE = 2 };
enum { CA_EDGES_BOX = 0, CA_EDGES_CONTOUR = 1 };
typedef struct {
  int32_t kind;
  int32_t edges;
  int64_t thr_num;
  int64_t thr_den;
} ca_constraint;

/* Alignment paths for the cosine track (paper Sec. 3.2.1(1), Eqs. 3-5).
 *   CA_PATH_MIXED: FP16 whitened spectra, batched per representative, pruned
 *     inverse transform as dense contractions on MFMA with FP32 accumulation;
 *     near-tied peaks are re-decided in FP64.  Clip sets of one raster size
 *     (64, 128 or 256) and half-windows up to 32 (CA_EUNSUPPORTED for sets
 *     that mix raster sizes: CA_PATH_AUTO takes those).
 *   CA_PATH_FP32: FP32 whitened spectra of both clips read per pair, one
 *     workgroup per pair, inverse transform by FFT on the vector ALUs; near
 *     ties re-decided in FP64.  All raster sizes and windows.
 *   CA_PATH_FP64: the FP64 surface and exact tie rule for every pair.
 *   CA_PATH_DIRECT: the window surface as a direct circular cross-correlation
 *     of the clips' FP16 whitened images (Parseval form of Eq. 5), batched
 *     16 members per representative on MFMA with FP32 accumulation; near ties
 *     re-decided in FP64.  Clip sets made with CA_CLIPS_IMAGE, one raster size
 *     (64, 128 or 256), half-windows <= 7 (CA_EUNSUPPORTED otherwise).
 *     Not enabled in this version of the library: every call with it returns
 *     CA_EUNSUPPORTED, and CA_PATH_AUTO never selects it.
 *   CA_PATH_AUTO: pairs of any raster size and window in one call.  The pairs
 *     are partitioned (stably) into buckets by raster size and window class
 *     (the larger half-window: <= 4, <= 7, <= 15, 16, <= 23, <= 31, more);
 *     each bucket runs the path the context's tuning table names for it.  A
 *     bucket met for the first time is tuned on up to 4,096 of its pairs
 *     (repeated to at least 1,024 when the bucket is smaller):
 *     every applicable path is timed, a path is admitted only if its results
 *     equal CA_PATH_FP64's bit for bit, the admitted ones are timed again on a
 *     contiguous run of up to 32,768 (64 x 64), 16,384 (128 x 128) or 8,192
 *     (256 x 256) of the bucket's pairs, and the fastest admitted one is kept
 *     (see ca_autotune_*).  Results return in the caller's order.
 * All of them return identical shifts, counts, scores and bits.
 *   CA_PATH_XCORR: a different objective, the one Sec. 3.2 states for
 *     alignment: per direction, the shift of the member's window with the
 *     largest overlap count c(s) = sum_x a_rep(x) a_mem((x + s) mod N), ties to
 *     the smaller |dy| + |dx|, then the smaller (dy, dx); score and bit of
 *     Eq. 2 there; empty clips as on the other paths.  Integer bit counts on
 *     the vector ALUs, one workgroup per pair, so the result is exact.  It can
 *     differ from the phase-correlation paths (their peak is the objective's
 *     maximiser only for pure translations); the count it returns is never
 *     smaller.  Rasters of 64 or 128 and half-windows <= 16 (CA_EUNSUPPORTED
 *     otherwise); CA_PATH_AUTO never selects it.
 *   CA_PATH_XYSEP: the geometric alternative of Sec. 3.2.1(2), "interval
 *     competition", in place of phase correlation: the polygon correspondence
 *     of the edge track at T0; per matched polygon pair the x and y intervals
 *     [min, max] of its two box-edge displacements (member minus
 *     representative); per axis the narrowest interval (ties: the first pair
 *     in (member polygon, rep polygon) order, polygons numbered in raster
 *     order) gives the shift as its midpoint, rounded half toward zero and
 *     clamped to the member's window, named as the cosine window names it.
 *     Without a correspondence (no polygon on a side, the exactly-one rule
 *     fails, a clip with more than 64 polygons) the global bounding boxes give
 *     the shift (T0).  Count, score and bit of Eq. 2 at the shift; empty clips
 *     as on the other paths (CA_FLAG_EMPTY).  Integer arithmetic only; rasters
 *     64, 128 and 256, any half-window; no spectra are read.  CA_PATH_AUTO
 *     never selects it. */
enum { CA_PATH_MIXED = 0, CA_PATH_FP32 = 1, CA_PATH_FP64 = 2, CA_PATH_AUTO = 3, CA_PATH_DIRECT = 4,
       CA_PATH_XCORR = 5, CA_PATH_XYSEP = 6 };

/* Per-pair flag bits written by the alignment calls. */
enum {
  CA_FLAG_RESCORED_FWD = 1u << 0, /* forward peak re-decided in FP64 */
  CA_FLAG_RESCORED_REV = 1u << 1, /* reverse peak re-decided in FP64 */
  CA_FLAG_EMPTY = 1u << 2,        /* a clip of the pair has no set pixel */
  CA_FLAG_NO_MATCH_FWD = 1u << 3, /* edge: no polygon correspondence (forward) */
  CA_FLAG_NO_MATCH_REV = 1u << 4, /* edge: no polygon correspondence (reverse) */
  CA_FLAG_RECHECK_FWD = 1u << 5,  /* edge: correspondence changed at final shift */
  CA_FLAG_RECHECK_REV = 1u << 6,
  CA_FLAG_INVALID = 1u << 7       /* graph replay: a pair id out of range (no result) */
};

/* Run statistics accumulated on a context since creation or the last reset. */
typedef struct {
  int64_t pairs_aligned;      /* unordered pairs through a cosine alignment call */
  int64_t pairs_rescored;     /* of those, pairs with a direction re-decided in FP64 */
  int64_t pairs_edge;         /* unordered pairs through the edge track */
  int64_t pairs_screened;     /* unordered pairs examined by ca_prune */
  int64_t pairs_survived;     /* of those, pairs written as candidates */
  int64_t n_main_launch;      /* launches of the main cosine alignment kernel */
  double t_main_ms;           /* their summed duration (HIP events on the launch stream) */
  double main_alg_bytes;      /* their algorithmic HBM bytes (spectra and bit rasters read) */
  double max_surface_err;     /* max |low-precision - FP64| peak value seen on
                                 re-decided pairs, both as K r / K_hi */
  double tie_band_mixed;      /* CA_PATH_MIXED re-decides a peak whose top-2 gap of K r is below
                                 tie_band_mixed * sqrt(K_hi), K_hi = N^2 - max(zero bins) */
  double tie_band_fp32;       /* CA_PATH_FP32 re-decides a peak whose normalised gap is below this */
  double tie_band_direct;     /* as tie_band_mixed, for CA_PATH_DIRECT */
  double max_peak_err_sqrt;   /* max_surface_err in the band's units: |low - FP64| peak difference
                                 of K r divided by sqrt(K_hi); stays below tie_band_mixed / 2 */
  int64_t groups_exact;       /* candidate groups the FP32 screen (clip sets with CA_CLIPS_FP32)
                                 left to the FP64 re-decision; without FP32 spectra, all groups */
  int64_t pairs_full_fp64;    /* of pairs_rescored, pairs whose whole window was re-evaluated in
                                 FP64 (their near-tied candidates overflowed the candidate list) */
  int64_t cover_nnz;          /* entries of the last cover relation built (ca_cover, ca_cluster) */
  int64_t members_verified;   /* members checked at their centers (ca_verify_centers, ca_cluster) */
  int64_t center_violations;  /* of those, members that failed the check (0 for ca_cluster's output) */
  int64_t check_pairs;        /* decided pairs re-evaluated on the full FP64 surface (check_sample) */
  int64_t check_changed;      /* of those, pairs whose FP64 answer differed (the band failed; 0 expected) */
  double check_peak_err_sqrt; /* max |low - FP64| peak value of K r / sqrt(K_hi) over the checked pairs,
                                 in the units of tie_band_mixed */
  double check_band_frac;     /* the same error as a fraction of the band the call used (tie_band_mixed
                                 for rasters up to 128, tie_band_mixed * N / 128 above): a decision
                                 is safe while it stays below 0.5 */
} ca_run_stats;

/* ---- context ------------------------------------------------------------ */

/* Create a context on cfg->device.  out: receives the handle. */
ca_status ca_create(const ca_config* cfg, ca_ctx** out);
/* Destroy a context.  All clip sets and servers made on it must be destroyed
 * first (CA_ESTATE otherwise). */
ca_status ca_destroy(ca_ctx* ctx);
/* Last error message of this context ("" if none).  ctx may be NULL, then the
 * message of the last failed ca_create is returned. */
const char* ca_last_error(const ca_ctx* ctx);
ca_status ca_get_stats(const ca_ctx* ctx, ca_run_stats* out);
ca_status ca_reset_stats(ca_ctx* ctx);

/* ---- clips: rasterise, pack and transform (paper Sec. 2.1 Eq. 1, Sec. 2.2.1
 *      steps 1-2, Sec. 3.2.1(1) Eq. 4 per-clip whitening) ------------------- */

/* Build a device-resident clip set of n clips.
 *   rect_ptr [n+1] int64: clip i owns rectangles rect_ptr[i] .. rect_ptr[i+1]-1.
 *   rects [rect_ptr[n]][4] int32: (x0, x1, y0, y1) in the clip's window frame;
 *     pixel (y, x) is set iff x0 <= x < x1 and y0 <= y < y1 for some rectangle;
 *     coordinates outside [0, N) are clipped.
 *   raster_n [n] int16: N_i in {64, 128, 256}.
 *   marker_w [n] int16: half-window w_i in [0, 32767]; the member's shifts are
 *     [-w_i, w_i]^2 (mod N_i on the cosine track, every residue once).
 *   flags: CA_CLIPS_DEVICE_PTRS if the four arrays are device pointers (else
 *     host pointers; the library copies them either way).
 *     CA_CLIPS_FP32 keeps FP32 spectra (8 (N/2+1) N bytes a clip) for
 *     CA_PATH_FP32; the FP64 re-decision of CA_PATH_MIXED then also screens
 *     its candidates on them first (same results, half the bytes read for
 *     the groups the screen settles).
 *     CA_CLIPS_IMAGE keeps each clip's whitened image w_i = IDFT2(W_i) (the
 *     spatial form of the whitened spectrum), scaled by N and stored as FP16
 *     (2 N^2 bytes a clip), for CA_PATH_DIRECT.
 *     CA_CLIPS_NO_FP64 keeps no FP64 spectra (16 (N/2+1) N bytes a clip
 *     saved; 128 x 128 sets without CA_CLIPS_IMAGE only, CA_EUNSUPPORTED
 *     otherwise), so that millions of clips fit in HBM: the FP64
 *     re-decision of CA_PATH_MIXED / CA_PATH_FP32 then computes the FP64
 *     spectra of just the clips it needs (same results).  CA_PATH_FP64,
 *     CA_PATH_AUTO and ca_graph_create return CA_EUNSUPPORTED on such sets.
 *     CA_CLIPS_CONTOURS also traces every polygon's boundary into contours
 *     (2 bytes an edge, 388 bytes a clip of tables) for the edge track over
 *     full boundary edges (CA_EDGES_CONTOUR; ca_clips_contours reads them).
 * The library rasterises, counts pixels, row/column sums, 4-connected polygons
 * (at most 64 per clip; larger counts mark the clip and make the edge track
 * fail with CA_EUNSUPPORTED on it), and computes FP64 spectra, whitened with
 * |F| > 1e-2 kept, stored as FP16 (and FP32 / FP64 as requested).
 * Returns CA_EINVAL on a bad size or N, CA_ENOMEM if it does not fit. */
enum { CA_CLIPS_DEVICE_PTRS = 1, CA_CLIPS_FP32 = 2, CA_CLIPS_FP64 = 4, CA_CLIPS_IMAGE = 8, CA_CLIPS_NO_FP64 = 16,
       CA_CLIPS_CONTOURS = 32 };
ca_status ca_clips_create(ca_ctx* ctx, void* stream, int64_t n, const int64_t* rect_ptr,
                          const int32_t* rects, const int16_t* raster_n,
                          const int16_t* marker_w, int32_t flags, ca_clipset** out);
ca_status ca_clips_destroy(ca_clipset* cs);
ca_status ca_clips_count(const ca_clipset* cs, int64_t* n);

/* Copy per-clip tables of clip i to host buffers (test and inspection
 * access; any pointer may be NULL to skip it).
 *   bits [N*N/64] uint64: row-major, bit x of row y at word y*N/64 + x/64, bit x%64.
 *   n_pix: set pixels.  rowsum [N], colsum [N] uint16.
 *   n_poly: polygon count (-1 if over the 64 cap).  boxes [64][4] int16 of
 *   (x0, x1, y0, y1), half-open.  zero_bins: count of grid bins with |F| <= 1e-2.
 *   spec16 [N][N/2+1][2] float: the FP16 whitened half-spectrum widened to
 *   float, bin (u, v) at (u*(N/2+1) + v)*2. */
ca_status ca_clips_inspect(const ca_clipset* cs, int64_t i, uint64_t* bits, int32_t* n_pix,
                           uint16_t* rowsum, uint16_t* colsum, int32_t* n_poly,
                           int16_t* boxes, int32_t* zero_bins, float* spec16);

/* Copy clip i's whitened image to a host buffer img [N*N] float, row-major:
 * img(y, x) = N * w_i(y, x), w_i = (1/N^2) sum_{u,v} W_i(u, v) e^{+2 pi i (u y + v x)/N}
 * (the inverse DFT of the whitened spectrum of Eq. 4, real since W_i is
 * Hermitian), as stored in FP16.  Its energy sum_x img^2 equals the number of
 * non-zero bins, so the values are of order one.  The phase-correlation
 * surface of Eq. 5 is the circular cross-correlation of two such images:
 *   K r(s) = sum_x img_rep(x) img_mem(x + s).
 * CA_ESTATE if the set was created without CA_CLIPS_IMAGE. */
ca_status ca_clips_image(const ca_clipset* cs, int64_t i, float* img);

/* Copy clip i's stored whitened half-spectrum W(u, v) = F/|F| (Eq. 4 with
 * each clip whitened on its own; 0 where |F| <= 1e-2), u < N, v <= N/2, into
 * host memory out[N][N/2 + 1][2] (real, imaginary) as doubles, read from the
 * copy of the given precision (16, 32 or 64 bits).  CA_ESTATE if that copy is
 * not kept (32: the set was made without CA_CLIPS_FP32). */
ca_status ca_clips_spectrum(const ca_clipset* cs, int64_t i, int32_t precision, double* out);

/* Copy clip i's polygon contours (Sec. 2.2.2 over full boundary edges) to
 * host buffers; any pointer may be NULL to skip it.
 *   n_edges: edges of the clip, or -1 when it has no contour data (its
 *     polygons were not kept, or it has more than 4,096 boundary edges).
 *   edges [cap] uint16: the clip's edges, polygon 0, 1, ... in turn; a
 *     polygon lists its outer contour, then its holes in raster order of their
 *     first vertex, each contour from the start of its least rotation.  A word
 *     is coordinate (y of an E/W edge, x of an S/N edge; 0..N) | direction
 *     (E 0, S 1, W 2, N 3) << 9 | (first edge of a contour) << 11.
 *     CA_ETRUNC (n_edges written) if cap < n_edges.
 *   poly_ptr [65] uint16: first edge of polygon p; entries from n_poly on
 *     hold n_edges.
 *   hashes [64] uint32: per polygon, FNV-1a (64-bit offset basis and prime)
 *     over the bytes of its direction codes, each contour followed by the
 *     byte 4, low 32 bits; 0 past the last polygon.
 * CA_ESTATE if the set was created without CA_CLIPS_CONTOURS. */
ca_status ca_clips_contours(const ca_clipset* cs, int64_t i, int32_t* n_edges, uint16_t* edges, int64_t cap,
                            uint16_t* poly_ptr, uint32_t* hashes);

/* ---- alignment on an explicit pair list (paper Sec. 3.2) ----------------- */

/* Align n_pairs unordered pairs (rep[k], mem[k]) in both directions.
 * Direction 0 aligns member mem[k] to the fixed representative rep[k];
 * direction 1 aligns rep[k] to mem[k].  Both clips of a pair must have the
 * same raster size (else CA_EINVAL).  All arrays are device pointers:
 *   rep, mem [n_pairs] int32 (clip ids)
 *   bits [n_pairs] uint8: bit0 = rep covers mem, bit1 = mem covers rep
 *   shift [n_pairs][2][2] int16: (dy, dx) of direction 0, then direction 1
 *   count [n_pairs][2] int32: cosine track: overlap count c at the shift;
 *     edge track: residual E in pixels (-1 if no correspondence)
 *   score [n_pairs][2] double: cosine c / sqrt(n_mem n_rep) (0 for the edge track)
 *   flags [n_pairs] uint32: CA_FLAG_* bits
 * Cosine track (con->kind == CA_COSINE, paper Eqs. 2-5): the shift is the
 * window maximum of the whitened phase-correlation surface; shifts within
 * 1e-9 of the maximum are tied and resolved by the larger overlap count, then
 * the smaller |dy|+|dx|, then the lexicographically smaller (dy, dx).
 * Edge track (CA_EDGE, paper Sec. 2.2.2, Eq. 6): polygon correspondence at the
 * global-bounding-box Min-Max shift, per-axis Min-Max midpoint over the
 * corresponding edges of the matched polygons (bounding-box sides, or every
 * boundary edge with con->edges == CA_EDGES_CONTOUR), re-check at the final
 * shift, bit iff E <= thr_num; `path` is ignored.
 * Asynchronous on `stream` for CA_PATH_FP64 and the edge track; the other
 * paths synchronise once to size the FP64 re-decision pass, and
 * CA_PATH_AUTO allocates its work space and synchronises per bucket. */
ca_status ca_align_pairs(ca_ctx* ctx, void* stream, const ca_clipset* cs,
                         const ca_constraint* con, int32_t path, int64_t n_pairs,
                         const int32_t* rep, const int32_t* mem, uint8_t* bits,
                         int16_t* shift, int32_t* count, double* score, uint32_t* flags);

/* Allocation-free variant of ca_align_pairs, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, layouts and results as
 * ca_align_pairs (all arrays are caller-owned device pointers), with these
 * limits:
 *   - n_pairs <= CA_NOALLOC_MAX_PAIRS (CA_EINVAL above it);
 *   - cosine track: path CA_PATH_MIXED or CA_PATH_FP32 only, on clip sets that
 *     keep FP64 spectra (CA_EUNSUPPORTED otherwise); the edge track as in
 *     ca_align_pairs.
 * The call makes no device allocation: its work space (the FP64 re-decision
 * queue, counters and a validation word, about 45 MB) is one static array per
 * device, set up by ca_create and held until the process ends.  Every call on
 * a device shares that array, so calls that overlap in time on one device
 * (from several threads or contexts, or on streams that run concurrently)
 * race and must be serialised by the caller.  Synchronises `stream` as
 * ca_align_pairs does. */
#define CA_NOALLOC_MAX_PAIRS 1048576
ca_status ca_align_pairs_noalloc(ca_ctx* ctx, void* stream, const ca_clipset* cs,
                                 const ca_constraint* con, int32_t path, int64_t n_pairs,
                                 const int32_t* rep, const int32_t* mem, uint8_t* bits,
                                 int16_t* shift, int32_t* count, double* score, uint32_t* flags);

/* Test and calibration access: the low-precision window surface of direction
 * 0 (member mem[k] against representative rep[k]) exactly as CA_PATH_MIXED or
 * CA_PATH_DIRECT computes it before any FP64 re-decision, for dy, dx in
 * [-16, 16] (CA_PATH_DIRECT writes only the entries with |dy|, |dx| <= 7):
 * surf[k][dy + 16][dx + 16] = K r(dy, dx) / K_hi with K_hi = N^2 minus the
 * larger zero-bin count of the two clips (paper Eq. 5 up to that positive
 * factor).  rep, mem, surf are device pointers; surf has n_pairs*33*33 floats.
 * CA_EUNSUPPORTED unless path is CA_PATH_MIXED or CA_PATH_DIRECT on a set that
 * path accepts.
 * Synchronises. */
ca_status ca_surface(ca_ctx* ctx, void* stream, const ca_clipset* cs, int32_t path, int64_t n_pairs,
                     const int32_t* rep, const int32_t* mem, float* surf);

/* Autotuner table of CA_PATH_AUTO (paper Sec. 3.2, the alignment of each
 * candidate pair; the choice only affects speed, never results).
 *   ca_autotune_report: one text line per tuned bucket (raster size, window
 *     class bound, chosen path, measured microseconds per 1,000 pairs of each
 *     path, -1 when not applicable or not admitted, sample size) into buf
 *     (NUL-terminated, at most cap bytes); *len gets the full length, and
 *     CA_ETRUNC is returned when cap is too small.
 *   ca_autotune_save / ca_autotune_load: the table as a text file (path is a
 *     host string); load replaces the table and rejects files of other
 *     formats with CA_EINVAL.
 *   ca_autotune_clear: empties the table (buckets are tuned again on use). */
ca_status ca_autotune_report(ca_ctx* ctx, char* buf, int64_t cap, int64_t* len);
ca_status ca_autotune_save(ca_ctx* ctx, const char* path);
ca_status ca_autotune_load(ca_ctx* ctx, const char* path);
ca_status ca_autotune_clear(ca_ctx* ctx);

/* ---- captured alignment (hipGraph) ---------------------------------------- */

/* A HIP graph of the whole CA_PATH_MIXED cosine alignment (paper Eqs. 2-5) of
 * a fixed device pair buffer: counters cleared by a kernel, the pair ids
 * copied and range-checked, the batched MFMA surface kernel, the FP64
 * re-decision sized on the device, and a fix-up of rejected pairs, with no
 * host synchronisation, so a replay is one graph launch.
 *   ca_graph_create: rep, mem, bits, shift, count, score, flags are device
 *     buffers of n_pairs entries (layouts as ca_align_pairs) that the graph
 *     reads and writes at every launch; the caller may change the pair ids
 *     between launches.  The clip set must be one CA_PATH_MIXED accepts
 *     (CA_EUNSUPPORTED otherwise) and must outlive the graph; cosine only.
 *     The graph owns its work space (allocated here, counted against the
 *     context's budget).  Captures on `stream`.
 *   ca_graph_launch: replays on `stream` (asynchronous).  A pair whose ids are
 *     out of range gets bits 0, shifts 0, counts -1, scores 0 and flags
 *     CA_FLAG_INVALID; every other pair gets exactly ca_align_pairs' result.
 *   ca_graph_invalid: synchronises `stream` and returns the number of pairs
 *     rejected by the last launch.
 *   ca_graph_destroy: releases the graph and its work space.
 * Launches of one graph must not overlap (they share the work space). */
typedef struct ca_graph ca_graph;
ca_status ca_graph_create(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                          int64_t n_pairs, const int32_t* rep, const int32_t* mem, uint8_t* bits,
                          int16_t* shift, int32_t* count, double* score, uint32_t* flags, ca_graph** out);
ca_status ca_graph_launch(ca_graph* g, void* stream);
ca_status ca_graph_invalid(ca_graph* g, void* stream, int64_t* n_invalid);
ca_status ca_graph_destroy(ca_graph* g);

/* ---- multi-stage pruning (paper Sec. 3.1 stage 1, Table 2) --------------- */

/* Candidate generation over all same-size unordered pairs of the clip set,
 * with safe bounds.  CA_COSINE: the pixel-area bound (B1: a pair whose smaller
 * pixel count n_min has n_min q^2 <= p^2 n_max cannot pass) and the row/column
 * signature bound over the window (B2).  CA_EDGE: every same-size pair is a
 * candidate of the polygon bounding-box size bound only (B3: every polygon of
 * the side with fewer polygons needs a partner whose box width and height
 * differ by at most 2 thr_num; with con->edges == CA_EDGES_CONTOUR also the same
 * polygon hash).  A rejected pair can never pass `con`, so pruned results
 * equal unpruned ones.
 * Output (device pointers): candidate pairs (rep[k], mem[k]), both directions
 * to be aligned; CA_EDGE writes rep[k] < mem[k] sorted by (rep, mem), CA_COSINE
 * groups the pairs by the anchor of the smaller pixel count; capacity `cap`
 * pairs.  *n_out (host) receives the survivor count; if it exceeds cap,
 * nothing is written past cap and CA_ETRUNC is returned.  Synchronises.
 * Call with cap = 0 to size, then again to write: the bounds pass of the
 * sizing call is kept on the context for the writing call.  Its candidate
 * mask (one bit per pair in each anchor's partner range) is held at most a
 * quarter of the free device memory at a time (the environment variable
 * CLIPALIGN_PRUNE_CHUNK_BYTES sets another limit, in bytes); a larger mask is
 * built over chunks of consecutive anchors, and the writing call then rebuilds
 * each chunk before writing its pairs (same results, twice the bounds work). */
ca_status ca_prune(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                   int64_t cap, int32_t* rep, int32_t* mem, int64_t* n_out);

/* ---- the cover relation (paper Sec. 3.1 stage 2, the sparse similarity
 *      graph consumed by the set cover of Sec. 3.3) --------------------------- */

/* Prune (ca_prune's bounds), align both directions of every candidate pair
 * (`path` for CA_COSINE: any but CA_PATH_DIRECT; ignored for CA_EDGE) and
 * compact the directions that pass `con` into a CSR relation sorted by
 * (representative, member):
 *   row r, entries row_ptr[r] .. row_ptr[r+1]-1, lists the clips m != r that r
 *   covers (cosine: Eq. 2 strictly above thr_num/thr_den at the aligned shift;
 *   edge: correspondence and residual <= thr_num), members ascending.  The
 *   diagonal (every clip covers itself) is implicit.
 *   row_ptr [n+1] int64, col [cap] int32 (member id),
 *   shift [cap][2] int16 (member's (dy, dx) relative to r),
 *   value [cap] int32 (cosine: overlap count c; edge: residual E),
 *   score [cap] double (cosine c / sqrt(n_m n_r); edge 0).
 * All output arrays are device pointers; any of col, shift, value, score may
 * be NULL to skip it.  *nnz (host) always receives the number of entries.
 * row_ptr == NULL sizes only.  If nnz > cap nothing is written and CA_ETRUNC
 * is returned.  The relation is compacted on the device and kept on the
 * context: a following call with the same clip set, constraint and path (the
 * copying call after a sizing call, or ca_cluster's loosest threshold) reuses
 * it.  A candidate list longer than the piece size (45 bytes of per-pair
 * results each: an eighth of the free device memory, at most 2^30 pairs and
 * at least n; the environment variable CLIPALIGN_COVER_PIECE_PAIRS sets
 * another size) is written, aligned and reduced to its pairs with a set
 * direction one piece at a time, with the same result; when the bounds pass
 * runs in anchor chunks (see ca_prune), one sweep counts and writes each
 * chunk's candidates.  Returns
 * CA_EUNSUPPORTED when 2^31 or more candidate pairs have a set direction.
 * Synchronises. */
ca_status ca_cover(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con, int32_t path,
                   int64_t cap, int64_t* row_ptr, int32_t* col, int16_t* shift, int32_t* value, double* score,
                   int64_t* nnz);

/* The same relation as a dense bit matrix for small sets (n <= 65,536):
 * bits [n][ceil(n/64)] uint64 (device pointer), bit m % 64 of word
 * r * ceil(n/64) + m / 64 set iff r covers m; the diagonal is set.
 * CA_EUNSUPPORTED above CA_COVER_DENSE_MAX clips.  Synchronises. */
#define CA_COVER_DENSE_MAX 65536
ca_status ca_cover_dense(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con, int32_t path,
                         uint64_t* bits);

/* Center verification (paper Sec. 2.3: center validity and cluster
 * consistency) of an assignment given as host arrays of length n:
 * rep_of [n] int32 and center_shift [n][2] int16 (as ca_cluster writes them).
 * A clip i is a violation if rep_of[i] is out of range, if a representative
 * (rep_of[i] == i) has a non-zero shift, if rep_of[rep_of[i]] != rep_of[i], or
 * if the constraint does not hold for i at its center against rep_of[i],
 * recomputed on the device from the clips' rasters:
 *   CA_COSINE: the shift is a residue of i's window (as in ca_align_pairs) and
 *     the overlap count c at it satisfies c^2 q^2 > p^2 n_i n_r exactly;
 *   CA_EDGE: |dy|, |dx| <= i's half-window, the polygons of the side with
 *     fewer polygons (both if equal) each overlap exactly one polygon of the
 *     other clip at the shift, and over their matched bounding-box edges
 *     max |d - s| per axis is at most thr_num.
 * *n_violations (host) receives the count, *first_violation (host, may be
 * NULL) the smallest violating clip id or -1.  Synchronises. */
ca_status ca_verify_centers(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                            const int32_t* rep_of, const int16_t* center_shift, int64_t* n_violations,
                            int64_t* first_violation);

/* ---- clustering: set cover and closed loop (paper Secs. 3.1, 3.3) -------- */

/* Full method on a clip set: the cover relation at the loosest threshold of
 * the schedule (ca_cover), surprisal lazy-greedy set cover (Eqs. 7-9) inside
 * the coarse-to-fine loop with `iterations` >= 1 relaxed-to-strict thresholds
 * (cosine T - 0.02 (K-t)/(K-1); edge T + (K - t) px), orphans re-attached to
 * the first representative that covers them strictly, then every member
 * verified at its center (ca_verify_centers; a violation returns CA_ESTATE).
 * The host holds O(n + nnz) memory.  Outputs are host arrays of length n:
 *   rep_of [n] int32: representative of each clip (itself for representatives)
 *   center_shift [n][2] int16: the clip's shift relative to its representative
 *   n_clusters: number of representatives. */
ca_status ca_cluster(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                     int32_t path, int32_t iterations, int32_t* rep_of, int16_t* center_shift,
                     int64_t* n_clusters);
/* ca_cluster with the relaxation of the coarse-to-fine schedule (Sec. 3.1:
 * coarse stages under relaxed constraints, the last one strict) as a
 * parameter, for schedule studies.  CA_COSINE: the thresholds are
 * T - R (K - t) / (K - 1) for t = 1..K with R = relax_num / relax_den an exact
 * rational, 0 <= R < T (ca_cluster uses R = 2/100).  CA_EDGE: T + relax_num
 * (K - t) pixels, relax_den = 1 (ca_cluster uses 1 px).  CA_EINVAL otherwise.
 * Everything else as ca_cluster. */
ca_status ca_cluster_schedule(ca_ctx* ctx, void* stream, const ca_clipset* cs, const ca_constraint* con,
                              int32_t path, int32_t iterations, int64_t relax_num, int64_t relax_den,
                              int32_t* rep_of, int16_t* center_shift, int64_t* n_clusters);

/* ---- serving: continuous batching against a device-resident library ---- */

/* Serving applies the refinement step of the paper (Sec. 3.1, step 3: a
 * pattern is aligned to fixed representatives and accepted under the strict
 * threshold, Eqs. 2-5) to request batches that arrive over time.
 *   library: a clip set on ctx (128 x 128 clips, half-windows <= 16) holding
 *     the representatives; it must outlive the server.  If it was created
 *     with CA_CLIPS_FP32, request batches get FP32 spectra too and the
 *     exact re-decision of near-tied peaks runs behind the FP32 screen; if
 *     it was created with CA_CLIPS_NO_FP64, so are the batches.
 *   con: the cosine constraint (CA_EUNSUPPORTED for the edge track).
 *   slots: 1..32 concurrent requests; each slot has its own HIP stream and
 *     worker thread, so requests on different slots overlap on the device.
 *   hbm_budget_bytes: admission budget for the requests' own device memory
 *     (0 = none); a request whose estimated footprint does not fit is refused
 *     with CA_EBUSY and may be resubmitted later. */
ca_status ca_server_create(ca_ctx* ctx, const ca_clipset* library, const ca_constraint* con, int32_t slots,
                           uint64_t hbm_budget_bytes, ca_server** out);
/* Stop the workers (queued requests still finish) and free the server. */
ca_status ca_server_destroy(ca_server* srv);
/* Submit a batch of n clips given as host arrays in the layout of
 * ca_clips_create (128 x 128, half-windows <= 16).  The arrays are copied
 * before return.  req_id (host) receives the request id.  Thread-safe. */
ca_status ca_server_submit(ca_server* srv, int64_t n, const int64_t* rect_ptr, const int32_t* rects,
                           const int16_t* raster_n, const int16_t* marker_w, uint64_t* req_id);
/* Non-blocking poll.  *done = 0 while the request runs; when it has finished,
 * *done = 1, the per-clip results are copied to the host arrays (any may be
 * NULL) and the request is released:
 *   best_rep [n] int32: library clip id of the best covering representative
 *     (highest score, ties to the lowest id), -1 if none covers the clip;
 *   shift [n][2] int16: the clip's shift (dy, dx) relative to that representative;
 *   score [n] double: its cosine score; matched [n] uint8: 1 if covered.
 * A failed request returns its error status with *done = 1.  Thread-safe. */
ca_status ca_server_poll(ca_server* srv, uint64_t req_id, int32_t* best_rep, int16_t* shift, double* score,
                         uint8_t* matched, int32_t* done);
/* Block until the request has finished (timeout_ms < 0: no limit); CA_EBUSY
 * on timeout.  Thread-safe. */
ca_status ca_server_wait(ca_server* srv, uint64_t req_id, int32_t timeout_ms);
/* Finished requests, candidate pairs aligned for them, and admitted bytes
 * currently in flight.  Thread-safe. */
ca_status ca_server_stats(ca_server* srv, int64_t* requests_done, int64_t* candidate_pairs,
                          uint64_t* inflight_bytes);
/* Run statistics of the server's slots (ca_run_stats, summed over the slots,
 * maxima for the error fields) as of each slot's last finished request: the
 * requests' alignment counts and the FP64 check of decided pairs.
 * Thread-safe. */
ca_status ca_server_run_stats(ca_server* srv, ca_run_stats* out);
/* Last error message of the server (valid until its next failing call). */
const char* ca_server_last_error(ca_server* srv);

/* ---- measurement aid (not part of the method) ----------------------------- */

/* For callers that time the alignment kernels against the memory roof: reads
 * the device buffer `buf` (16-byte aligned, `bytes` a multiple of 16) with a
 * plain streaming kernel, reps + 1 times on `stream` (the first untimed), and
 * returns the average milliseconds per read from HIP events, so bytes /
 * ms_per_read is the read bandwidth an ordinary kernel reaches on the device.
 * CA_EINVAL on a bad argument, CA_EDEVICE on a HIP failure.  Synchronises. */
ca_status ca_probe_read_bandwidth(void* stream, const void* buf, uint64_t bytes, int32_t reps,
                                  double* ms_per_read);

#ifdef __cplusplus
}
#endif

#endif /* CLIPALIGN_H */
