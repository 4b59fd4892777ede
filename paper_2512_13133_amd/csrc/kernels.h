// Host-side launchers of the device kernels (each defined next to its kernel).
#pragma once

#include <algorithm>

#include "internal.h"

namespace ca {

constexpr int SPEC_LINE_ELEMS = 2048;  // complex FP64 elements per spectrum workgroup
// Workgroups per launch: the grid size in work-items must stay below 2^32, so
// per-pair and per-clip launches are split into chunks of this many groups.
constexpr int64_t LAUNCH_CHUNK = 1 << 22;

hipError_t launch_pack(const int64_t* rect_ptr, const int32_t* rects, const ClipsDev& cs, int64_t n,
                       hipStream_t s);
hipError_t launch_label(const ClipsDev& cs, int64_t n, hipStream_t s);
// Zero n 64-bit words with a kernel (no memset node under graph capture).
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s);
// Range check of a pair list into a copy (out-of-range pairs become (0, 0)
// and are marked), and the no-result outputs of the marked pairs.
hipError_t launch_sanitize_pairs(int64_t n, const int32_t* rep, const int32_t* mem, int64_t n_r, int64_t n_m,
                                 int32_t* rep_o, int32_t* mem_o, uint8_t* bad, unsigned long long* n_bad,
                                 hipStream_t s);
hipError_t launch_reject_pairs(int64_t n, const uint8_t* bad, const PairIO& io, hipStream_t s);
// 128 x 128 clips only: the same spectra from one fused kernel (no scratch).
hipError_t launch_spectrum128(const ClipsDev& cs, const int64_t* ids, int64_t n_ids, const double2* tw256,
                              hipStream_t s);
hipError_t launch_spectrum(const ClipsDev& cs, const int64_t* ids, int64_t n_ids, int N,
                           double2* scratch, const double2* tw256, hipStream_t s);
// Whitened images of the listed clips of size N from their FP64 spectra
// (scratch: n_ids * N * (N/2+1) complex doubles).
// Direct window surface (half-windows <= 7) on MFMA from the whitened images;
// every pair has raster N (64, 128 or 256).  `tiles`: one device counter.
hipError_t launch_pcm_direct(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, int N, Threshold thr,
                             float band, const RescoreQueue& q, const CandQueue& cq, float* surf_out,
                             unsigned long long* tiles, hipStream_t s);
hipError_t launch_image(const ClipsDev& cs, const int64_t* ids, int64_t n_ids, int N, double2* scratch,
                        const double2* tw256, hipStream_t s);
// Shared-memory bytes of the per-pair FFT kernel for (scalar size, N, CH, LINES, Lmax).
size_t pcm_fft_smem(int scalar_bytes, int N, int CH, int LINES, int Lmax);
// Per-pair FFT surface over n_blocks pairs (list[b] when list is given); with
// n_dev the count is read on the device (at most n_blocks), so the launch
// needs no host synchronisation.
hipError_t launch_pcm_fft32(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, const int64_t* list, int64_t n_blocks,
                            int mode, Threshold thr, double band, const float2* tw256, int CH,
                            int LINES, int Lmax, int maxN, const RescoreQueue& q, hipStream_t s,
                            const unsigned long long* n_dev = nullptr);
hipError_t launch_pcm_fft64(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, const int64_t* list, int64_t n_blocks,
                            int mode, Threshold thr, double band, const double2* tw256, int CH,
                            int LINES, int Lmax, int maxN, const RescoreQueue& q, hipStream_t s,
                            const unsigned long long* n_dev = nullptr);
hipError_t launch_edge(const ClipsDev& cs, const PairIO& io, Threshold thr, hipStream_t s);
// Contours of every clip: the count pass writes edges per clip (or -1) into
// counts; the trace pass (after cedge_off is set) writes cedges, cpoly, chash.
hipError_t launch_contour_count(const ClipsDev& cs, int32_t* counts, hipStream_t s);
hipError_t launch_contour_trace(const ClipsDev& cs, int maxN, hipStream_t s);
// Edge track over full boundary edges (clip sets with contours).
hipError_t launch_edge_contour(const ClipsDev& cs, const PairIO& io, Threshold thr, hipStream_t s);
// XY-separation alignment of the cosine track: shifts of both directions
// (io.shift, io.flags), then count, score and bit at them.
hipError_t launch_xysep(const ClipsDev& cs, const PairIO& io, Threshold thr, hipStream_t s);
hipError_t launch_cosine_prune(const ClipsDev& cs, const PruneArgs& pa, Threshold thr, int maxN, hipStream_t s);
// Edge bounds pass: bits ORed into the survivor mask, which the caller
// zeroes (ranges start on 64-bit words, range_off in bits), and survivor
// counts; the pairs are written by launch_prune128(..., write = true) with
// order_ids set.
// Transposed polygon box sizes (MAX_POLY x n words) and counts (n) of the clips in `order`, with
// soa_hash the polygon hashes in the layout of the sizes (edge track over contours), and with
// soa_ext the extremes of the box sizes (2 x n words; the bounds pass needs them).
hipError_t launch_edge_soa(const ClipsDev& cs, const int32_t* order, int64_t n, uint32_t* soa_wh, int32_t* soa_np,
                           hipStream_t s, uint32_t* soa_hash = nullptr, uint32_t* soa_ext = nullptr);
hipError_t launch_edge_prune(const ClipsDev& cs, const PruneArgs& pa, Threshold thr, const int64_t* range_off,
                             unsigned long long* mask, hipStream_t s);
// Batched MFMA surface for raster 128, half-windows <= 16 (fragment tables from
// build_mfma128_tables: 4*3*64*8 and 8*3*64*8 halves).
void build_mfma128_tables(_Float16* b1, _Float16* a2);
// Persistent launch: `tiles` is device memory for the tile counter (cleared
// here on the stream).
hipError_t launch_pcm_mfma128(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr, float band,
                              const RescoreQueue& q, const CandQueue& cq, const void* b1frag,
                              const void* a2frag, float* surf_out, unsigned long long* tiles, hipStream_t s);
// Batched MFMA surface for rasters 64, 128 and 256 with NB x NB blocks of 16
// window positions per axis (shifts [-8 NB, 8 NB - 1]); mfma_gen_blocks gives
// the NB a half-window needs (0: unsupported), the fragment tables (b1 then
// a2, mfma_gen_table_halves halves) come from build_mfma_gen_tables.
int mfma_gen_blocks(int N, int half_window);
size_t mfma_gen_table_halves(int N, int NB);
void build_mfma_gen_tables(int N, int NB, _Float16* b1, _Float16* a2);
// sel (n_pairs int32) and n_sel (one counter): the list of pairs a queue-free
// first pass leaves undecided, where an instance runs two passes (null: one).
hipError_t launch_pcm_mfma_gen(int N, int NB, const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr,
                               float band, const RescoreQueue& q, const CandQueue& cq, const void* b1, const void* a2,
                               unsigned long long* tiles, int32_t* sel, unsigned long long* n_sel, hipStream_t s);
// FP64 re-decision of queued directions at their candidate shifts: the group
// count is read on the device (*cq.n_groups, at most cq.cap_groups).  With
// FP32 spectra on both sides and `exact.groups` set, a screen over the FP32
// spectra settles what it can and appends the rest to `exact` (its own group
// array and counter, cq's shifts and capacity), which the FP64 pass then takes.
hipError_t launch_rescore_candidates(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr,
                                     const CandQueue& cq, const CandQueue& exact, const double2* tw256,
                                     unsigned long long* peak_err_bits, unsigned long long* peak_ratio_bits,
                                     const float* r1_low, hipStream_t s);
// The FP32 screen alone (groups it cannot settle go to `exact`), and the FP64
// pass alone over a group queue.
hipError_t launch_rescore_screen(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr,
                                 const CandQueue& cq, const CandQueue& exact, const double2* tw256,
                                 unsigned long long* peak_err_bits, unsigned long long* peak_ratio_bits,
                                 const float* r1_low, hipStream_t s);
hipError_t launch_rescore_exact(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, Threshold thr,
                                const CandQueue& groups, const double2* tw256, unsigned long long* peak_err_bits,
                                unsigned long long* peak_ratio_bits, const float* r1_low, hipStream_t s);
// FP64 check of a sample of decided pairs (up to `count` of n pairs, spread
// evenly): the pick queues them (need = 3) in `list` / *len and saves their
// results; after an FP64 pass over that list the compare counts changed
// answers and restores the flags of the unchanged ones (cap: the pick's count).
hipError_t launch_sample_pick(int64_t n, int64_t count, const PairIO& io, uint8_t* need, int64_t* list,
                              unsigned long long* len, SampleSave* saved, hipStream_t s);
hipError_t launch_sample_compare(int64_t cap, const int64_t* list, const unsigned long long* len,
                                 const SampleSave* saved, const PairIO& io, uint8_t* need,
                                 unsigned long long* mismatches, hipStream_t s);
// Collect the clips whose FP64 spectra the re-decision needs: the pairs of the
// first n_groups groups and of list[0 .. n_list); remap tables start at -1.
hipError_t launch_mark_fp64(const PairIO& io, const CandGroup* groups, int64_t n_groups, const int64_t* list,
                            int64_t n_list, int64_t* remap_r, int64_t* ids_r, unsigned long long* cnt_r,
                            int64_t* remap_m, int64_t* ids_m, unsigned long long* cnt_m, int64_t per, hipStream_t s);
// Exact-objective alignment: per pair the window shift of the largest overlap
// count (tie rule as in the re-decision), both directions; rasters of 64 or
// 128 (pairs of the other size are skipped), half-windows <= 16.
hipError_t launch_xcorr(const ClipsDev& cr, const ClipsDev& cm, const PairIO& io, int N, Threshold thr,
                        hipStream_t s);
// Cosine candidate generation for 128 x 128 clips with half-windows <= 16:
// write = false runs the bounds pass (bitmask + counts), write = true the
// ordered write of the survivors (needs pa.offs).
// Transposed copies of the partners' sliding sums in `order` (64 x n words each).
hipError_t launch_prune128_soa(const ClipsDev& cb, const int32_t* order, int64_t n, uint32_t* soa_row,
                               uint32_t* soa_col, uint32_t* soa_grp, hipStream_t s);
hipError_t launch_prune128(const ClipsDev& ca, const ClipsDev& cb, const PruneArgs& pa, Threshold thr,
                           const int64_t* range_off, uint32_t* mask, bool write, hipStream_t s);
hipError_t launch_validate(const ClipsDev& cr, const ClipsDev& cm, int64_t n_pairs, const int32_t* rep,
                           const int32_t* mem, int need_poly, int* bad, hipStream_t s);

// Cover compaction (cover.hip): row counts of the set directions, the keys
// (member << 32 | 2 k + d) scattered to their rows, the per-row sort (rows of
// <= 64 keys in small_rows, longer ones in large_rows; tmp: nnz keys of
// merge space, needed when a row exceeds 4,096 keys), and the gather of
// column, shift, count and score per sorted key.
hipError_t launch_cover_count(int64_t n_pairs, const int32_t* rep, const int32_t* mem, const uint8_t* bits,
                              unsigned long long* rowcnt, hipStream_t s);
// A piece of a long candidate list: *n_keep += its pairs with a set direction
// (keep_count), then those pairs and their results copied to the kept arrays
// at slots taken from *slot (keep; the kept arrays hold *slot + that many).
hipError_t launch_cover_keep_count(int64_t n_pairs, const uint8_t* bits, unsigned long long* n_keep, hipStream_t s);
hipError_t launch_cover_keep(int64_t n_pairs, const int32_t* rep, const int32_t* mem, const uint8_t* bits,
                             const int16_t* shift, const int32_t* count, const double* score,
                             unsigned long long* slot, int32_t* k_rep, int32_t* k_mem, uint8_t* k_bits,
                             int16_t* k_shift, int32_t* k_count, double* k_score, hipStream_t s);
hipError_t launch_cover_scatter(int64_t n_pairs, const int32_t* rep, const int32_t* mem, const uint8_t* bits,
                                const int64_t* row_ptr, unsigned long long* fill, uint64_t* keys, hipStream_t s);
hipError_t launch_cover_sort(const int32_t* small_rows, int64_t n_small, const int32_t* large_rows, int64_t n_large,
                             const int64_t* row_ptr, uint64_t* keys, uint64_t* tmp, hipStream_t s);
hipError_t launch_cover_gather(int64_t nnz, const uint64_t* keys, const int16_t* shift, const int32_t* count,
                               const double* score, int32_t* col, int16_t* col_shift, int32_t* value,
                               double* col_score, hipStream_t s);
// Dense relation bits (out zeroed by the caller; n x words 64-bit words).
hipError_t launch_cover_dense(int64_t n, int64_t words, const int64_t* row_ptr, const int32_t* col,
                              unsigned long long* out, hipStream_t s);
// Center verification of n (member, representative, shift) triples: counts
// the violations into *viol and the smallest violating index into *first
// (callers clear *viol to 0 and *first to all ones).
hipError_t launch_verify_cosine(const ClipsDev& cs, int64_t n, const int32_t* mem, const int32_t* rep,
                                const int16_t* shift, Threshold thr, unsigned long long* viol,
                                unsigned long long* first, hipStream_t s);
hipError_t launch_verify_edge(const ClipsDev& cs, int64_t n, const int32_t* mem, const int32_t* rep,
                              const int16_t* shift, Threshold thr, unsigned long long* viol, unsigned long long* first,
                              hipStream_t s, bool contour = false);

}  // namespace ca
