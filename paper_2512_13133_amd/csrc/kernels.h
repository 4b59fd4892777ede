// Host-side launchers of the device kernels (each defined next to its kernel).
#pragma once

#include "internal.h"

namespace ca {

constexpr int SPEC_LINE_ELEMS = 2048;  // complex FP64 elements per spectrum workgroup

hipError_t launch_pack(const int64_t* rect_ptr, const int32_t* rects, const ClipsDev& cs, int64_t n,
                       hipStream_t s);
hipError_t launch_label(const ClipsDev& cs, int64_t n, hipStream_t s);
hipError_t launch_spectrum(const ClipsDev& cs, const int64_t* ids, int64_t n_ids, int N,
                           double2* scratch, const double2* tw256, hipStream_t s);
// Shared-memory bytes of the per-pair FFT kernel for (scalar size, N, CH, LINES, Lmax).
size_t pcm_fft_smem(int scalar_bytes, int N, int CH, int LINES, int Lmax);
hipError_t launch_pcm_fft32(const ClipsDev& cs, const PairIO& io, const int64_t* list, int64_t n_blocks,
                            int mode, Threshold thr, double band, const float2* tw256, int CH,
                            int LINES, int Lmax, int maxN, const RescoreQueue& q, hipStream_t s);
hipError_t launch_pcm_fft64(const ClipsDev& cs, const PairIO& io, const int64_t* list, int64_t n_blocks,
                            int mode, Threshold thr, double band, const double2* tw256, int CH,
                            int LINES, int Lmax, int maxN, const RescoreQueue& q, hipStream_t s);
hipError_t launch_edge(const ClipsDev& cs, const PairIO& io, Threshold thr, hipStream_t s);
hipError_t launch_cosine_prune(const ClipsDev& cs, const PruneArgs& pa, Threshold thr, hipStream_t s);
hipError_t launch_edge_prune(const ClipsDev& cs, const PruneArgs& pa, Threshold thr, hipStream_t s);
hipError_t launch_validate(const ClipsDev& cs, int64_t n_pairs, const int32_t* rep, const int32_t* mem,
                           int need_poly, int* bad, hipStream_t s);

}  // namespace ca
