// Host-side structures shared by the runtime translation units.
#pragma once

#include <stdint.h>

#include <map>
#include <vector>

namespace capriv {

// Path chosen by the autotuner for one (raster size, window class) bucket,
// with the measured time of every path tried on the calibration sample
// (microseconds per 1,000 pairs; negative when not applicable or not valid).
struct TuneEntry {
  int path = -1;
  double us_per_kpair[5] = {-1.0, -1.0, -1.0, -1.0, -1.0};  // indexed by CA_PATH_*
  int64_t sample = 0;
};

// Result of the last bounds pass of ca_prune (cosine on 128 x 128 sets, edge), kept
// on the context so that a sizing call and the following writing call share it.
struct PruneCache {
  uint64_t gen = 0;              // clip-set generation (0 = empty)
  int64_t kind = 0, p = 0, q = 0;
  int64_t na = 0, total = 0;
  size_t b_mask = 0;             // bytes of the survivor bitmask
  void* dev = nullptr;           // order | hi | range_off | counts | offsets | mask | partner tables
  size_t bytes = 0;
  std::vector<int64_t> counts;
  std::vector<int64_t> cuts;     // anchor chunks of the bounds pass: [cuts[c], cuts[c + 1])
  std::vector<int64_t> cut_bit0; // first mask bit of each chunk (64-bit aligned)
  // the plan (anchor order, ranges, chunks and partner tables on the device)
  // of the key below, valid before the counts are in
  uint64_t plan_gen = 0;
  int64_t plan_kind = 0, plan_p = 0, plan_q = 0, plan_screened = 0;
  int64_t plan_pairs = 0;        // pairs in the partner ranges (bounds the candidates)
};

// The last cover relation built by ca_cover / ca_cluster (CSR sorted by
// (representative, member), directions passing the constraint), kept on the
// context so that a sizing call and the following copying call, or a cluster
// call after a cover call, share it.  Device arrays in one allocation; the
// host keeps the row pointers.
struct CoverCache {
  uint64_t gen = 0;  // clip-set generation (0 = empty)
  int64_t kind = 0, p = 0, q = 0;
  int path = -1;
  int64_t n = 0, nnz = 0;
  void* dev = nullptr;
  size_t bytes = 0;
  int64_t* row_ptr = nullptr;  // [n + 1]
  int32_t* col = nullptr;      // [nnz]
  int16_t* shift = nullptr;    // [nnz][2]
  int32_t* value = nullptr;    // [nnz] cosine overlap count / edge residual
  double* score = nullptr;     // [nnz]
  std::vector<int64_t> h_row_ptr;
};

// Grow-only device region that a serving slot reuses for every request, so the
// steady state makes no hipMalloc / hipFree calls (hipFree waits for the
// device).  Allocations that do not fit fall back to hipMalloc.
struct DevArena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
};

}  // namespace capriv
