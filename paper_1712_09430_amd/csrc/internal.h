// Internal declarations shared by the kernels and the host runtime of catpc.
// Not part of the public C ABI (include/catpc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace catpc {

// Grid-sorted hit: position in the row grid, sector-local input index.
struct alignas(16) SortedHit {
  float y, z;
  int32_t idx;
  int32_t pad;
};

// Method constants, every value already rounded the way the filter uses it.
struct Consts {
  float kb;         // -0.00299792458 * Bz, curvature per unit q/pT (cm^-1 per GeV^-1)
  float sy2, sz2;   // cluster variances
  float wy, wz;     // neighbour windows
  float chi2;       // neighbour chord-residual cut
  float nsig;       // following gate
  int32_t max_miss;
  int32_t min_hits;
  int32_t precision;
  double sy2d, sz2d; // cluster variances for the binary64-covariance refit
};

struct Workspace {
  int32_t* row_first;    // [S*(R+1)] sector-local first hit of each row (row-major by sector)
  float4* grid_f;        // [S*R] per row: y_min, z_min, bins per cm in y, in z
  int2* grid_n;          // [S*R] per row: bins in y, in z (0 = empty row)
  int32_t* bins;         // [2H + 2SR] per row: first sorted position of each bin, then n_row
  SortedHit* sorted;     // [H] hits in bin order per row
  int32_t* raw_up;       // [H] neighbour-finder links when the caller does not keep them
  int32_t* raw_dn;       // [H]
  uint64_t* start_mask;  // [H/64 + 8] start-hit bits per wave
  int32_t* blk_cnt;      // [H/256 + 8] start hits per block
  int64_t* blk_off;      // [H/256 + 8] first slot of each block
  int32_t* start_glob;   // [H] global hit index of each tracklet slot
  unsigned long long* counters; // [8]: 0 work counter, 1 error bits
};

// Call geometry: sectors [s0, s1), hits [h0, h1) (global indices).
struct Span {
  int32_t s0, s1;
  int64_t h0, h1;
};

struct Inputs {
  const float* y;
  const float* z;
  const int32_t* row;
  const int64_t* hit_offset;
};

struct TrackletOut {
  float* x_ref;
  float* param;
  float* cov;
  int32_t* row_hit;
  int32_t* start_row;
  int32_t* first_row;
  int32_t* last_row;
  int32_t* n_hits;
  int32_t* flags;
};

constexpr int kHitsPerBlock = 256;  // per-hit kernels: block size of clean/start/compaction
constexpr int kMaxBinsPerRow = 1024;
constexpr float kBinMargin = 1.0e-2f;  // cm, widens bin ranges beyond rounding of window edges

// Launchers (kernels.hip).  All asynchronous on `st`.
hipError_t launch_reset(unsigned long long* counters, int n, hipStream_t st);
hipError_t launch_row_index(const Inputs& in, Span sp, int n_rows, const Workspace& ws, int block, hipStream_t st);
hipError_t launch_grid(const Inputs& in, Span sp, int n_rows, float bin_hits, const Workspace& ws, hipStream_t st);
hipError_t launch_neighbours(const Inputs& in, Span sp, int n_rows, const float* row_x, const Consts& c,
                             const Workspace& ws, int32_t* up, int32_t* dn, int block, hipStream_t st);
hipError_t launch_clean_start(const Inputs& in, Span sp, const int32_t* up, const int32_t* dn, int32_t* up_c,
                              int32_t* dn_c, const Workspace& ws, hipStream_t st);
hipError_t launch_scan(Span sp, int64_t* toff, const Workspace& ws, hipStream_t st);
hipError_t launch_compact(const Inputs& in, Span sp, int64_t* toff, int32_t* start_hit, const Workspace& ws,
                          hipStream_t st);
hipError_t launch_tracklets(const Inputs& in, Span sp, int n_rows, const float* row_x, const Consts& c,
                            const Workspace& ws, const int32_t* up_c, const int64_t* toff, int64_t first,
                            int64_t cap, const TrackletOut& out, int grid, int block, hipStream_t st);
hipError_t launch_refit64(const Inputs& in, Span sp, int n_rows, const float* row_x, const Consts& c,
                          const Workspace& ws, const int64_t* toff, int64_t first, int64_t cap,
                          const TrackletOut& out, int grid, hipStream_t st);
hipError_t launch_fp32_probe(int op, const float* a, const float* b, float* out, int64_t n, hipStream_t st);

}  // namespace catpc
