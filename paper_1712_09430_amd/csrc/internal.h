// Internal declarations shared by the kernels and the host runtime of catpc.
// Not part of the public C ABI (include/catpc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace catpc {

// Grid-sorted hit: position, sector-local input index, pad row.
struct alignas(16) SortedHit {
  float y, z;
  int32_t idx;
  int32_t row;
};

// Per-hit record in input order, written by the link-cleaning stage: the
// coordinates and the cleaned upward link, so that a step along a seed chain
// reads one 16-byte record.
struct alignas(16) ChainHit {
  float y, z;
  int32_t up;
  int32_t pad;
};

// Per (sector, row) grid header, one 32-byte record: bin origin and bins per
// cm, bin counts (ny == 0: empty row; at most kMaxBinsPerRow each), global
// position of the row's first sorted hit, half the offset of its bin table
// (the table sits at 2 * (first hit + row id), always even), and the row's
// hit count.
struct alignas(32) RowHdr {
  float ymin, zmin, iby, ibz;
  int16_t ny, nz;
  int32_t hit_base;
  int32_t bin_half;
  int32_t n;
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
  double kbd;        // kb in binary64 for the full refit
};

struct Workspace {
  int32_t* row_first;    // [S*(R+1)] sector-local first hit of each row (row-major by sector)
  RowHdr* hdr;           // [S*R] per row grid header
  int32_t* bins;         // [2H + 2SR] per row: first sorted position of each bin, then n_row
  SortedHit* sorted;     // [H] hits in bin order per row
  int32_t* raw_up;       // [H] neighbour-finder links when the caller does not keep them
  int32_t* raw_dn;       // [H]
  uint64_t* start_mask;  // [H/64 + 8] start-hit bits per wave
  int32_t* blk_sec;      // [H/256 + 8] sector of the first hit of each block of kHitsPerBlock hits of the span
  int32_t* blk_cnt;      // [H/256 + 8] start hits per block
  int64_t* blk_off;      // [H/256 + 8] first slot of each block, relative to its group of 1024 blocks
  int64_t* grp_off;      // [H/256/1024 + 8] first slot of each group of 1024 blocks
  int32_t* start_glob;   // [H] global hit index of each tracklet slot
  int32_t* batch_off;    // [S + 1] first tracklet batch of each sector (64 slots of one sector per batch)
  ChainHit* chain;       // [H] coordinates + cleaned up-link per hit (input order)
  unsigned* owner;               // [H] tracklet selection: weight of the tracklet that keeps each hit (row chunks too dense for LDS)
  int32_t* sel_cnt;              // [H/3 + 2] hits a selected tracklet keeps, or -1
  int32_t* sel_local;            // [H/3 + 2] sector-local index of each valid tracklet (claim pass)
  int2* sel_loc;                 // [H/3 + 2] track and hit offsets within the slot's group of 1024
  longlong2* sel_grp;            // [(H/3)/1024 + 8] group offsets
  uint16_t* sel_mask;            // [(H/3 + 2) * sel_chunks(R)] kept rows of each valid tracklet, per row chunk
  float4* mrec;                  // [H/3 + 2] segment merging: start x, y, z of each track's tracklet, rows
  unsigned long long* mkey_a;    // [H/3 + 2] segment merging: best continuation as (chi^2 bits, track)
  unsigned long long* mkey_b;    // [H/3 + 2] segment merging: best predecessor as (chi^2 bits, track)
  int2* mpair;                   // [kMergePairsPerSlot * (H/3 + 2)] segment merging: candidate pairs
  int32_t* mover;                // [H/3 + 2] segment merging: 1 when a pair of the track did not fit the list
  int32_t* mslot;                // [H/3 + 2] segment merging: tracklet slot of each track, or -1
  int32_t* mchunk;               // [S + 1] segment merging: first chunk of 256 tracks of each sector
  unsigned long long* counters; // [kNumCounters], see kCtr*
};

constexpr int kXcds = 8;         // MI355X: 8 accelerator dies, workgroups dispatched round-robin over them
constexpr int kCtrWork = 0;      // [0, kXcds): work counters of the tracklet kernel, one per slot partition
constexpr int kCtrError = 8;     // bit 0: invalid rows seen; bit 1: selection saw only part of the tracklets;
                                 // bit 2: a tracklet record names a hit outside its sector; bit 3: x differs
                                 // from the row planes; bit 4: too many tracklets in a sector for the selection;
                                 // bit 5: more tracks than the refit output holds; bit 6: pad-row planes given
                                 // on the device are not positive and strictly ascending
constexpr int kCtrCounts = 9;    // [9, 13): transports, updates, gated candidates, row searches
constexpr int kCtrSelTracks = 13;  // selected tracks
constexpr int kCtrSelHits = 14;    // hits they keep
constexpr int kCtrMergePairs = 15;  // candidate pairs of the segment merging
constexpr int kCtrMergeSteps = 16;  // row steps of their transports
constexpr int kNumCounters = 24;
constexpr int64_t kMergePairsPerSlot = 4;  // candidate-pair list length per track slot

// Call geometry: sectors [s0, s1), hits [h0, h1) (global indices).
struct Span {
  int32_t s0, s1;
  int64_t h0, h1;
};

struct Inputs {
  const float* x;  // NULL or checked against the row planes
  const float* y;
  const float* z;
  const int32_t* row;
  const int64_t* hit_offset;
};

struct TracksOut {
  int64_t* track_offset;
  int32_t* track_tracklet;
  int32_t* track_n_hits;
  int64_t* track_hit_offset;
  int64_t track_capacity;
  int32_t* track_hits;
  int64_t hit_capacity;
};

struct FitsOut {
  float* x;
  float* param;
  float* cov;
  float* chi2;
  int32_t* ndf;
  int32_t* flags;
  int64_t capacity;
};

struct MergeOut {
  int32_t* next;
  int32_t* prev;
  int32_t* head;
  float* chi2;
  int64_t capacity;
};

struct MergeCuts {
  int32_t max_gap;
  double window;
  double chi2_max;
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

// Row stride of the hit-per-row output (whole chunks of 8 rows).
__host__ __device__ inline int row_stride(int R) { return (R + 7) & ~7; }
// The selection works on chunks of 16 rows; a tracklet's kept rows are one
// 16-bit mask per chunk.
constexpr int kSelRows = 16;
__host__ __device__ inline int sel_chunks(int R) { return (R + kSelRows - 1) / kSelRows; }

constexpr int kMaxRows = 4096;       // pad rows per sector (row indices are wave-reduced as 16-bit values)
constexpr int kHitsPerBlock = 256;  // per-hit kernels: block size of clean/start/compaction
constexpr int kMaxBinsPerRow = 1024;
constexpr float kBinMargin = 1.0e-2f;  // cm, widens bin ranges beyond rounding of window edges

// Launchers (kernels.hip).  All asynchronous on `st`.
hipError_t launch_reset(unsigned long long* counters, int n, hipStream_t st);
hipError_t launch_rowk(const float* row_x, int n_rows, float4* rowk, unsigned long long* counters, hipStream_t st);
hipError_t launch_status(const unsigned long long* counters, uint64_t* status, hipStream_t st);
hipError_t launch_row_index(const Inputs& in, Span sp, int n_rows, const float* row_x, const Workspace& ws,
                            int block, hipStream_t st);
hipError_t launch_grid(const Inputs& in, Span sp, int n_rows, float bin_hits, const Workspace& ws, hipStream_t st);
hipError_t launch_neighbours(const Inputs& in, Span sp, int n_rows, const float4* rowk, const Consts& c,
                             const Workspace& ws, int32_t* up, int32_t* dn, int block, int rows, int lds_bytes,
                             hipStream_t st);
hipError_t launch_clean_start(const Inputs& in, Span sp, const int32_t* up, const int32_t* dn, int32_t* up_c,
                              int32_t* dn_c, const Workspace& ws, hipStream_t st);
hipError_t launch_scan(Span sp, int64_t* toff, const Workspace& ws, hipStream_t st);
hipError_t launch_compact(const Inputs& in, Span sp, int64_t* toff, int32_t* start_hit, const Workspace& ws,
                          hipStream_t st);
hipError_t launch_tracklets(const Inputs& in, Span sp, int n_rows, const float* row_x, const Consts& c,
                            const Workspace& ws, const int64_t* toff, int64_t first, int64_t cap,
                            const TrackletOut& out, int grid, int block, int nparts, int waves, int sync,
                            hipStream_t st);
hipError_t launch_select(const Inputs& in, int S, const int64_t* toff, int64_t cap, int64_t max_slots, int n_rows,
                         const TrackletOut& trk, const Consts& c, const Workspace& ws, const TracksOut& out,
                         int64_t n_hits, int grid, hipStream_t st);
hipError_t launch_fullfit(const Inputs& in, int S, int n_rows, const float* row_x, const Consts& c,
                          const int64_t* toff, const TrackletOut& trk, int64_t trk_cap, const TracksOut& tr,
                          const FitsOut& out, const Workspace& ws, int grid, hipStream_t st);
hipError_t launch_merge(const Inputs& in, int S, int n_rows, const float* row_x, const Consts& c,
                        const MergeCuts& m, const int64_t* toff, const TrackletOut& trk, int64_t trk_cap,
                        const TracksOut& tr, const FitsOut& fits, const MergeOut& out, const Workspace& ws,
                        int64_t max_slots, int grid, int pair_grid, int64_t pair_cap, hipStream_t st);
hipError_t launch_refit64(const Inputs& in, Span sp, int n_rows, const float* row_x, const Consts& c,
                          const Workspace& ws, const int64_t* toff, int64_t first, int64_t cap,
                          const TrackletOut& out, int grid, hipStream_t st);
hipError_t launch_probe_copy(const void* src, void* dst, int64_t n16, hipStream_t st);
hipError_t launch_probe_fma(float* out, int64_t n, int iters, hipStream_t st);
hipError_t launch_fp32_probe(int op, const float* a, const float* b, float* out, int64_t n, hipStream_t st);

// Phase clocks of the row-synchronous tracklet kernel (profiling build,
// -DCATPC_PHASE_CLOCKS=1): cycles summed over slot batches of each phase,
// row steps of the two passes, slot batches, and whole-wave cycles and waves.
enum {
  kPhaseStart, kPhaseOut, kPhaseBack, kPhaseIn, kPhaseOutSteps, kPhaseInSteps, kPhaseBatches, kPhaseWave, kPhaseWaves,
  kPhaseSlots
};
hipError_t phase_clocks(unsigned long long* out, bool clear);  // hipErrorNotSupported outside the profiling build

}  // namespace catpc
