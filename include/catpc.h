/*
 * catpc -- TPC sector tracking hot path on MI355X (gfx950): cellular-automaton
 * neighbour finding over the pad rows and Kalman tracklet construction.
 *
 * Method: Rohr, Gorbunov, Lindenstruth, "GPU-accelerated track reconstruction
 * in the ALICE High Level Trigger" (arXiv:1712.09430), Sec. 2 items 1-2
 * (seeding with a cellular automaton, track following with a simplified
 * Kalman filter), Fig. 2 c-d, Tab. 1 rows 1-2; problem statement per sector
 * (Sec. 2: sectors are tracked independently), output size unknown in advance
 * with a late fetch of what did not fit (Sec. 3.1), many events on one GPU at
 * once (Sec. 3.2).
 *
 * Conventions for every call below
 *  - Pointers named "device" are HIP device memory owned by the caller; the
 *    library never frees them.  "host" pointers are read during the call only.
 *  - Hits are given per sector, sectors concatenated: hits of sector s are the
 *    global indices [hit_offset[s], hit_offset[s+1]), sorted by pad row inside
 *    the sector.  Coordinates are sector-local (x along the pad-row normal),
 *    float32, cm.  Every hit index the library returns is SECTOR-LOCAL
 *    (0 .. n_s - 1), so a sector gives identical output alone or in a batch.
 *  - All compute calls are asynchronous on the given stream (a hipStream_t
 *    passed as void*; NULL = the null stream); results are valid after the
 *    stream has been synchronised.  catpc_result() synchronises and reports
 *    errors found on the device.
 *  - Errors: a negative status; catpc_last_error() returns a thread-local
 *    message describing the last failure.  Host-side validation failures leave
 *    every output untouched.
 *  - The hot calls allocate nothing: the workspace is allocated once by
 *    catpc_create for the maximum sizes given there.
 */
#ifndef CATPC_H
#define CATPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t catpc_status;
#define CATPC_OK 0
#define CATPC_E_INVALID (-1)  /* bad argument or invalid input hits */
#define CATPC_E_CAPACITY (-2) /* more tracklets than output slots: fetch the rest */
#define CATPC_E_HIP (-3)      /* a HIP runtime call failed */
#define CATPC_E_STATE (-5)    /* call out of order (e.g. fetch before any track call) */

/* tracklet flag bits */
#define CATPC_FLAG_VALID 1       /* n_hits >= min_hits */
#define CATPC_FLAG_STOP_SINPHI 2 /* a pass ended because |sin phi| reached 0.999 */
#define CATPC_FLAG_STOP_ARC 4    /* a pass ended because |k * chord / 2| exceeded 0.2 */
#define CATPC_FLAG_SPD_FAIL 8    /* binary32 covariance failed the positive-definiteness check */
#define CATPC_FLAG_REFIT64 16    /* parameters come from the binary64-covariance refit */

/* Method parameters (all float32 / int32).  Defaults in brackets. */
typedef struct {
  float bz;             /* solenoid field, T [0.5] */
  float sigma_y;        /* cluster error in y, cm [0.1] */
  float sigma_z;        /* cluster error in z, cm [0.1] */
  float nf_win_y;       /* neighbour search half-window around the ray from the origin, y, cm [3] */
  float nf_win_z;       /* same in z, cm [3] */
  float nf_chi2_max;    /* cut on the 3-point chord residual dy^2 + dz^2, cm^2 [0.2] */
  float tc_gate_nsigma; /* following gate in predicted standard deviations [3] */
  int32_t tc_max_miss;  /* following ends after more consecutive empty rows than this [4] */
  int32_t min_hits;     /* a tracklet is flagged valid with at least this many hits [10] */
  int32_t precision;    /* 0: binary32 only; 1: refit SPD failures with a binary64 covariance;
                           2: refit every tracklet that way (test hook) [0] */
} catpc_params;

/* Launch-shape tuning.  Results never depend on these values (tested). */
typedef struct {
  float bin_hits;        /* target hits per grid bin [2.0] */
  int32_t nf_block;      /* threads per workgroup of the per-hit kernels [256] */
  int32_t tc_block;      /* threads per workgroup of the tracklet kernel [256] */
  int32_t tc_waves_per_cu; /* resident waves per CU of the persistent tracklet kernel [20] */
  int32_t use_graph;     /* 1: replay the batched stage chain as a captured hipGraph [1] */
  int32_t nf_rows;       /* pad rows per neighbour-finder workgroup (row chunk) [4] */
  int32_t nf_lds_kb;     /* LDS budget (KiB) for staging a row chunk and its two neighbour rows (a chunk that does
                            not fit is searched in place); 0: every hit is searched in place, one thread per hit in
                            grid order (a separate kernel) [32] */
  int32_t tc_xcd;        /* 1: tracklet slots split into one contiguous part per die, each die starting on its
                            own part (L2 locality) [1] */
  int32_t tc_occupancy;  /* resident waves per SIMD the tracklet kernel's registers are fitted for:
                            0 (the compiler's own allocation), 5, 6 or 8 (may spill to scratch) [0] */
  int32_t tc_sync;       /* 1: the lanes of a wave step through the pad rows together, reading the same row
                            grids at the same time [0] */
  int32_t merge_pair_cap; /* segment merging: at most this many candidate pairs are listed for the per-pair
                             pass, 0 for the whole list (4 per track slot); a track with a pair beyond the
                             list evaluates all its pairs in its own lane [0] */
} catpc_tuning;

/* Input hits (device pointers). */
typedef struct {
  const float* y;                /* device [n_hits] */
  const float* z;                /* device [n_hits] */
  const int32_t* row;            /* device [n_hits], pad row 0 .. n_rows-1, sorted within each sector */
  const int64_t* hit_offset;     /* device [n_sectors+1], hit_offset[0] == 0 */
  const int64_t* hit_offset_host;/* host copy of hit_offset; required by catpc_track_plain, optional otherwise */
  int32_t n_sectors;
  int64_t n_hits;                /* == hit_offset[n_sectors] */
  const float* x;                /* device [n_hits] or NULL: x of each hit (cm); every hit lies on its pad-row
                                    plane, so the path uses row_x[row]; when given, x[i] == row_x[row[i]] is
                                    checked and a difference reported by catpc_result as CATPC_E_INVALID */
} catpc_input;

/* Outputs (device pointers, caller-owned). */
typedef struct {
  int32_t* link_up;          /* device [n_hits]: cleaned upward link (sector-local index) or -1 */
  int32_t* link_dn;          /* device [n_hits]: cleaned downward link or -1 */
  int32_t* nf_up;            /* device [n_hits] or NULL: raw neighbour-finder upward link */
  int32_t* nf_dn;            /* device [n_hits] or NULL: raw neighbour-finder downward link */
  int32_t* start_hit;        /* device [n_hits]: start hits, sector-local, ascending within each
                                sector; sector s owns slots [tracklet_offset[s], tracklet_offset[s+1]) */
  int64_t* tracklet_offset;  /* device [n_sectors+1]; tracklet slot j belongs to start_hit[j] */
  int64_t tracklet_capacity; /* number of tracklet slots in the arrays below */
  float* x_ref;              /* device [cap]: x of the fitted state (x of first_row) */
  float* param;              /* device [cap][5]: y, z, sin phi, tan lambda, q/pT at x_ref */
  float* cov;                /* device [cap][15]: packed lower triangle over the same order */
  int32_t* row_hit;          /* device [cap][catpc_row_stride(n_rows)], 16-byte aligned: entry
                                t*stride + r is the hit (sector-local) that tracklet t picked in row r,
                                or -1 (also in the padding rows r >= n_rows) */
  int32_t* start_row;        /* device [cap] */
  int32_t* first_row;        /* device [cap] */
  int32_t* last_row;         /* device [cap] */
  int32_t* n_hits;           /* device [cap] */
  int32_t* flags;            /* device [cap]: CATPC_FLAG_* */
} catpc_output;

/* Selected track segments (caller-owned device memory), written by
 * catpc_select_tracklets.  Tracks of sector s are [track_offset[s],
 * track_offset[s+1]), in tracklet order; the hits of track k are
 * track_hits[track_hit_offset[k] .. + track_n_hits[k]), sector-local, rows
 * ascending.  No hit is in two tracks, so hit_capacity = n_hits and
 * track_capacity = the number of tracklets always suffice. */
typedef struct {
  int64_t* track_offset;     /* device [n_sectors+1] */
  int32_t* track_tracklet;   /* device [track_capacity]: sector-local index of the tracklet the track comes from
                                (its slot is tracklet_offset[s] + this) */
  int32_t* track_n_hits;     /* device [track_capacity]: hits the track keeps */
  int64_t* track_hit_offset; /* device [track_capacity]: first entry of its hits in track_hits */
  int64_t track_capacity;
  int32_t* track_hits;       /* device [hit_capacity] */
  int64_t hit_capacity;
} catpc_tracks;

/* Refitted tracks (caller-owned device memory), one entry per selected track,
 * at the track's outermost hit: x, parameters (y, z, sin phi, tan lambda,
 * q/pT), packed lower-triangle covariance over the same order, chi^2, ndf =
 * 2 hits - 5, flags (1 done; 2 |sin phi| limit; 4 arc-length limit; 8
 * innovation covariance not positive; 64 inconsistent track record). */
typedef struct {
  float* x;        /* device [capacity] */
  float* param;    /* device [capacity][5] */
  float* cov;      /* device [capacity][15] */
  float* chi2;     /* device [capacity] */
  int32_t* ndf;    /* device [capacity] */
  int32_t* flags;  /* device [capacity] */
  int64_t capacity;
} catpc_fits;

/* Cuts of the segment merging (catpc_merge_tracks). */
typedef struct {
  int32_t max_gap;  /* a continuation starts 1 .. max_gap rows above the segment's outermost hit (30) */
  float window;     /* cm: straight-line window in y and z at the continuation's start (10) */
  float chi2_max;   /* cut on the 5-parameter chi^2 of the two states (25) */
} catpc_merge_params;

/* Merged segments (caller-owned device memory), one entry per selected
 * track: next = the track that continues it (same sector, further out), or
 * -1; prev = the track it continues, or -1; head = the first segment of its
 * chain (itself when prev is -1), so the tracks of one chain share head;
 * chi2 = the chi^2 of the link to next, or -1. */
typedef struct {
  int32_t* next;  /* device [capacity] */
  int32_t* prev;  /* device [capacity] */
  int32_t* head;  /* device [capacity] */
  float* chi2;    /* device [capacity] */
  int64_t capacity;
} catpc_merges;

typedef struct catpc_ctx catpc_ctx;

/* Detector geometry (Sec. 2: the TPC's two halves are each divided into 18
 * trapezoidal sectors, every sector tracked on its own in its own frame, the
 * hits lying on the planes of its pad rows).  The sector frame: x along the
 * normal of the pad rows, y across them, z along the beam axis (the same
 * axis in every frame).  Sector s (0 <= s < 2 * sectors_per_side) sits on
 * side A (z >= 0) for s < sectors_per_side, else on side C, rotated about the
 * beam axis by alpha_s = ((s mod sectors_per_side) + 1/2) * 2 pi /
 * sectors_per_side; a point of the sector frame is (X, Y, Z) = (x cos alpha -
 * y sin alpha, x sin alpha + y cos alpha, z) in the global frame. */
typedef struct {
  int32_t n_rows;            /* pad rows per sector, 3 .. 4096 */
  const float* row_x;        /* host [n_rows]: x of each pad-row plane, cm, positive, strictly ascending */
  int32_t sectors_per_side;  /* sectors in each half of the TPC (18); 0 takes 18 */
} catpc_geometry;

/* Defaults of the method parameters and of the tuning. */
void catpc_default_params(catpc_params* p);
void catpc_default_tuning(catpc_tuning* t);
void catpc_default_merge_params(catpc_merge_params* m);

/* Row stride of the hit-per-row output: n_rows rounded up to a multiple of 8
 * (each tracklet's record is written in aligned 32-byte chunks). */
int32_t catpc_row_stride(int32_t n_rows);

/* Device workspace bytes catpc_create allocates for these maximum sizes. */
size_t catpc_workspace_bytes(int32_t n_rows, int64_t max_hits, int32_t max_sectors);

/* Create a tracker on the current HIP device for the geometry `geom` (its
 * row_x is copied) and the method parameters `params` (field, cluster
 * errors, cuts).  One tracker instance holds internal buffers sized once for
 * the largest input it will see (Sec. 4.1: the tracker's internal memory is
 * about three times the input): max_hits / max_sectors bound every later
 * call, and no later call allocates.  Returns CATPC_E_INVALID for a NULL or
 * inconsistent argument (n_rows outside [3, 4096], row_x not positive and
 * strictly ascending, sectors_per_side < 0, sizes out of range, bad
 * parameters), CATPC_E_HIP if allocation fails; *out is NULL on failure. */
catpc_status catpc_create(const catpc_geometry* geom, const catpc_params* params, int64_t max_hits,
                          int32_t max_sectors, catpc_ctx** out);
/* Free the tracker's device and pinned host memory and its captured graphs
 * (a NULL ctx is ignored).  Work enqueued with ctx must have completed; the
 * caller's output buffers are not touched. */
void catpc_destroy(catpc_ctx* ctx);

/* Frame of sector `sector_id` (host call, no device needed): its rotation
 * about the beam axis, rad, and side (+1 A, -1 C), as stated at
 * catpc_geometry.  CATPC_E_INVALID for a NULL argument or a sector id outside
 * [0, 2 * sectors_per_side). */
catpc_status catpc_sector_frame(const catpc_geometry* geom, int32_t sector_id, double* alpha, int32_t* side);

/* Tracklet (or track) parameters of sector `sector_id` in the global frame
 * (host call on host arrays, not part of the hot path; Sec. 2: tracking runs
 * in each sector's frame, the later steps across sectors need the global
 * one).  For each of the n entries: x[i] and param[i][0..4] = (y, z, sin phi,
 * tan lambda, q/pT) in the sector frame give out[i][0..5] = (X, Y, Z, phi,
 * tan lambda, q/pT): the global position, the global azimuth of the momentum
 * (asin(sin phi) + alpha, in (-pi, pi]), and the unchanged dip and signed
 * curvature parameters.  Computed in binary64.  CATPC_E_INVALID for NULL
 * arrays, n < 0, a sector id out of range, or |sin phi| > 1 (that entry's
 * output is NaN; the others are written). */
catpc_status catpc_to_global(const catpc_geometry* geom, int32_t sector_id, int64_t n, const float* x,
                             const float* param, double* out);

/* Replace the method parameters (field, cluster errors, windows, cuts,
 * limits, precision form) for later track calls; a captured graph made with
 * other parameters is captured again at the next batched call.
 * CATPC_E_INVALID for a NULL argument or a parameter out of range (cluster
 * errors <= 0, a negative window, cut, miss limit or hit count, precision
 * not 0-2); the previous parameters then stay. */
catpc_status catpc_set_params(catpc_ctx* ctx, const catpc_params* params);
/* Replace the launch shape for later calls (results never depend on it); a
 * graph captured with another shape is captured again.  CATPC_E_INVALID for a
 * NULL argument or a field out of its documented range; the previous tuning
 * then stays. */
catpc_status catpc_set_tuning(catpc_ctx* ctx, const catpc_tuning* tuning);
/* Copy the tracker's current launch shape to *tuning (CATPC_E_INVALID for a
 * NULL argument). */
catpc_status catpc_get_tuning(const catpc_ctx* ctx, catpc_tuning* tuning);

/* Batched form: the whole hot path (row index and grid build, neighbour
 * finding, link cleaning and start hits, tracklet construction, optional
 * precision refit) over all sectors of the input in a fixed chain of
 * launches, independent of the number of sectors (Sec. 3: one sector alone
 * does not hold enough parallel work for the GPU, and sectors are
 * independent; Sec. 3.2: several events are processed on the GPU at once);
 * replayed as a hipGraph when tuning.use_graph is set and the arguments
 * match the captured chain.  Tracklet slots [0, tracklet_capacity) are
 * written; see catpc_result.  CATPC_E_INVALID (outputs untouched) for NULL
 * arguments, sizes beyond those given to catpc_create, n_hits !=
 * hit_offset[n_sectors] when hit_offset_host is given, or misaligned
 * row_hit; CATPC_E_HIP if a launch fails. */
catpc_status catpc_track_batch(catpc_ctx* ctx, const catpc_input* in, const catpc_output* out, void* stream);

/* Plain form: the same stages launched sector by sector (Sec. 3, Fig. 3:
 * the earlier scheme processed one sector per kernel launch) -- the baseline
 * the batched form is measured against.  input.hit_offset_host is required
 * (CATPC_E_INVALID without it); errors as catpc_track_batch.  Output
 * identical to catpc_track_batch. */
catpc_status catpc_track_plain(catpc_ctx* ctx, const catpc_input* in, const catpc_output* out, void* stream);

/* Synchronise the stream and report (Sec. 3.1: the number of tracks is not
 * known in advance; the host reads the count back and fetches what did not
 * fit): CATPC_E_INVALID if the device found hits
 * that are not row-sorted or a row out of range (outputs undefined), else
 * CATPC_E_CAPACITY if the last track call found more tracklets than its
 * output slots, else CATPC_OK.  *n_tracklets (may be NULL) receives the total
 * number of tracklets of the last track call. */
catpc_status catpc_result(catpc_ctx* ctx, void* stream, int64_t* n_tracklets);

/* Late fetch (Sec. 3.1: queue an estimated output buffer, fetch the rest
 * afterwards): construct tracklet slots [first, first + out->tracklet_capacity)
 * of the last track call into out (slot first goes to index 0).  Only the
 * tracklet arrays of out are used.  The input must be the same, unchanged,
 * and no other track call may have run on ctx since. */
catpc_status catpc_fetch_tracklets(catpc_ctx* ctx, const catpc_input* in, int64_t first, const catpc_output* out,
                                   void* stream);

/* Number of stages reported by catpc_stage_times, in chain order:
 * 0 row index + input validation, 1 row grids, 2 neighbour finding,
 * 3 link cleaning + start-hit bits, 4 start-count scan, 5 start-list
 * compaction + per-sector tracklet offsets, 6 tracklet construction,
 * 7 precision refit (0 when precision == 0). */
#define CATPC_N_STAGES 8

/* Measurement: run the batched chain once without the graph, with a HIP event
 * before each stage, on `stream`; synchronise and write the elapsed
 * milliseconds of each stage to ms[CATPC_N_STAGES] (host).  Outputs as
 * catpc_track_batch. */
catpc_status catpc_stage_times(catpc_ctx* ctx, const catpc_input* in, const catpc_output* out, void* stream,
                               float* ms);

/* Measurement: the tracklet kernel's own count of method steps in the last
 * track call (accumulated over fetches): counts[0] helix transports,
 * [1] Kalman updates, [2] cluster candidates inside a following gate,
 * [3] row searches (host int64[4]).  Synchronises the stream. */
catpc_status catpc_work_counts(catpc_ctx* ctx, void* stream, int64_t* counts);

/* Numerics probe: out[i] = a[i] OP b[i] on the device in binary32 for
 * op 0 '+', 1 '-', 2 '*', 3 '/', 4 sqrt(a[i]), 5 the tracklet filter's
 * shorter correctly rounded square root (valid for normal a[i] >= 2^-96; b
 * unused for ops 4 and 5); device pointers, n elements.  Used to check that
 * the device rounds like the host and that op 5 equals op 4 on its domain. */
catpc_status catpc_fp32_probe(int32_t op, const float* a, const float* b, float* out, int64_t n, void* stream);

/* Phase clocks of the row-synchronous tracklet kernel, for a profiling build
 * of this library (kernels compiled with -DCATPC_PHASE_CLOCKS=1; in the
 * product build every call returns CATPC_E_INVALID and the kernel records
 * nothing).  The kernel sums shader-clock cycles over its waves, read by one
 * lane at points every lane of the wave reaches.  out (host uint64[
 * CATPC_PHASE_SLOTS]): [0] start of a slot batch (slots, chain records, seed
 * state), [1] outward pass (seed chain and following), [2] record store and
 * back-transport to the start row, [3] inward pass, [4] outward row steps,
 * [5] inward row steps, [6] slot batches, [7] whole-wave cycles, [8] waves;
 * summed since the last clear.  clear != 0: zero them (out unused).  The
 * device must be idle. */
#define CATPC_PHASE_SLOTS 9
catpc_status catpc_phase_clocks(uint64_t* out, int32_t clear);

/* Tracklet selection (Sec. 2 item 2: duplicate tracklets -- several seeds
 * that grew into the same segment -- are reduced to one per segment; Sec. 3:
 * this step follows the tracklet construction, many sectors per launch).
 * Reads the tracklets of a finished track call (`trk`: tracklet_offset,
 * flags, n_hits, row_hit) for the hits `in`.  Every hit goes to the heaviest
 * valid tracklet that lists it (weight: hit count, then the smaller
 * sector-local tracklet index); a tracklet that keeps at least min_hits of
 * its hits becomes a track of those hits.  Deterministic: the result does not
 * depend on the order of the device's atomics.  Asynchronous on `stream`;
 * catpc_select_result reports the totals.  Returns CATPC_E_INVALID for
 * missing or misaligned arrays. */
catpc_status catpc_select_tracklets(catpc_ctx* ctx, const catpc_input* in, const catpc_output* trk,
                                    const catpc_tracks* out, void* stream);

/* Full Kalman refit of the selected tracks (Sec. 2 item 4: the final fit
 * uses the full Kalman filter; constant field here).  Per track: the
 * tracklet's parameters carried row by row to the innermost hit, prior
 * covariance diag(sigma_y^2, sigma_z^2, 1, 1, 100), then row by row outward:
 * helix transport of the state, C <- F C F^T with the full first-order
 * Jacobian (z coupled to sin phi and q/pT), a 2-d Kalman update at each of
 * the track's hits; result at the outermost hit.  Reads `trk` (x_ref, param,
 * first_row, tracklet_offset) and `tracks` from a finished selection.
 * Requires out->capacity >= tracks->track_capacity (CATPC_E_INVALID
 * otherwise).  Asynchronous on `stream`. */
catpc_status catpc_refit_tracks(catpc_ctx* ctx, const catpc_input* in, const catpc_output* trk,
                                const catpc_tracks* tracks, const catpc_fits* out, void* stream);

/* Merging of track segments inside each sector (Sec. 2 item 3: segments of
 * one track that the following split, e.g. at a gap of rows without
 * clusters, are merged before the tracks are merged across sector borders;
 * that border step is not provided).  For a refitted track A (fit flags 1)
 * and a refitted track B of the same sector whose tracklet starts 1 to
 * max_gap rows above A's outermost hit:
 *  - A's fitted state carried along a straight line to B's start x must land
 *    within `window` of B's start state (the tracklet's state at x_ref) in y
 *    and in z;
 *  - A's state and covariance are carried row by row to B's first row with
 *    the refit's helix transport and Jacobian (binary64);
 *  - chi^2 = d^T (C_A + C_B)^-1 d over the five parameters, d = B's start
 *    state - A's carried state, by Cholesky factorisation; the pair is
 *    compatible when C_A + C_B is positive definite and chi^2 <= chi2_max.
 * A's best continuation and B's best predecessor order by chi^2 rounded to
 * binary32, ties to the smaller track index; A and B are linked when each is
 * the other's best.  Deterministic (the best predecessor is a 64-bit atomic
 * minimum of (chi^2, index), independent of the order of the atomics).
 * Reads `trk` (x_ref, param, cov, first_row, tracklet_offset), `tracks`
 * (with track_hits, for the outermost hit's row) and `fits` of the same
 * selection; `mp` NULL takes the defaults.  Requires fits->capacity and
 * out->capacity >= tracks->track_capacity (CATPC_E_INVALID otherwise);
 * CATPC_E_INVALID for max_gap outside [1, 4096] or negative cuts.
 * Asynchronous on `stream`. */
catpc_status catpc_merge_tracks(catpc_ctx* ctx, const catpc_input* in, const catpc_output* trk,
                                const catpc_tracks* tracks, const catpc_fits* fits, const catpc_merge_params* mp,
                                const catpc_merges* out, void* stream);

/* Measurement: synchronise `stream` and report the last merge call's
 * candidate pairs (those that passed the row and window tests) and the row
 * steps their transports took. */
catpc_status catpc_merge_counts(catpc_ctx* ctx, void* stream, int64_t* n_pairs, int64_t* n_steps);

/* Synchronise `stream` and report the last selection: the number of tracks
 * and of their hits.  CATPC_E_CAPACITY if the output held fewer, or if the
 * tracklet output held only part of the tracklets (then the selection covers
 * only those); CATPC_E_INVALID if a tracklet record named a hit that is not
 * a hit of its sector in the row the entry stands for (such entries are
 * skipped); CATPC_E_STATE without a selection since the last track call. */
catpc_status catpc_select_result(catpc_ctx* ctx, void* stream, int64_t* n_tracks, int64_t* n_track_hits);

/* The batched form without any allocation, for callers that cannot allocate
 * device or pinned memory: code being captured into a HIP graph, tight
 * serving loops, harnesses that forbid hipMalloc.  Same stage chain, results
 * and tuning as catpc_track_batch (launched directly, no graph), without a
 * context: the workspace is a fixed 96 MiB device array inside the library,
 * one copy per device, held until the process ends -- enough for about
 * 1.9 M hits in 36 sectors of 159 pad rows (a central event); larger inputs
 * are rejected with CATPC_E_INVALID (nothing enqueued).  row_x: DEVICE
 * [n_rows], the pad-row planes; params / tuning: host (tuning NULL = the
 * defaults).  status: DEVICE uint64, written at the end of the chain with the
 * error bits found on the device (1: hits not row-sorted or a row out of
 * range; 8: x differs from the row planes; 64: row_x not positive and
 * strictly ascending; 0: none).  The number of tracklets is
 * tracklet_offset[n_sectors]; slots beyond tracklet_capacity are not
 * written (no late fetch).  Asynchronous on `stream`.  Every call on a
 * device shares that device's array: calls that overlap on one device (other
 * streams, other threads) race and must be serialised by the caller. */
catpc_status catpc_track_batch_noalloc(int32_t n_rows, const float* row_x, const catpc_params* params,
                                       const catpc_tuning* tuning, const catpc_input* in, const catpc_output* out,
                                       uint64_t* status, void* stream);

/* Achievable-peak probes (measurement only, no tracking): a device copy of
 * n_bytes (a multiple of 16; 16-byte aligned device pointers), and in each of
 * n_threads threads 8 independent chains of n_iter binary32 fused
 * multiply-adds (16 * n_iter flops per thread; out[i] receives a sum so the
 * work stays).  Asynchronous on `stream`; time them with events there. */
catpc_status catpc_probe_copy(const void* src, void* dst, int64_t n_bytes, void* stream);
catpc_status catpc_probe_fma(float* out, int64_t n_threads, int32_t n_iter, void* stream);

/* Thread-local text of the last error. */
const char* catpc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
