/*
 * Plain CPU oracle for the sector-tracking hot path (test infrastructure).
 *
 * ONLY tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py
 * may load or call this library.  It shares no code with the HIP path.
 *
 * Everything here works on ONE sector: hits in the sector-local frame, sorted
 * by pad row, indices sector-local.  The floating-point functions exist in two
 * builds of the same source: *_f32 (every + - * / sqrt rounded to nearest in
 * binary32, no contraction) and *_f64 (the same sequence in binary64).
 *
 * Paper: Rohr, Gorbunov, Lindenstruth, "GPU-accelerated track reconstruction
 * in the ALICE High Level Trigger" (arXiv:1712.09430), Sec. 2 (seeding by a
 * cellular automaton, track following with a simplified Kalman filter).
 */
#ifndef CATPC_ORACLE_H
#define CATPC_ORACLE_H
#include <stdint.h>

typedef struct {
  float bz;             /* field, T */
  float sigma_y;        /* cluster error in y, cm */
  float sigma_z;        /* cluster error in z, cm */
  float nf_win_y;       /* neighbour window half-width in y, cm */
  float nf_win_z;       /* neighbour window half-width in z, cm */
  float nf_chi2_max;    /* cut on the 3-point residual, cm^2 */
  float tc_gate_nsigma; /* following gate in units of the predicted error */
  int32_t tc_max_miss;  /* following stops after more consecutive misses than this */
  int32_t min_hits;     /* tracklets with fewer hits are not flagged valid */
  int32_t precision;    /* f32 build: 0 none, 1 refit SPD failures with FP64 covariance, 2 refit all */
} oracle_params;

/* tracklet flag bits */
#define ORACLE_VALID 1
#define ORACLE_STOP_SINPHI 2
#define ORACLE_STOP_ARC 4
#define ORACLE_SPD_FAIL 8
#define ORACLE_REFIT64 16

/* state vector layout used by the unit entry points (15 values):
 * x, y, z, s=sin(phi), l=tan(lambda), q=q/pT,
 * transverse covariance over (y, s, q): c_yy, c_sy, c_ss, c_qy, c_qs, c_qq,
 * longitudinal covariance over (z, l): c_zz, c_lz, c_ll */

#define ORACLE_DECL(SFX, REAL)                                                                     \
  int32_t oracle_neighbours##SFX(int32_t n_rows, const float* row_x, int32_t n, const float* y,   \
                                 const float* z, const int32_t* row, const oracle_params* p,       \
                                 int32_t* link_up, int32_t* link_dn);                              \
  int32_t oracle_tracklets##SFX(int32_t n_rows, const float* row_x, int32_t n, const float* y,    \
                                const float* z, const int32_t* row, const int32_t* up_clean,       \
                                int32_t n_start, const int32_t* start, const oracle_params* p,     \
                                REAL* x_ref, REAL* param, REAL* cov, int32_t* row_hit,             \
                                int32_t* start_row, int32_t* first_row, int32_t* last_row,         \
                                int32_t* n_hits, int32_t* flags, int64_t* counters);               \
  int32_t oracle_refit##SFX(int32_t n_rows, const float* row_x, int32_t n, const float* y,        \
                            const float* z, int32_t n_trk, const int32_t* row_hit,                 \
                            const int32_t* start_row, const oracle_params* p, REAL* x_ref,         \
                            REAL* param, REAL* cov, int32_t* flags);                               \
  int32_t oracle_init##SFX(const REAL* h0, const REAL* h1, const oracle_params* p, REAL* st);     \
  int32_t oracle_propagate##SFX(REAL* st, REAL x1, const oracle_params* p);                       \
  int32_t oracle_update##SFX(REAL* st, REAL my, REAL mz, const oracle_params* p);                 \
  int32_t oracle_spd##SFX(const REAL* st);

ORACLE_DECL(_f32, float)
ORACLE_DECL(_f64, double)

int32_t oracle_clean_links(int32_t n, const int32_t* link_up, const int32_t* link_dn,
                           int32_t* up_clean, int32_t* dn_clean, uint8_t* is_start);

int32_t oracle_refit_mixed(int32_t n_rows, const float* row_x, int32_t n, const float* y,
                           const float* z, int32_t n_trk, const int32_t* row_hit,
                           const int32_t* start_row, const oracle_params* p, float* x_ref,
                           float* param, float* cov, int32_t* spd_ok);

/* Tracklet selection of one sector (select.c).  row_hit [n_trk][n_rows];
 * outputs: owned[t] = hits tracklet t keeps if selected, else 0; track_hits =
 * the selected tracklets' kept hits, tracklet by tracklet, rows ascending;
 * n_tracks, n_track_hits = counts.  Returns 0, or <0 for a hit index out of
 * range (-2) or no memory (-1). */
int32_t oracle_select(int32_t n_hits, int32_t n_rows, int32_t n_trk, const int32_t* row_hit,
                      const int32_t* trk_n_hits, const int32_t* flags, int32_t min_hits,
                      int32_t* owned, int32_t* track_hits, int32_t* n_tracks, int32_t* n_track_hits);

/* Full Kalman refit of one track (fullfit.c), both builds.  rows/hy/hz: the
 * track's hits by ascending row; (x_start, p_start) the start state at
 * row start_row.  Outputs at the outermost hit: x, p[5], packed covariance
 * C[15] over (y, z, sin phi, tan lambda, q/pT), chi^2, ndf = 2 hits - 5,
 * flags: 1 done, 2 |sin phi| limit, 4 arc-length limit, 8 innovation
 * covariance not positive, 64 bad input. */
#define ORACLE_FULLFIT_DECL(SFX, REAL)                                                                   \
  int32_t oracle_fullfit##SFX(int32_t n_rows, const float* row_x, int32_t n, const int32_t* rows,        \
                              const float* hy, const float* hz, REAL x_start, const REAL* p_start,       \
                              int32_t start_row, const oracle_params* prm, REAL* x_out, REAL* p_out,      \
                              REAL* C_out, REAL* chi2_out, int32_t* ndf_out, int32_t* flags_out);
ORACLE_FULLFIT_DECL(_f32, float)
ORACLE_FULLFIT_DECL(_f64, double)
/* One transport step of the refit (state x, p[5], packed C[15]) to x1:
 * returns 0, 2 or 4 as the transport of the tracklet filter. */
int32_t oracle_fullfit_transport_f32(float* x, float* p, float* C, float x1, const oracle_params* prm);
int32_t oracle_fullfit_transport_f64(double* x, double* p, double* C, double x1, const oracle_params* prm);

/* Merging of track segments of one sector across row gaps (merge.c), binary64.
 * Per track: ok (refit done), a_last (row of its outermost hit), end state
 * e_x, e_p[5], e_C[15] (the refit result), b_first (its tracklet's first
 * row), start state s_x, s_p[5], s_C[15] (the tracklet's state at x_ref).
 * Output: next[a] = the track that continues track a, or -1, and the chi^2
 * of that link rounded to binary32, else -1. */
typedef struct {
  int32_t max_gap; /* B's first row at most this many rows above A's last */
  float window;    /* cm, straight-line window in y and z */
  float chi2_max;  /* cut on the 5-parameter chi^2 */
} oracle_merge_params;
int32_t oracle_merge(int32_t n_rows, const float* row_x, const oracle_params* prm, const oracle_merge_params* mp,
                     int32_t n, const int32_t* ok, const int32_t* a_last, const float* e_x, const float* e_p,
                     const float* e_C, const int32_t* b_first, const float* s_x, const float* s_p, const float* s_C,
                     int32_t* next, float* chi2_out);

#endif
