/*
 * CPU oracle: tracklet selection (integer work).  Test infrastructure only;
 * see oracle.h.
 *
 * Sec. 2 item 2: duplicate tracklets (several seeds grown into one segment)
 * are reduced to one per segment; Sec. 3: this step follows the tracklet
 * construction, several sectors per launch.
 * Reading used here (one pass, order-independent):
 *  - only valid tracklets (flag VALID: at least min_hits hits) take part;
 *  - a tracklet's weight is its hit count; between equal counts the smaller
 *    sector-local tracklet index is better;
 *  - every hit belongs to the best tracklet that lists it;
 *  - a tracklet is selected when it owns at least min_hits of its hits; its
 *    track segment is the list of hits it owns, by ascending row;
 *  - hits owned by a tracklet that is not selected are not handed on.
 */
#include <stdlib.h>

#include "oracle.h"

/* weight of tracklet t with n hits: larger is better */
static uint64_t weight(int32_t n, int32_t t) {
  return ((uint64_t)(uint32_t)n << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)t);
}

int32_t oracle_select(int32_t n_hits, int32_t n_rows, int32_t n_trk, const int32_t* row_hit,
                      const int32_t* trk_n_hits, const int32_t* flags, int32_t min_hits,
                      int32_t* owned, int32_t* track_hits, int32_t* n_tracks, int32_t* n_track_hits) {
  uint64_t* owner = (uint64_t*)calloc((size_t)(n_hits > 0 ? n_hits : 1), sizeof(uint64_t));
  if (!owner) return -1;
  for (int32_t t = 0; t < n_trk; ++t) {
    if (!(flags[t] & ORACLE_VALID)) continue;
    const uint64_t w = weight(trk_n_hits[t], t);
    for (int32_t r = 0; r < n_rows; ++r) {
      const int32_t h = row_hit[(int64_t)t * n_rows + r];
      if (h < 0) continue;
      if (h >= n_hits) { free(owner); return -2; }
      if (w > owner[h]) owner[h] = w;
    }
  }
  int32_t nt = 0, nh = 0;
  for (int32_t t = 0; t < n_trk; ++t) {
    owned[t] = 0;
    if (!(flags[t] & ORACLE_VALID)) continue;
    const uint64_t w = weight(trk_n_hits[t], t);
    int32_t c = 0;
    for (int32_t r = 0; r < n_rows; ++r) {
      const int32_t h = row_hit[(int64_t)t * n_rows + r];
      if (h >= 0 && owner[h] == w) ++c;
    }
    if (c < min_hits) continue;
    owned[t] = c;
    for (int32_t r = 0; r < n_rows; ++r) {
      const int32_t h = row_hit[(int64_t)t * n_rows + r];
      if (h >= 0 && owner[h] == w) track_hits[nh++] = h;
    }
    ++nt;
  }
  *n_tracks = nt;
  *n_track_hits = nh;
  free(owner);
  return 0;
}
