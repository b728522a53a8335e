/*
 * CPU oracle: link cleaning and start hits (integer work).  Test
 * infrastructure only; see oracle.h.
 *
 * Sec. 2 item 1: the cellular automaton builds short seeds ("usually 3 to
 * about 10 clusters") out of neighbour links; seeds are oriented along x and
 * every hit carries at most one hypothesis (Sec. 2, linearity paragraph).
 * Reading used here: a link survives only if it is mutual (the up-neighbour of
 * i names i as its down-neighbour, and vice versa), all decided on the
 * uncleaned links; a hit starts a seed when it has no surviving down-link, a
 * surviving up-link j, and j has a surviving up-link (at least 3 hits).
 * Surviving links form disjoint chains that climb one row per link.
 */
#include "oracle.h"

int32_t oracle_clean_links(int32_t n, const int32_t* up, const int32_t* dn, int32_t* up_clean,
                           int32_t* dn_clean, uint8_t* is_start) {
  for (int32_t i = 0; i < n; ++i) {
    const int32_t j = up[i];
    up_clean[i] = (j >= 0 && dn[j] == i) ? j : -1;
    const int32_t k = dn[i];
    dn_clean[i] = (k >= 0 && up[k] == i) ? k : -1;
  }
  for (int32_t i = 0; i < n; ++i) {
    const int32_t j = up_clean[i];
    is_start[i] = (uint8_t)(dn_clean[i] < 0 && j >= 0 && up_clean[j] >= 0);
  }
  return 0;
}
