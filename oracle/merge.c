/*
 * CPU oracle: merging of track segments inside a sector across a row gap
 * (test infrastructure only; see oracle.h).
 *
 * Sec. 2 item 3: track segments inside one sector that belong to one track
 * (the following lost the track over a gap) are merged, before the merging
 * across sector borders (not built here).  Reading used here, in binary64:
 *  - candidates: two refitted tracks A, B of one sector, B's tracklet
 *    starting 1 to max_gap rows above A's outermost hit;
 *  - a straight-line window: A's end state carried along its direction to
 *    B's start x lands within `window` cm of B's start in y and in z;
 *  - A's end state and covariance carried row by row with the refit's
 *    transport (no updates) to B's first row; with d = (B's start state) -
 *    (A's carried state) and V = C_A + C_B, chi^2 = d^T V^-1 d (Cholesky of
 *    V, forward substitution); compatible when V is positive definite and
 *    chi^2 <= chi2_max;
 *  - the best B of A and the best A of B order by chi^2 rounded to binary32,
 *    ties to the smaller track index; A and B are linked when each is the
 *    other's best.
 */
#include <math.h>

#include "oracle.h"

static int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

/* chi^2 of the pair (A's end, B's start), or -1 when not compatible */
static double pair_chi2(int32_t n_rows, const float* row_x, const oracle_params* prm, const oracle_merge_params* mp,
                        int32_t a_last, float a_x, const float* a_p, const float* a_C, int32_t b_first, float b_x,
                        const float* b_p, const float* b_C) {
  if (!(b_first > a_last && b_first - a_last <= mp->max_gap && b_first < n_rows && a_last >= 0)) return -1.0;
  const double dx0 = (double)b_x - (double)a_x;
  const double s = (double)a_p[2];
  const double c = sqrt(1.0 - s * s);
  const double yw = ((double)a_p[0] + dx0 * (s / c)) - (double)b_p[0];
  const double zw = ((double)a_p[1] + dx0 * ((double)a_p[3] / c)) - (double)b_p[1];
  if (!(fabs(yw) <= (double)mp->window && fabs(zw) <= (double)mp->window)) return -1.0;
  double x = (double)a_x, p[5], C[15];
  for (int i = 0; i < 5; ++i) p[i] = (double)a_p[i];
  for (int q = 0; q < 15; ++q) C[q] = (double)a_C[q];
  for (int32_t r = a_last + 1; r <= b_first; ++r)
    if (oracle_fullfit_transport_f64(&x, p, C, (double)row_x[r], prm)) return -1.0;
  double d[5], L[5][5];
  for (int i = 0; i < 5; ++i) d[i] = (double)b_p[i] - p[i];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) L[i][j] = 0.0;
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j) {
      double acc = C[tri(i, j)] + (double)b_C[tri(i, j)];
      for (int q = 0; q < j; ++q) acc = acc - L[i][q] * L[j][q];
      if (i == j) {
        if (!(acc > 0.0)) return -1.0;
        L[i][i] = sqrt(acc);
      } else {
        L[i][j] = acc / L[j][j];
      }
    }
  double w[5], chi2 = 0.0;
  for (int i = 0; i < 5; ++i) {
    double acc = d[i];
    for (int q = 0; q < i; ++q) acc = acc - L[i][q] * w[q];
    w[i] = acc / L[i][i];
    chi2 = chi2 + w[i] * w[i];
  }
  return chi2 <= (double)mp->chi2_max ? chi2 : -1.0;
}

int32_t oracle_merge(int32_t n_rows, const float* row_x, const oracle_params* prm, const oracle_merge_params* mp,
                     int32_t n, const int32_t* ok, const int32_t* a_last, const float* e_x, const float* e_p,
                     const float* e_C, const int32_t* b_first, const float* s_x, const float* s_p, const float* s_C,
                     int32_t* next, float* chi2_out) {
#define CHI2(A, B)                                                                                            \
  pair_chi2(n_rows, row_x, prm, mp, a_last[A], e_x[A], e_p + 5 * (A), e_C + 15 * (A), b_first[B], s_x[B], \
            s_p + 5 * (B), s_C + 15 * (B))
  for (int32_t a = 0; a < n; ++a) {
    next[a] = -1;
    chi2_out[a] = -1.0f;
  }
  for (int32_t a = 0; a < n; ++a) {
    if (!ok[a]) continue;
    /* A's best continuation */
    int32_t b_best = -1;
    float c_best = 0.0f;
    for (int32_t b = 0; b < n; ++b) {
      if (b == a || !ok[b]) continue;
      const double c = CHI2(a, b);
      if (c < 0.0) continue;
      const float cf = (float)c;
      if (b_best < 0 || cf < c_best) {
        b_best = b;
        c_best = cf;
      }
    }
    if (b_best < 0) continue;
    /* the best predecessor of that continuation */
    int32_t a_best = -1;
    float ca_best = 0.0f;
    for (int32_t a2 = 0; a2 < n; ++a2) {
      if (a2 == b_best || !ok[a2]) continue;
      const double c = CHI2(a2, b_best);
      if (c < 0.0) continue;
      const float cf = (float)c;
      if (a_best < 0 || cf < ca_best) {
        a_best = a2;
        ca_best = cf;
      }
    }
    if (a_best == a) {
      next[a] = b_best;
      chi2_out[a] = c_best;
    }
  }
#undef CHI2
  return 0;
}
