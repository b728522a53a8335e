/*
 * CPU oracle: neighbour finding and tracklet construction for one TPC sector.
 * Test infrastructure only (see oracle.h): plain loops, brute-force searches,
 * no blocking, no binning, no reordering.
 *
 * Compiled twice from this one source: with ORACLE_F32 defined every
 * arithmetic operation is a binary32 operation rounded to nearest (the build
 * uses -ffp-contract=off, so no fused multiply-add), otherwise binary64.
 *
 * The paper (arXiv:1712.09430) states the method in words only: Sec. 2 item 1
 * (seeding: a cellular automaton links each hit to neighbours in adjacent pad
 * rows, seeds are short chains oriented along x, one hypothesis per seed),
 * Sec. 2 item 2 (track following: fit the seed, extrapolate row by row
 * through the sector, add the closest cluster of each row, refine the
 * parameters with a simplified Kalman filter that takes uncorrelated
 * coordinate errors and a constant field), Fig. 2 c, d and Tab. 1.  Every
 * number and formula below that the text does not give is a reading, named
 * where it is used.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#ifdef ORACLE_F32
typedef float real;
#define SFX(name) name##_f32
#define RSQRT(v) sqrtf(v)
#define RABS(v) fabsf(v)
#define LIT(v) v##f
#define RMAX FLT_MAX
#else
typedef double real;
#define SFX(name) name##_f64
#define RSQRT(v) sqrt(v)
#define RABS(v) fabs(v)
#define LIT(v) v
#define RMAX DBL_MAX
#endif

/* ------------------------------------------------------------ constants */
typedef struct {
  real kb;       /* curvature per unit q/pT: k = kb * q, kb = -0.00299792458 * Bz (cm^-1 / (GeV^-1)) */
  real sy2, sz2; /* cluster variances */
  real wy, wz, chi2;
  real nsig;
  int max_miss, min_hits;
} consts;

static consts make_consts(const oracle_params* p) {
  consts c;
  c.kb = LIT(-0.00299792458) * (real)p->bz;
  c.sy2 = (real)p->sigma_y * (real)p->sigma_y;
  c.sz2 = (real)p->sigma_z * (real)p->sigma_z;
  c.wy = (real)p->nf_win_y;
  c.wz = (real)p->nf_win_z;
  c.chi2 = (real)p->nf_chi2_max;
  c.nsig = (real)p->tc_gate_nsigma;
  c.max_miss = p->tc_max_miss;
  c.min_hits = p->min_hits;
  return c;
}

/* Row ranges of a row-sorted sector: hits of row r are [first[r], first[r+1]).
 * Returns NULL if the rows are not sorted or out of range. */
static int32_t* row_ranges(int32_t n_rows, int32_t n, const int32_t* row) {
  int32_t* first = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_rows + 1));
  int32_t r = 0;
  first[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (row[i] < 0 || row[i] >= n_rows || (i > 0 && row[i] < row[i - 1])) { free(first); return NULL; }
    while (r < row[i]) first[++r] = i;
  }
  while (r < n_rows) first[++r] = n;
  return first;
}

/* ================================================ neighbour finding (CA) */
/*
 * Sec. 2 item 1 and Fig. 2c: for each hit of row r (1 <= r <= n_rows-2) the
 * cellular automaton looks for the best pair of neighbours, one in row r+1
 * ("up") and one in row r-1 ("down").  Primary tracks are taken to run
 * outward from the origin along x (Sec. 2), so a candidate is searched around
 * the straight line from the origin through the hit, scaled to the other
 * row's x:  y * x_{r+-1} / x_r, z * x_{r+-1} / x_r, inside a window of
 * half-width (wy, wz).  A pair (up j, down k) is scored by the squared
 * distance between the hit and the chord from k to j evaluated at x_r; the
 * pair with the smallest score wins if the score is within chi2.  Ties go to
 * the smaller (j, k).  Rows 0 and n_rows-1 get no links.
 *
 * This is the plain definition: all hits of the two adjacent rows are
 * examined.
 */
int32_t SFX(oracle_neighbours)(int32_t n_rows, const float* row_x, int32_t n, const float* y,
                               const float* z, const int32_t* row, const oracle_params* p,
                               int32_t* link_up, int32_t* link_dn) {
  const consts c = make_consts(p);
  int32_t* first = row_ranges(n_rows, n, row);
  if (!first) return -1;
  for (int32_t i = 0; i < n; ++i) { link_up[i] = -1; link_dn[i] = -1; }
  for (int32_t i = 0; i < n; ++i) {
    const int32_t r = row[i];
    if (r < 1 || r > n_rows - 2) continue;
    const real xr = (real)row_x[r], xu = (real)row_x[r + 1], xd = (real)row_x[r - 1];
    const real fu = xu / xr;
    const real fd = xd / xr;
    const real t = (xr - xd) / (xu - xd);
    const real yi = (real)y[i], zi = (real)z[i];
    const real yu = yi * fu, zu = zi * fu;
    const real yd = yi * fd, zd = zi * fd;
    int32_t bj = -1, bk = -1;
    real best = 0;
    for (int32_t j = first[r + 1]; j < first[r + 2]; ++j) {
      const real yj = (real)y[j], zj = (real)z[j];
      if (!(RABS(yj - yu) <= c.wy && RABS(zj - zu) <= c.wz)) continue;
      for (int32_t k = first[r - 1]; k < first[r]; ++k) {
        const real yk = (real)y[k], zk = (real)z[k];
        if (!(RABS(yk - yd) <= c.wy && RABS(zk - zd) <= c.wz)) continue;
        const real ey = yi - (yk + t * (yj - yk));
        const real ez = zi - (zk + t * (zj - zk));
        const real chi2 = ey * ey + ez * ez;
        if (!(chi2 <= c.chi2)) continue;
        if (bj < 0 || chi2 < best || (chi2 == best && (j < bj || (j == bj && k < bk)))) {
          best = chi2; bj = j; bk = k;
        }
      }
    }
    link_up[i] = bj;
    link_dn[i] = bk;
  }
  free(first);
  return 0;
}

/* ====================================================== Kalman filter */
/*
 * Track model (Sec. 2 item 2): a helix in a constant field Bz.  State at
 * position x: (y, z, s = sin phi, l = tan lambda, q = q/pT).  The simplified
 * filter takes the y and z measurement errors as uncorrelated, which is read
 * here as two independent blocks: transverse (y, s, q) and longitudinal (z, l);
 * the covariance between the blocks is zero throughout.
 */
typedef struct {
  real x, y, z, s, l, q;
  real c00, c10, c11, c20, c21, c22; /* (y,y) (s,y) (s,s) (q,y) (q,s) (q,q) */
  real d00, d10, d11;                /* (z,z) (l,z) (l,l) */
} track;

enum { STEP_OK = 0, STEP_SINPHI = 1, STEP_ARC = 2 };

/* Seed initialisation from the start hit h0 and its upward neighbour h1:
 * position of h0, direction of the chord h0 -> h1, q/pT = 0, and a diffuse
 * prior diag(sy2, sz2, 1, 1, 100); h0 itself counts as already fitted. */
static int init_track(track* t, real x0, real y0, real z0, real x1, real y1, real z1, const consts* c) {
  const real dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
  const real L = RSQRT(dx * dx + dy * dy);
  t->x = x0; t->y = y0; t->z = z0;
  t->s = dy / L;
  t->l = dz / L;
  t->q = 0;
  t->c00 = c->sy2; t->c10 = 0; t->c11 = 1; t->c20 = 0; t->c21 = 0; t->c22 = 100;
  t->d00 = c->sz2; t->d10 = 0; t->d11 = 1;
  return RABS(t->s) < LIT(0.999) ? STEP_OK : STEP_SINPHI;
}

/*
 * Transport to the plane x1 along the exact helix (constant field):
 * sin phi moves linearly with x, s1 = s + k dx; y moves by dx times the chord
 * slope (s + s1) / (c + c1) with c = sqrt(1 - s^2); z moves by tan lambda
 * times the arc length, arc = chord * asin(u) / u with u = k chord / 2, where
 * asin(u)/u is its Maclaurin series through u^8 (no transcendental call).
 * Stops when |s1| >= 0.999 or |u| > 0.2 (outside the series' range).
 * Covariance: C <- J C J^T per block with
 *   dy/ds = dx / cm^3, dy/dq = kb dx^2 / 2 / cm^3, ds/dq = kb dx, dz/dl = arc,
 * cm the cosine at the mean sin phi; no process noise.
 */
static int propagate(track* t, real x1, const consts* c) {
  const real dx = x1 - t->x;
  const real k = c->kb * t->q;
  const real s0 = t->s;
  const real s1 = s0 + k * dx;
  if (!(RABS(s1) < LIT(0.999))) return STEP_SINPHI;
  const real c0 = RSQRT((real)1 - s0 * s0);
  const real c1 = RSQRT((real)1 - s1 * s1);
  const real T = (s0 + s1) / (c0 + c1);
  const real dy = dx * T;
  const real ch = RSQRT(dx * dx + dy * dy);
  const real u = (k * ch) * LIT(0.5);
  if (!(RABS(u) <= LIT(0.2))) return STEP_ARC;
  const real u2 = u * u;
  const real A = (real)1 + u2 * ((real)1 / (real)6 +
                            u2 * ((real)3 / (real)40 + u2 * ((real)5 / (real)112 + u2 * ((real)35 / (real)1152))));
  real dS = ch * A;
  if (dx < 0) dS = -dS;

  const real sm = (s0 + s1) * LIT(0.5);
  const real cm2 = (real)1 - sm * sm;
  const real cm3 = cm2 * RSQRT(cm2);
  const real a = dx / cm3;
  const real b = ((c->kb * dx) * dx * LIT(0.5)) / cm3;
  const real d = c->kb * dx;

  t->x = x1;
  t->y = t->y + dy;
  t->z = t->z + t->l * dS;
  t->s = s1;

  const real c00 = t->c00, c10 = t->c10, c11 = t->c11, c20 = t->c20, c21 = t->c21, c22 = t->c22;
  const real m0 = c00 + a * c10 + b * c20;
  const real m1 = c10 + a * c11 + b * c21;
  const real m2 = c20 + a * c21 + b * c22;
  const real n1 = c11 + d * c21;
  const real n2 = c21 + d * c22;
  t->c00 = m0 + a * m1 + b * m2;
  t->c10 = m1 + d * m2;
  t->c11 = n1 + d * n2;
  t->c20 = m2;
  t->c21 = n2;
  t->c22 = c22;

  const real tz = t->d10 + dS * t->d11;
  t->d00 = t->d00 + dS * t->d10 + dS * tz;
  t->d10 = tz;
  return STEP_OK;
}

/* One Kalman update with the measurement (my, mz) of a cluster at the
 * current x: two independent scalar updates (y on the transverse block, z on
 * the longitudinal block).  Fails (and the caller discards the result) if
 * |sin phi| reaches 0.999. */
static int update(track* t, real my, real mz, const consts* c) {
  const real ry = my - t->y;
  const real Sy = t->c00 + c->sy2;
  const real iy = (real)1 / Sy;
  const real k0 = t->c00 * iy, k1 = t->c10 * iy, k2 = t->c20 * iy;
  t->y = t->y + k0 * ry;
  t->s = t->s + k1 * ry;
  t->q = t->q + k2 * ry;
  const real c00 = t->c00, c10 = t->c10, c20 = t->c20;
  t->c00 = c00 - k0 * c00;
  t->c10 = c10 - k1 * c00;
  t->c20 = c20 - k2 * c00;
  t->c11 = t->c11 - k1 * c10;
  t->c21 = t->c21 - k2 * c10;
  t->c22 = t->c22 - k2 * c20;

  const real rz = mz - t->z;
  const real Sz = t->d00 + c->sz2;
  const real iz = (real)1 / Sz;
  const real g0 = t->d00 * iz, g1 = t->d10 * iz;
  t->z = t->z + g0 * rz;
  t->l = t->l + g1 * rz;
  const real d00 = t->d00, d10 = t->d10;
  t->d00 = d00 - g0 * d00;
  t->d10 = d10 - g1 * d00;
  t->d11 = t->d11 - g1 * d10;
  return RABS(t->s) < LIT(0.999) ? STEP_OK : STEP_SINPHI;
}

/* Positive-definiteness check: LDL^T pivots of the 3x3 transverse block and
 * the 2x2 longitudinal block must all be finite and > 0. */
static int spd_ok(const track* t) {
  const real p0 = t->c00;
  if (!(p0 > 0 && p0 <= RMAX)) return 0;
  const real i0 = (real)1 / p0;
  const real a = t->c10 * i0;
  const real p1 = t->c11 - a * t->c10;
  if (!(p1 > 0 && p1 <= RMAX)) return 0;
  const real b = t->c20 * i0;
  const real e = t->c21 - b * t->c10;
  const real g = e / p1;
  const real p2 = (t->c22 - b * t->c20) - g * e;
  if (!(p2 > 0 && p2 <= RMAX)) return 0;
  const real q0 = t->d00;
  if (!(q0 > 0 && q0 <= RMAX)) return 0;
  const real q1 = t->d11 - (t->d10 / q0) * t->d10;
  if (!(q1 > 0 && q1 <= RMAX)) return 0;
  return 1;
}

/* Closest cluster of row r to the predicted position (Fig. 2d): among hits
 * with |dy| <= nsig * sqrt(C_yy + sy2) and |dz| <= nsig * sqrt(C_zz + sz2),
 * the smallest dy^2 + dz^2, ties to the smaller index.  Brute force over the
 * whole row. */
static int32_t closest(const track* t, int32_t lo, int32_t hi, const float* y, const float* z,
                       const consts* c, int64_t* counters) {
  const real gy = c->nsig * RSQRT(t->c00 + c->sy2);
  const real gz = c->nsig * RSQRT(t->d00 + c->sz2);
  int32_t best = -1;
  real bd = 0;
  counters[3] += 1;
  for (int32_t j = lo; j < hi; ++j) {
    const real dy = (real)y[j] - t->y;
    const real dz = (real)z[j] - t->z;
    if (!(RABS(dy) <= gy && RABS(dz) <= gz)) continue;
    counters[2] += 1;
    const real d2 = dy * dy + dz * dz;
    if (best < 0 || d2 < bd) { best = j; bd = d2; }
  }
  return best;
}

static void store(const track* t, int64_t i, real* x_ref, real* param, real* cov) {
  x_ref[i] = t->x;
  real* pp = param + 5 * i;
  pp[0] = t->y; pp[1] = t->z; pp[2] = t->s; pp[3] = t->l; pp[4] = t->q;
  real* cc = cov + 15 * i;
  for (int k = 0; k < 15; ++k) cc[k] = 0;
  /* packed lower triangle over (y, z, s, l, q): (i,j) -> i(i+1)/2 + j */
  cc[0] = t->c00;  /* (y,y) */
  cc[2] = t->d00;  /* (z,z) */
  cc[3] = t->c10;  /* (s,y) */
  cc[5] = t->c11;  /* (s,s) */
  cc[7] = t->d10;  /* (l,z) */
  cc[9] = t->d11;  /* (l,l) */
  cc[10] = t->c20; /* (q,y) */
  cc[12] = t->c21; /* (q,s) */
  cc[14] = t->c22; /* (q,q) */
}

static int stop_flag(int e) { return e == STEP_SINPHI ? ORACLE_STOP_SINPHI : ORACLE_STOP_ARC; }

/*
 * Tracklet construction (Sec. 2 item 2, Fig. 2d, Tab. 1 row 2): one
 * hypothesis per seed, no branching.
 *  1. initialise from the start hit and its upward link;
 *  2. update with every hit of the seed chain (upward links), no gate;
 *  3. follow outward row by row to the last row: extrapolate, take the
 *     closest gated cluster, update; stop after more than max_miss
 *     consecutive rows without a cluster, or when transport fails;
 *  4. from the state at the outermost update, transport back row by row to
 *     the start row (no updates), then follow inward below the start row the
 *     same way;
 *  5. the result is the state right after the innermost update (at the start
 *     row if none), i.e. at x_ref = x of the first row with a hit.
 * Output per tracklet: x_ref, parameters, covariance, hit per row (-1 none),
 * start/first/last row, hit count, flags.  counters (may be NULL):
 * [0] transports, [1] updates, [2] gated candidates, [3] row searches.
 */
int32_t SFX(oracle_tracklets)(int32_t n_rows, const float* row_x, int32_t n, const float* y,
                              const float* z, const int32_t* row, const int32_t* up_clean,
                              int32_t n_start, const int32_t* start, const oracle_params* p,
                              real* x_ref, real* param, real* cov, int32_t* row_hit,
                              int32_t* start_row, int32_t* first_row, int32_t* last_row,
                              int32_t* n_hits, int32_t* flags, int64_t* counters) {
  const consts c = make_consts(p);
  int32_t* first = row_ranges(n_rows, n, row);
  if (!first) return -1;
  int64_t dummy[4] = {0, 0, 0, 0};
  int64_t* cnt = counters ? counters : dummy;
  for (int32_t it = 0; it < n_start; ++it) {
    int32_t* rh = row_hit + (int64_t)it * n_rows;
    for (int32_t r = 0; r < n_rows; ++r) rh[r] = -1;
    const int32_t h0 = start[it];
    const int32_t r0 = row[h0];
    const int32_t h1 = up_clean[h0];
    int32_t fl = 0;
    rh[r0] = h0;
    start_row[it] = r0;
    track st, last, snap;
    const int ei = init_track(&st, (real)row_x[r0], (real)y[h0], (real)z[h0], (real)row_x[row[h1]],
                              (real)y[h1], (real)z[h1], &c);
    if (ei != STEP_OK) {
      fl |= stop_flag(ei);
      snap = st;
    } else {
      last = st;
      int32_t lastr = r0;
      int stopped = 0;
      /* 2. seed chain */
      for (int32_t h = h1; h >= 0; h = up_clean[h]) {
        const int32_t r = row[h];
        cnt[0]++;
        const int e = propagate(&st, (real)row_x[r], &c);
        if (e) { fl |= stop_flag(e); stopped = 1; break; }
        track u = st;
        cnt[1]++;
        if (update(&u, (real)y[h], (real)z[h], &c)) { fl |= ORACLE_STOP_SINPHI; stopped = 1; break; }
        st = u; rh[r] = h; last = st; lastr = r;
      }
      /* 3. outward following */
      if (!stopped) {
        int miss = 0;
        for (int32_t r = lastr + 1; r < n_rows; ++r) {
          cnt[0]++;
          const int e = propagate(&st, (real)row_x[r], &c);
          if (e) { fl |= stop_flag(e); break; }
          const int32_t j = closest(&st, first[r], first[r + 1], y, z, &c, cnt);
          if (j >= 0) {
            track u = st;
            cnt[1]++;
            if (update(&u, (real)y[j], (real)z[j], &c)) { fl |= ORACLE_STOP_SINPHI; break; }
            st = u; rh[r] = j; last = st; lastr = r; miss = 0;
          } else if (++miss > c.max_miss) {
            break;
          }
        }
      }
      /* 4. back to the start row, then inward following */
      st = last;
      int ok = 1;
      for (int32_t r = lastr - 1; r >= r0; --r) {
        cnt[0]++;
        const int e = propagate(&st, (real)row_x[r], &c);
        if (e) { fl |= stop_flag(e); ok = 0; break; }
      }
      snap = ok ? st : last;
      if (ok) {
        int miss = 0;
        for (int32_t r = r0 - 1; r >= 0; --r) {
          cnt[0]++;
          const int e = propagate(&st, (real)row_x[r], &c);
          if (e) { fl |= stop_flag(e); break; }
          const int32_t j = closest(&st, first[r], first[r + 1], y, z, &c, cnt);
          if (j >= 0) {
            track u = st;
            cnt[1]++;
            if (update(&u, (real)y[j], (real)z[j], &c)) { fl |= ORACLE_STOP_SINPHI; break; }
            st = u; rh[r] = j; snap = st; miss = 0;
          } else if (++miss > c.max_miss) {
            break;
          }
        }
      }
    }
    /* 5. output */
    store(&snap, it, x_ref, param, cov);
    int32_t nh = 0, fr = -1, lr = -1;
    for (int32_t r = 0; r < n_rows; ++r)
      if (rh[r] >= 0) { nh++; if (fr < 0) fr = r; lr = r; }
    n_hits[it] = nh; first_row[it] = fr; last_row[it] = lr;
    if (nh >= c.min_hits) fl |= ORACLE_VALID;
    if (!spd_ok(&snap)) fl |= ORACLE_SPD_FAIL;
#ifdef ORACLE_F32
    if ((p->precision == 1 && (fl & ORACLE_SPD_FAIL)) || p->precision == 2) {
      int32_t spd64 = 0;
      float xr;
      oracle_refit_mixed(n_rows, row_x, n, y, z, 1, rh, &start_row[it], p, &xr,
                         (float*)param + 5 * (int64_t)it, (float*)cov + 15 * (int64_t)it, &spd64);
      x_ref[it] = xr;
      fl |= ORACLE_REFIT64;
    }
#endif
    flags[it] = fl;
  }
  free(first);
  return 0;
}

/*
 * Refit on a recorded hit list (one list of hit-per-row per tracklet), same
 * pass structure as the constructor without any search: initialise from the
 * hits of the start row r0 and row r0+1, update at every row above r0 that
 * has a hit (transporting through every row in between), transport back to
 * r0 from the outermost hit, then update at every row below r0 that has a
 * hit, down to the innermost one.  In the f64 build this is the reference for
 * the binary32 parameters; in the f32 build it reproduces the constructor's
 * state exactly.  flags: bit 0 set when the refit ran to the innermost hit;
 * stop bits as in the constructor.  A tracklet without a hit at r0+1 is not
 * refittable (flags = 0).
 */
int32_t SFX(oracle_refit)(int32_t n_rows, const float* row_x, int32_t n, const float* y,
                          const float* z, int32_t n_trk, const int32_t* row_hit,
                          const int32_t* start_row, const oracle_params* p, real* x_ref,
                          real* param, real* cov, int32_t* flags) {
  (void)n;
  const consts c = make_consts(p);
  for (int32_t it = 0; it < n_trk; ++it) {
    const int32_t* rh = row_hit + (int64_t)it * n_rows;
    const int32_t r0 = start_row[it];
    track st, last, snap;
    memset(&st, 0, sizeof st);
    flags[it] = 0;
    if (r0 < 0 || r0 + 1 >= n_rows || rh[r0] < 0 || rh[r0 + 1] < 0) { store(&st, it, x_ref, param, cov); continue; }
    const int32_t h0 = rh[r0], h1 = rh[r0 + 1];
    int fl = 0;
    int e = init_track(&st, (real)row_x[r0], (real)y[h0], (real)z[h0], (real)row_x[r0 + 1], (real)y[h1], (real)z[h1], &c);
    if (e) { store(&st, it, x_ref, param, cov); flags[it] = stop_flag(e); continue; }
    int32_t lastr = r0;
    for (int32_t r = r0 + 1; r < n_rows; ++r) if (rh[r] >= 0) lastr = r;
    int32_t fr = r0;
    for (int32_t r = r0 - 1; r >= 0; --r) if (rh[r] >= 0) fr = r;
    last = st;
    int complete = 1;
    int32_t lr = r0; /* row of the last update */
    for (int32_t r = r0 + 1; r <= lastr; ++r) {
      e = propagate(&st, (real)row_x[r], &c);
      if (e) { fl |= stop_flag(e); complete = 0; break; }
      if (rh[r] >= 0) {
        track u = st;
        if (update(&u, (real)y[rh[r]], (real)z[rh[r]], &c)) { fl |= ORACLE_STOP_SINPHI; complete = 0; break; }
        st = u; last = st; lr = r;
      }
    }
    st = last;
    int ok = 1;
    for (int32_t r = lr - 1; r >= r0; --r) {
      e = propagate(&st, (real)row_x[r], &c);
      if (e) { fl |= stop_flag(e); ok = 0; complete = 0; break; }
    }
    snap = ok ? st : last;
    if (ok) {
      for (int32_t r = r0 - 1; r >= fr; --r) {
        e = propagate(&st, (real)row_x[r], &c);
        if (e) { fl |= stop_flag(e); complete = 0; break; }
        if (rh[r] >= 0) {
          track u = st;
          if (update(&u, (real)y[rh[r]], (real)z[rh[r]], &c)) { fl |= ORACLE_STOP_SINPHI; complete = 0; break; }
          st = u; snap = st;
        }
      }
    }
    store(&snap, it, x_ref, param, cov);
    flags[it] = fl | (complete ? 1 : 0);
  }
  return 0;
}

/* ------------------------------------------- unit entry points (tests) */
static void from_vec(track* t, const real* v) {
  t->x = v[0]; t->y = v[1]; t->z = v[2]; t->s = v[3]; t->l = v[4]; t->q = v[5];
  t->c00 = v[6]; t->c10 = v[7]; t->c11 = v[8]; t->c20 = v[9]; t->c21 = v[10]; t->c22 = v[11];
  t->d00 = v[12]; t->d10 = v[13]; t->d11 = v[14];
}
static void to_vec(const track* t, real* v) {
  v[0] = t->x; v[1] = t->y; v[2] = t->z; v[3] = t->s; v[4] = t->l; v[5] = t->q;
  v[6] = t->c00; v[7] = t->c10; v[8] = t->c11; v[9] = t->c20; v[10] = t->c21; v[11] = t->c22;
  v[12] = t->d00; v[13] = t->d10; v[14] = t->d11;
}

/* h0, h1: (x, y, z) of the start hit and its upward neighbour */
int32_t SFX(oracle_init)(const real* h0, const real* h1, const oracle_params* p, real* st) {
  const consts c = make_consts(p);
  track t;
  const int e = init_track(&t, h0[0], h0[1], h0[2], h1[0], h1[1], h1[2], &c);
  to_vec(&t, st);
  return e;
}

int32_t SFX(oracle_propagate)(real* st, real x1, const oracle_params* p) {
  const consts c = make_consts(p);
  track t;
  from_vec(&t, st);
  const int e = propagate(&t, x1, &c);
  if (e == STEP_OK) to_vec(&t, st);
  return e;
}

int32_t SFX(oracle_update)(real* st, real my, real mz, const oracle_params* p) {
  const consts c = make_consts(p);
  track t;
  from_vec(&t, st);
  const int e = update(&t, my, mz, &c);
  if (e == STEP_OK) to_vec(&t, st);
  return e;
}

int32_t SFX(oracle_spd)(const real* st) {
  track t;
  from_vec(&t, st);
  return spd_ok(&t);
}
