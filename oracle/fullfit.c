/*
 * CPU oracle: full Kalman refit of a selected track segment (test
 * infrastructure only; see oracle.h).
 *
 * Sec. 2 item 4: in the end the tracks are refitted with the full Kalman
 * filter (the tracklet construction of item 2 uses a simplified one with
 * uncorrelated coordinate errors).  Reading used here (constant field: the
 * paper's polynomial field approximation is not given):
 *  - state (y, z, sin phi, tan lambda, q/pT) at x, full 5x5 covariance;
 *  - start: the tracklet's parameters at its x_ref, carried row by row (state
 *    only) to the track's innermost hit, covariance
 *    diag(sigma_y^2, sigma_z^2, 1, 1, 100) there;
 *  - row by row outward to the outermost hit: the same helix transport of the
 *    state as the tracklet filter, covariance C <- F C F^T with the Jacobian
 *    F = 1 + dy/dsin(phi), dy/d(q/pT), dsin(phi)/d(q/pT), dz/dtan(lambda) as
 *    in the tracklet filter plus the coupling terms dz/dsin(phi) and
 *    dz/d(q/pT) (first order in the step, at the mean angle);
 *  - at each hit a Kalman update with the 2-d measurement (y, z), 2x2
 *    innovation covariance; chi^2 accumulated; an update that would take
 *    |sin phi| to 0.999 or beyond is rejected and ends the fit;
 *  - result at the outermost hit.
 * Matrix products are written as plain loops (indices ascending), the same
 * order in both builds.
 */
#include <float.h>
#include <math.h>

#include "oracle.h"

#ifdef ORACLE_F32
typedef float real;
#define SFX(name) name##_f32
#define RSQRT(v) sqrtf(v)
#define RABS(v) fabsf(v)
#define LIT(v) v##f
#else
typedef double real;
#define SFX(name) name##_f64
#define RSQRT(v) sqrt(v)
#define RABS(v) fabs(v)
#define LIT(v) v
#endif

/* packed lower triangle index of (i, j), i >= j */
static int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

/* Helix transport of the state to x1 (the tracklet filter's formulas); fills
 * the Jacobian F when F != 0.  Returns 0, 2 (|sin phi| limit) or 4 (arc
 * length series limit). */
static int transport(real* x, real* p, real x1, real kb, real F[5][5]) {
  const real dx = x1 - *x;
  const real k = kb * p[4];
  const real s0 = p[2];
  const real s1 = s0 + k * dx;
  if (!(RABS(s1) < LIT(0.999))) return 2;
  const real c0 = RSQRT(LIT(1.0) - s0 * s0);
  const real c1 = RSQRT(LIT(1.0) - s1 * s1);
  const real T = (s0 + s1) / (c0 + c1);
  const real dy = dx * T;
  const real ch = RSQRT(dx * dx + dy * dy);
  const real u = (k * ch) * LIT(0.5);
  if (!(RABS(u) <= LIT(0.2))) return 4;
  const real u2 = u * u;
  const real A = LIT(1.0) + u2 * (LIT(1.0) / LIT(6.0) + u2 * (LIT(3.0) / LIT(40.0) +
                 u2 * (LIT(5.0) / LIT(112.0) + u2 * (LIT(35.0) / LIT(1152.0)))));
  real dS = ch * A;
  if (dx < LIT(0.0)) dS = -dS;
  if (F) {
    const real sm = (s0 + s1) * LIT(0.5);
    const real cm2 = LIT(1.0) - sm * sm;
    const real cm3 = cm2 * RSQRT(cm2);
    const real a = dx / cm3;                         /* dy / d sin(phi) */
    const real b = ((kb * dx) * dx * LIT(0.5)) / cm3; /* dy / d(q/pT) */
    const real d = kb * dx;                          /* d sin(phi) / d(q/pT) */
    const real e = ((p[3] * dx) * sm) / cm3;         /* dz / d sin(phi) */
    const real f = (e * d) * LIT(0.5);               /* dz / d(q/pT) */
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) F[i][j] = i == j ? LIT(1.0) : LIT(0.0);
    F[0][2] = a;
    F[0][4] = b;
    F[1][2] = e;
    F[1][3] = dS;
    F[1][4] = f;
    F[2][4] = d;
  }
  *x = x1;
  p[0] = p[0] + dy;
  p[1] = p[1] + p[3] * dS;
  p[2] = s1;
  return 0;
}

/* structurally nonzero entries of F: the identity and a, b, e, dS, f, d */
static int nz(int i, int j) { return i == j || (i == 0 && (j == 2 || j == 4)) || (i == 1 && j >= 2) || (i == 2 && j == 4); }

/* C <- F C F^T on the packed lower triangle; each sum runs over k ascending
 * and leaves out the terms where F is zero by construction */
static void transport_cov(real* C, real F[5][5]) {
  real M[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      real acc = LIT(0.0);
      for (int k = 0; k < 5; ++k)
        if (nz(i, k)) acc = acc + F[i][k] * C[tri(k, j)];
      M[i][j] = acc;
    }
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j) {
      real acc = LIT(0.0);
      for (int k = 0; k < 5; ++k)
        if (nz(j, k)) acc = acc + M[i][k] * F[j][k];
      C[tri(i, j)] = acc;
    }
}

/* Kalman update with (my, mz); returns 0, 2 (rejected: |sin phi| limit) or 8
 * (innovation covariance not positive). */
static int update2(real* p, real* C, real my, real mz, real sy2, real sz2, real* chi2) {
  const real r0 = my - p[0];
  const real r1 = mz - p[1];
  const real S00 = C[tri(0, 0)] + sy2;
  const real S01 = C[tri(1, 0)];
  const real S11 = C[tri(1, 1)] + sz2;
  const real det = S00 * S11 - S01 * S01;
  if (!(det > LIT(0.0))) return 8;
  const real i00 = S11 / det;
  const real i01 = (LIT(0.0) - S01) / det;
  const real i11 = S00 / det;
  real K[5][2];
  for (int i = 0; i < 5; ++i) {
    K[i][0] = C[tri(i, 0)] * i00 + C[tri(i, 1)] * i01;
    K[i][1] = C[tri(i, 0)] * i01 + C[tri(i, 1)] * i11;
  }
  const real s_new = p[2] + (K[2][0] * r0 + K[2][1] * r1);
  if (!(RABS(s_new) < LIT(0.999))) return 2;
  for (int i = 0; i < 5; ++i) p[i] = p[i] + (K[i][0] * r0 + K[i][1] * r1);
  real Cn[15];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j) Cn[tri(i, j)] = C[tri(i, j)] - (K[i][0] * C[tri(0, j)] + K[i][1] * C[tri(1, j)]);
  for (int q = 0; q < 15; ++q) C[q] = Cn[q];
  *chi2 = *chi2 + (r0 * (i00 * r0 + i01 * r1) + r1 * (i01 * r0 + i11 * r1));
  return 0;
}

int32_t SFX(oracle_fullfit)(int32_t n_rows, const float* row_x, int32_t n, const int32_t* rows, const float* hy,
                            const float* hz, real x_start, const real* p_start, int32_t start_row,
                            const oracle_params* prm, real* x_out, real* p_out, real* C_out, real* chi2_out,
                            int32_t* ndf_out, int32_t* flags_out) {
  const real kb = LIT(-0.00299792458) * (real)prm->bz;
  const real sy2 = (real)prm->sigma_y * (real)prm->sigma_y;
  const real sz2 = (real)prm->sigma_z * (real)prm->sigma_z;
  real x = x_start, p[5], C[15];
  for (int i = 0; i < 5; ++i) p[i] = p_start[i];
  for (int q = 0; q < 15; ++q) C[q] = LIT(0.0);
  real chi2 = LIT(0.0);
  int fl = 0, used = 0;
  if (n <= 0 || rows[0] < start_row || rows[n - 1] >= n_rows) {
    fl = 64;
  } else {
    /* the start state, carried to the innermost hit (state only) */
    for (int r = start_row + 1; r <= rows[0] && !fl; ++r) fl = transport(&x, p, (real)row_x[r], kb, 0);
    if (!fl) {
      C[tri(0, 0)] = sy2;
      C[tri(1, 1)] = sz2;
      C[tri(2, 2)] = LIT(1.0);
      C[tri(3, 3)] = LIT(1.0);
      C[tri(4, 4)] = LIT(100.0);
      real F[5][5];
      int k = 0;
      for (int r = rows[0]; r <= rows[n - 1] && !fl; ++r) {
        if (r > rows[0]) {
          fl = transport(&x, p, (real)row_x[r], kb, F);
          if (fl) break;
          transport_cov(C, F);
        }
        if (k < n && rows[k] == r) {
          fl = update2(p, C, (real)hy[k], (real)hz[k], sy2, sz2, &chi2);
          if (fl) break;
          ++k;
          ++used;
        }
      }
      if (!fl) fl = 1;
    }
  }
  *x_out = x;
  for (int i = 0; i < 5; ++i) p_out[i] = p[i];
  for (int q = 0; q < 15; ++q) C_out[q] = C[q];
  *chi2_out = chi2;
  *ndf_out = 2 * used - 5;
  *flags_out = fl;
  return 0;
}

/* One transport step of state and covariance (unit entry point for tests). */
int32_t SFX(oracle_fullfit_transport)(real* x, real* p, real* C, real x1, const oracle_params* prm) {
  const real kb = LIT(-0.00299792458) * (real)prm->bz;
  real F[5][5];
  const int rc = transport(x, p, x1, kb, F);
  if (!rc) transport_cov(C, F);
  return rc;
}
