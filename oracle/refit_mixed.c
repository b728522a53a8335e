/*
 * CPU oracle: precision-form refit.  Test infrastructure only; see oracle.h.
 *
 * Sec. 2 item 2 fixes only that the filter is a simplified Kalman filter; its
 * precision is not given.  Reading used for the precision form: a tracklet
 * whose binary32 covariance fails the positive-definiteness check is refit on
 * its recorded hit list (same initialisation, same hit order, same passes as
 * the binary64 refit, no new search) with the state kept in binary32 and the
 * covariance, gain and covariance transport in binary64.  The binary32
 * quantities are formed exactly as in the binary32 filter; a binary64 gain
 * times a binary32 residual is rounded to binary32 before it is added to the
 * binary32 state.
 */
#include <float.h>
#include <math.h>
#include <string.h>

#include "oracle.h"

typedef struct {
  float x, y, z, s, l, q;
  double c00, c10, c11, c20, c21, c22;
  double d00, d10, d11;
} mtrack;

static int prop_m(mtrack* t, float x1, float kb) {
  const float dx = x1 - t->x;
  const float k = kb * t->q;
  const float s0 = t->s;
  const float s1 = s0 + k * dx;
  if (!(fabsf(s1) < 0.999f)) return 1;
  const float c0 = sqrtf(1.0f - s0 * s0);
  const float c1 = sqrtf(1.0f - s1 * s1);
  const float T = (s0 + s1) / (c0 + c1);
  const float dy = dx * T;
  const float ch = sqrtf(dx * dx + dy * dy);
  const float u = (k * ch) * 0.5f;
  if (!(fabsf(u) <= 0.2f)) return 2;
  const float u2 = u * u;
  const float A = 1.0f + u2 * (1.0f / 6.0f + u2 * (3.0f / 40.0f + u2 * (5.0f / 112.0f + u2 * (35.0f / 1152.0f))));
  float dS = ch * A;
  if (dx < 0) dS = -dS;
  const float sm = (s0 + s1) * 0.5f;
  const float cm2 = 1.0f - sm * sm;
  const float cm3 = cm2 * sqrtf(cm2);
  const double a = (double)(dx / cm3);
  const double b = (double)(((kb * dx) * dx * 0.5f) / cm3);
  const double d = (double)(kb * dx);
  const double e = (double)dS;
  t->x = x1;
  t->y = t->y + dy;
  t->z = t->z + t->l * dS;
  t->s = s1;
  const double c00 = t->c00, c10 = t->c10, c11 = t->c11, c20 = t->c20, c21 = t->c21, c22 = t->c22;
  const double m0 = c00 + a * c10 + b * c20;
  const double m1 = c10 + a * c11 + b * c21;
  const double m2 = c20 + a * c21 + b * c22;
  const double n1 = c11 + d * c21;
  const double n2 = c21 + d * c22;
  t->c00 = m0 + a * m1 + b * m2;
  t->c10 = m1 + d * m2;
  t->c11 = n1 + d * n2;
  t->c20 = m2;
  t->c21 = n2;
  const double tz = t->d10 + e * t->d11;
  t->d00 = t->d00 + e * t->d10 + e * tz;
  t->d10 = tz;
  return 0;
}

static int upd_m(mtrack* t, float my, float mz, double sy2, double sz2) {
  const float ry = my - t->y;
  const double iy = 1.0 / (t->c00 + sy2);
  const double k0 = t->c00 * iy, k1 = t->c10 * iy, k2 = t->c20 * iy;
  t->y = t->y + (float)(k0 * (double)ry);
  t->s = t->s + (float)(k1 * (double)ry);
  t->q = t->q + (float)(k2 * (double)ry);
  const double c00 = t->c00, c10 = t->c10, c20 = t->c20;
  t->c00 = c00 - k0 * c00;
  t->c10 = c10 - k1 * c00;
  t->c20 = c20 - k2 * c00;
  t->c11 = t->c11 - k1 * c10;
  t->c21 = t->c21 - k2 * c10;
  t->c22 = t->c22 - k2 * c20;
  const float rz = mz - t->z;
  const double iz = 1.0 / (t->d00 + sz2);
  const double g0 = t->d00 * iz, g1 = t->d10 * iz;
  t->z = t->z + (float)(g0 * (double)rz);
  t->l = t->l + (float)(g1 * (double)rz);
  const double d00 = t->d00, d10 = t->d10;
  t->d00 = d00 - g0 * d00;
  t->d10 = d10 - g1 * d00;
  t->d11 = t->d11 - g1 * d10;
  return fabsf(t->s) < 0.999f ? 0 : 1;
}

static int spd_m(const mtrack* t) {
  const double p0 = t->c00;
  if (!(p0 > 0 && p0 <= DBL_MAX)) return 0;
  const double a = t->c10 / p0;
  const double p1 = t->c11 - a * t->c10;
  if (!(p1 > 0 && p1 <= DBL_MAX)) return 0;
  const double b = t->c20 / p0;
  const double e = t->c21 - b * t->c10;
  const double p2 = (t->c22 - b * t->c20) - (e / p1) * e;
  if (!(p2 > 0 && p2 <= DBL_MAX)) return 0;
  const double q1 = t->d11 - (t->d10 / t->d00) * t->d10;
  return t->d00 > 0 && q1 > 0 && q1 <= DBL_MAX;
}

int32_t oracle_refit_mixed(int32_t n_rows, const float* row_x, int32_t n, const float* y,
                           const float* z, int32_t n_trk, const int32_t* row_hit,
                           const int32_t* start_row, const oracle_params* p, float* x_ref,
                           float* param, float* cov, int32_t* spd_ok) {
  (void)n;
  const float kb = -0.00299792458f * p->bz;
  const double sy2 = (double)p->sigma_y * (double)p->sigma_y;
  const double sz2 = (double)p->sigma_z * (double)p->sigma_z;
  for (int32_t it = 0; it < n_trk; ++it) {
    const int32_t* rh = row_hit + (int64_t)it * n_rows;
    const int32_t r0 = start_row[it];
    mtrack st, last, snap;
    memset(&st, 0, sizeof st);
    int ok = r0 >= 0 && r0 + 1 < n_rows && rh[r0] >= 0 && rh[r0 + 1] >= 0;
    if (ok) {
      const int32_t h0 = rh[r0], h1 = rh[r0 + 1];
      const float x0 = row_x[r0], x1 = row_x[r0 + 1];
      const float dx = x1 - x0, dy = y[h1] - y[h0], dz = z[h1] - z[h0];
      const float L = sqrtf(dx * dx + dy * dy);
      st.x = x0; st.y = y[h0]; st.z = z[h0]; st.s = dy / L; st.l = dz / L; st.q = 0.0f;
      st.c00 = sy2; st.c11 = 1.0; st.c22 = 100.0;
      st.d00 = sz2; st.d11 = 1.0;
      ok = fabsf(st.s) < 0.999f;
    }
    snap = st;
    if (ok) {
      int32_t lastr = r0, fr = r0;
      for (int32_t r = r0 + 1; r < n_rows; ++r) if (rh[r] >= 0) lastr = r;
      for (int32_t r = r0 - 1; r >= 0; --r) if (rh[r] >= 0) fr = r;
      last = st;
      int32_t lr = r0; /* row of the last update */
      for (int32_t r = r0 + 1; r <= lastr; ++r) {
        if (prop_m(&st, row_x[r], kb)) break;
        if (rh[r] >= 0) {
          mtrack u = st;
          if (upd_m(&u, y[rh[r]], z[rh[r]], sy2, sz2)) break;
          st = u; last = st; lr = r;
        }
      }
      st = last;
      int back = 1;
      for (int32_t r = lr - 1; r >= r0; --r)
        if (prop_m(&st, row_x[r], kb)) { back = 0; break; }
      snap = back ? st : last;
      if (back) {
        for (int32_t r = r0 - 1; r >= fr; --r) {
          if (prop_m(&st, row_x[r], kb)) break;
          if (rh[r] >= 0) {
            mtrack u = st;
            if (upd_m(&u, y[rh[r]], z[rh[r]], sy2, sz2)) break;
            st = u; snap = st;
          }
        }
      }
    }
    x_ref[it] = snap.x;
    float* pp = param + 5 * (int64_t)it;
    pp[0] = snap.y; pp[1] = snap.z; pp[2] = snap.s; pp[3] = snap.l; pp[4] = snap.q;
    float* cc = cov + 15 * (int64_t)it;
    for (int k = 0; k < 15; ++k) cc[k] = 0.0f;
    cc[0] = (float)snap.c00; cc[2] = (float)snap.d00; cc[3] = (float)snap.c10; cc[5] = (float)snap.c11;
    cc[7] = (float)snap.d10; cc[9] = (float)snap.d11; cc[10] = (float)snap.c20; cc[12] = (float)snap.c21;
    cc[14] = (float)snap.c22;
    if (spd_ok) spd_ok[it] = spd_m(&snap);
  }
  return 0;
}
