/*
 * Seeded synthetic TPC events: primary helices from the origin in a constant
 * solenoid field, intersected with the pad-row planes of the 36 trapezoidal
 * sectors (2 sides x 18, Sec. 2), smeared, plus uniform noise hits.
 *
 * This module is the detector simulation only.  It holds none of the tracking
 * method's arithmetic: the helix is evaluated in closed form in the global
 * frame (sin/cos/asin in double), not by the row-by-row propagation the
 * tracker uses, so it can serve as an independent check of that propagation.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), keyed by (seed, event) with one counter
 * stream per purpose, so every hit is reproducible on its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYNTH_PI 3.14159265358979323846

/* ---------------------------------------------------------------- Philox */
typedef struct { uint32_t v[4]; } u32x4;

static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0];
  const uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

/* Philox4x32 with 10 rounds; the key is bumped by the Weyl constants between
 * rounds. */
void synth_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
    philox_round(c, k);
  }
  memcpy(out, c, sizeof c);
}

enum { ST_TRACK = 1, ST_SMEAR = 2, ST_NOISE = 3, ST_PERM = 4, ST_MULT = 5, ST_TRACK2 = 6 };

static u32x4 draw(uint64_t seed, uint32_t event, uint32_t a, uint32_t b, uint32_t c, uint32_t stream) {
  const uint32_t key[2] = {(uint32_t)seed, event};
  const uint32_t ctr[4] = {a, b, c, stream};
  u32x4 o;
  synth_philox4x32_10(ctr, key, o.v);
  return o;
}

/* uniform on the open interval (0, 1) */
static double unif(uint32_t r) { return ((double)r + 0.5) * (1.0 / 4294967296.0); }

/* ------------------------------------------------------------- geometry */
/* Pad-row positions: 159 rows evenly spaced from 85 to 247 cm, computed in
 * double and rounded to float; hits lie exactly on these float planes. */
void synth_row_x(int32_t n_rows, double x_first, double x_last, float* out) {
  for (int r = 0; r < n_rows; ++r)
    out[r] = (float)(x_first + (double)r * (x_last - x_first) / (double)(n_rows - 1));
}

/* Sector rotation: sector s in [0,36), side A for s < 18, C otherwise;
 * alpha = ((s mod 18) + 0.5) * 20 degrees. */
double synth_sector_alpha(int32_t s) { return ((double)(s % 18) + 0.5) * (20.0 * SYNTH_PI / 180.0); }

typedef struct {
  int32_t n_rows;
  double x_first, x_last;  /* cm */
  double bz;               /* T */
  double sigma;            /* cm, Gaussian smear of y and z */
  double noise_frac;       /* noise hits per signal hit, per sector */
  double tan_half_open;    /* tan(10 deg) */
  double z_max;            /* cm */
  double pt_min, pt_max;   /* GeV, log-uniform */
  double eta_min, eta_max; /* uniform */
  double phi_min, phi_max; /* rad, uniform */
  int32_t sector_first, sector_count; /* sectors read out */
  uint64_t seed;
  int32_t dead_first, dead_count;     /* pad rows [first, first + count) read out nothing */
} synth_cfg;

typedef struct {
  int32_t n_sectors;       /* = sector_count */
  int64_t n_hits;
  int64_t* hit_offset;     /* [n_sectors+1] */
  float *x, *y, *z;        /* [n_hits] */
  int32_t *row, *label;    /* label: track id or -1 for noise */
  double *y_true, *z_true, *sinphi_true; /* [n_hits] when truth requested */
  int32_t n_tracks;
  double *trk_q, *trk_pt, *trk_eta, *trk_phi0; /* [n_tracks] */
} synth_event;

typedef struct {
  float y, z; int32_t row, label; uint32_t key; int32_t serial;
  double yt, zt, st;
} hitrec;

static int hitrec_cmp(const void* a, const void* b) {
  const hitrec* p = (const hitrec*)a; const hitrec* q = (const hitrec*)b;
  if (p->row != q->row) return p->row < q->row ? -1 : 1;
  if (p->key != q->key) return p->key < q->key ? -1 : 1;
  return (p->serial > q->serial) - (p->serial < q->serial);
}

typedef struct { hitrec* h; int64_t n, cap; } hitvec;
static void push(hitvec* v, hitrec r) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 1024;
    v->h = (hitrec*)realloc(v->h, (size_t)v->cap * sizeof(hitrec));
  }
  v->h[v->n++] = r;
}

static double wrap_pi(double a) { /* to [-pi, pi) */
  a = fmod(a + SYNTH_PI, 2.0 * SYNTH_PI);
  if (a < 0) a += 2.0 * SYNTH_PI;
  return a - SYNTH_PI;
}

/* Generate one event with n_tracks primary tracks. Returns NULL on allocation
 * failure.  Free with synth_free. */
synth_event* synth_generate_tracks(const synth_cfg* cfg, int32_t n_tracks, const double* tq, const double* tpt,
                                   const double* teta, const double* tphi0, uint32_t event_id, int32_t want_truth);

synth_event* synth_generate(const synth_cfg* cfg, int32_t n_tracks, uint32_t event_id, int32_t want_truth) {
  const size_t m = (size_t)(n_tracks > 0 ? n_tracks : 1);
  double* q = (double*)malloc(sizeof(double) * m);
  double* pt = (double*)malloc(sizeof(double) * m);
  double* eta = (double*)malloc(sizeof(double) * m);
  double* phi0 = (double*)malloc(sizeof(double) * m);
  for (int32_t t = 0; t < n_tracks; ++t) {
    const u32x4 a = draw(cfg->seed, event_id, (uint32_t)t, 0, 0, ST_TRACK);
    q[t] = unif(a.v[0]) < 0.5 ? -1.0 : 1.0;
    pt[t] = exp(log(cfg->pt_min) + unif(a.v[1]) * (log(cfg->pt_max) - log(cfg->pt_min)));
    eta[t] = cfg->eta_min + unif(a.v[2]) * (cfg->eta_max - cfg->eta_min);
    phi0[t] = cfg->phi_min + unif(a.v[3]) * (cfg->phi_max - cfg->phi_min);
  }
  synth_event* ev = synth_generate_tracks(cfg, n_tracks, q, pt, eta, phi0, event_id, want_truth);
  free(q); free(pt); free(eta); free(phi0);
  return ev;
}

/* Same as synth_generate with an explicit track table (charge sign, pT in
 * GeV, eta, phi0 in rad). */
synth_event* synth_generate_tracks(const synth_cfg* cfg, int32_t n_tracks, const double* tq, const double* tpt,
                                   const double* teta, const double* tphi0, uint32_t event_id, int32_t want_truth) {
  const int nr = cfg->n_rows;
  float* rx = (float*)malloc(sizeof(float) * (size_t)nr);
  synth_row_x(nr, cfg->x_first, cfg->x_last, rx);
  const int ns = cfg->sector_count;
  hitvec* sec = (hitvec*)calloc((size_t)ns, sizeof(hitvec));
  int64_t* n_signal = (int64_t*)calloc((size_t)ns, sizeof(int64_t));
  synth_event* ev = (synth_event*)calloc(1, sizeof(synth_event));
  ev->n_tracks = n_tracks;
  ev->trk_q = (double*)malloc(sizeof(double) * (size_t)(n_tracks > 0 ? n_tracks : 1));
  ev->trk_pt = (double*)malloc(sizeof(double) * (size_t)(n_tracks > 0 ? n_tracks : 1));
  ev->trk_eta = (double*)malloc(sizeof(double) * (size_t)(n_tracks > 0 ? n_tracks : 1));
  ev->trk_phi0 = (double*)malloc(sizeof(double) * (size_t)(n_tracks > 0 ? n_tracks : 1));
  const double cB = 0.00299792458; /* GeV / (T cm) */
  const double rho_lo = cfg->x_first, rho_hi = cfg->x_last * sqrt(1.0 + cfg->tan_half_open * cfg->tan_half_open);
  const double half_open = atan(cfg->tan_half_open);

  for (int32_t t = 0; t < n_tracks; ++t) {
    const double q = tq[t], pt = tpt[t], eta = teta[t], phi0 = tphi0[t];
    ev->trk_q[t] = q; ev->trk_pt[t] = pt; ev->trk_eta[t] = eta; ev->trk_phi0[t] = phi0;
    const double tanl = sinh(eta);
    /* signed curvature d(phi)/ds, s = transverse path length from the origin */
    const double k = -cB * cfg->bz * q / pt;
    const int sideA = tanl >= 0.0;
    /* azimuth of the position at radius rho: phi0 + asin(rho k / 2) */
    double th_lo, th_hi;
    {
      double v1 = rho_lo * k * 0.5, v2 = rho_hi * k * 0.5;
      if (v1 > 1) v1 = 1; if (v1 < -1) v1 = -1;
      if (v2 > 1) v2 = 1; if (v2 < -1) v2 = -1;
      const double t1 = phi0 + asin(v1), t2 = phi0 + asin(v2);
      th_lo = t1 < t2 ? t1 : t2; th_hi = t1 < t2 ? t2 : t1;
    }
    for (int si = 0; si < ns; ++si) {
      const int s = cfg->sector_first + si;
      if ((s < 18) != sideA) continue;
      const double al = synth_sector_alpha(s);
      /* does [th_lo, th_hi] overlap [al - half_open, al + half_open] (mod 2pi)? */
      const double mid = 0.5 * (th_lo + th_hi), hw = 0.5 * (th_hi - th_lo);
      if (fabs(wrap_pi(mid - al)) > hw + half_open + 0.02) continue;
      const double psi0 = phi0 - al; /* sector-local initial direction */
      const double sp0 = sin(psi0), cp0 = cos(psi0);
      for (int r = 0; r < nr; ++r) {
        const double xr = (double)rx[r];
        double path, yl, sphi;
        if (fabs(k) < 1e-14) {
          if (cp0 <= 0.0) continue;
          path = xr / cp0; yl = path * sp0; sphi = sp0;
        } else {
          const double w = sp0 + k * xr; /* sin(psi) at the crossing */
          if (!(fabs(w) < 1.0)) continue;
          const double psi = asin(w);  /* outward branch: cos(psi) > 0 */
          double d = wrap_pi(psi - psi0);
          /* smallest positive path: d/k > 0 */
          if (k > 0 && d < 0) d += 2.0 * SYNTH_PI;
          if (k < 0 && d > 0) d -= 2.0 * SYNTH_PI;
          if (fabs(d) > SYNTH_PI) continue; /* past the apex: the track has left the TPC */
          path = d / k;
          yl = (cp0 - cos(psi)) / k;
          sphi = w;
        }
        if (!(path > 0.0)) continue;
        const double zl = tanl * path;
        if (fabs(yl) > xr * cfg->tan_half_open) continue;
        if (fabs(zl) > cfg->z_max) continue;
        if (sideA ? zl < 0.0 : zl >= 0.0) continue;
        if (r >= cfg->dead_first && r < cfg->dead_first + cfg->dead_count) continue;
        const u32x4 g = draw(cfg->seed, event_id, (uint32_t)t, (uint32_t)s, (uint32_t)r, ST_SMEAR);
        const double u1 = unif(g.v[0]), u2 = unif(g.v[1]);
        const double rad = sqrt(-2.0 * log(u1));
        const double n1 = rad * cos(2.0 * SYNTH_PI * u2), n2 = rad * sin(2.0 * SYNTH_PI * u2);
        hitrec h;
        h.y = (float)(yl + cfg->sigma * n1);
        h.z = (float)(zl + cfg->sigma * n2);
        h.row = r; h.label = t; h.key = g.v[2]; h.serial = 0;
        h.yt = yl; h.zt = zl; h.st = sphi;
        push(&sec[si], h);
        n_signal[si]++;
      }
    }
  }
  /* uniform noise, a fraction of the signal hits of each sector */
  for (int si = 0; si < ns; ++si) {
    const int s = cfg->sector_first + si;
    const int64_t nn = llround(cfg->noise_frac * (double)n_signal[si]);
    for (int64_t m = 0; m < nn; ++m) {
      const u32x4 g = draw(cfg->seed, event_id, (uint32_t)m, (uint32_t)s, 0, ST_NOISE);
      int r = (int)(unif(g.v[0]) * nr);
      if (r >= nr) r = nr - 1;
      if (r >= cfg->dead_first && r < cfg->dead_first + cfg->dead_count) continue;
      const double xr = (double)rx[r];
      const double yl = (2.0 * unif(g.v[1]) - 1.0) * xr * cfg->tan_half_open;
      double zl = unif(g.v[2]) * cfg->z_max;
      if (s >= 18) zl = -zl;
      hitrec h;
      h.y = (float)yl; h.z = (float)zl; h.row = r; h.label = -1; h.key = g.v[3]; h.serial = 0;
      h.yt = yl; h.zt = zl; h.st = 0.0;
      push(&sec[si], h);
    }
  }
  /* sort by row, random order inside a row (so an index carries no MC
   * information); the serial number only breaks key collisions */
  int64_t total = 0;
  for (int si = 0; si < ns; ++si) {
    for (int64_t i = 0; i < sec[si].n; ++i) sec[si].h[i].serial = (int32_t)i;
    for (int64_t i = 0; i < sec[si].n; ++i) {
      const u32x4 g = draw(cfg->seed, event_id, (uint32_t)i, (uint32_t)(cfg->sector_first + si), 1, ST_PERM);
      sec[si].h[i].key ^= g.v[0];
    }
    if (sec[si].n > 1) qsort(sec[si].h, (size_t)sec[si].n, sizeof(hitrec), hitrec_cmp);
    total += sec[si].n;
  }
  ev->n_sectors = ns;
  ev->n_hits = total;
  ev->hit_offset = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ns + 1));
  const size_t nalloc = (size_t)(total > 0 ? total : 1);
  ev->x = (float*)malloc(sizeof(float) * nalloc);
  ev->y = (float*)malloc(sizeof(float) * nalloc);
  ev->z = (float*)malloc(sizeof(float) * nalloc);
  ev->row = (int32_t*)malloc(sizeof(int32_t) * nalloc);
  ev->label = (int32_t*)malloc(sizeof(int32_t) * nalloc);
  if (want_truth) {
    ev->y_true = (double*)malloc(sizeof(double) * nalloc);
    ev->z_true = (double*)malloc(sizeof(double) * nalloc);
    ev->sinphi_true = (double*)malloc(sizeof(double) * nalloc);
  }
  int64_t o = 0;
  for (int si = 0; si < ns; ++si) {
    ev->hit_offset[si] = o;
    for (int64_t i = 0; i < sec[si].n; ++i, ++o) {
      const hitrec* h = &sec[si].h[i];
      ev->x[o] = rx[h->row]; ev->y[o] = h->y; ev->z[o] = h->z;
      ev->row[o] = h->row; ev->label[o] = h->label;
      if (want_truth) { ev->y_true[o] = h->yt; ev->z_true[o] = h->zt; ev->sinphi_true[o] = h->st; }
    }
    free(sec[si].h);
  }
  ev->hit_offset[ns] = o;
  free(sec); free(n_signal); free(rx);
  return ev;
}

void synth_free(synth_event* ev) {
  if (!ev) return;
  free(ev->hit_offset); free(ev->x); free(ev->y); free(ev->z); free(ev->row); free(ev->label);
  free(ev->y_true); free(ev->z_true); free(ev->sinphi_true);
  free(ev->trk_q); free(ev->trk_pt); free(ev->trk_eta); free(ev->trk_phi0);
  free(ev);
}

/* Multiplicity of event e in the uneven batch: floor(exp(U(ln lo, ln hi))). */
int32_t synth_multiplicity(uint64_t seed, uint32_t e, double lo, double hi) {
  const u32x4 a = draw(seed, 0xFFFFFFFFu, e, 0, 0, ST_MULT);
  return (int32_t)floor(exp(log(lo) + unif(a.v[0]) * (log(hi) - log(lo))));
}

/* Closed-form global helix from the origin, evaluated in a sector-local frame
 * at transverse path length `path`: writes (x, y, z, sin(phi_local)).  Used by
 * tests as the independent reference for the tracker's propagation. */
void synth_helix_point(double q_over_pt, double tanl, double phi0, double bz, double alpha,
                       double path, double out[4]) {
  const double k = -0.00299792458 * bz * q_over_pt;
  const double psi0 = phi0 - alpha;
  double x, y;
  if (fabs(k) < 1e-14) { x = path * cos(psi0); y = path * sin(psi0); }
  else { x = (sin(psi0 + k * path) - sin(psi0)) / k; y = (cos(psi0) - cos(psi0 + k * path)) / k; }
  out[0] = x; out[1] = y; out[2] = tanl * path; out[3] = sin(psi0 + k * path);
}
