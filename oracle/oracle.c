/*
 * Plain CPU oracle of the Hough trigger path -- TEST INFRASTRUCTURE ONLY.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Written for a reader holding the paper: each function names the passage it
 * follows.  The paper gives the method in prose only (no equations); the
 * track parameterisation, the float32 vote formula and the association, fit
 * and vertex rules below are the readings adopted for this implementation and
 * are the definition the GPU library is checked against.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp.
 * Every float32 operation is written as a separate statement or in an
 * expression evaluated left to right, and contraction to FMA is disabled, so
 * each operation is one IEEE-754 round-to-nearest operation.
 *
 * Parity status: vote, peaks and association are pinned by closed forms,
 * brute force and invariants in the test suite; the Gauss-Newton fit is
 * pinned by noiseless tracks (exact truth recovery); the vertex transform is
 * pinned by noiseless tracks from a known vertex.  Physics efficiency figures
 * are not pinned against the paper (its figures carry no numbers).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define C_LIGHT 0.299792458e-2 /* cm^-1 per (T GeV^-1) */

/* ------------------------------------------------------------------------ */
/* Canonical arcsine.  Abramowitz & Stegun, Handbook of Mathematical
 * Functions, formula 4.4.46: for 0 <= a <= 1,
 *   arcsin a = pi/2 - sqrt(1 - a) * (a0 + a1 a + ... + a7 a^7) + e(a),
 *   |e(a)| <= 2e-8,
 * with the published coefficients below.  Evaluated in float32: Horner with
 * separate multiply and add, correctly rounded sqrt, and the sign of u
 * restored by copysign (an odd function, including signed zero). */
static const float AS_A0 = 1.5707963050f;
static const float AS_A1 = -0.2145988016f;
static const float AS_A2 = 0.0889789874f;
static const float AS_A3 = -0.0501743046f;
static const float AS_A4 = 0.0308918810f;
static const float AS_A5 = -0.0170881256f;
static const float AS_A6 = 0.0066700901f;
static const float AS_A7 = -0.0012624911f;
static const float HALF_PI_F = 1.57079632679489661923f;

float oracle_asin_f(float u) {
  float a = fabsf(u);
  float p = AS_A7;
  p = p * a; p = p + AS_A6;
  p = p * a; p = p + AS_A5;
  p = p * a; p = p + AS_A4;
  p = p * a; p = p + AS_A3;
  p = p * a; p = p + AS_A2;
  p = p * a; p = p + AS_A1;
  p = p * a; p = p + AS_A0;
  float one_minus = 1.0f - a;
  float s = sqrtf(one_minus);
  float sp = s * p;
  float r = HALF_PI_F - sp;
  return copysignf(r, u);
}

void oracle_asin_f_array(const float* u, float* out, int64_t n) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = oracle_asin_f(u[i]);
}

/* ------------------------------------------------------------------------ */
/* Track parameterisation (the paper says only that the tracking Hough finds
 * the transverse momentum of prompt and non-prompt tracks).  Reading used:
 * curvature kappa = -c_B q/pT (counter-clockwise positive), c_B =
 * 0.299792458e-2 B; perigee point d0 (-sin phi0, cos phi0) with direction
 * phi0.  A point of that circle at radius r has azimuth phi_h with
 *   sin(phi_h - phi0) = u = (kappa (r^2 + d0^2) + 2 d0) / (2 r (1 + kappa d0)),
 * and the outgoing branch is phi_h = phi0 + asin(u).  Hence a hit votes, in
 * column (q/pT_j, d0_k), for phi0 = phi_h - asin(u).
 *
 * Tables at bin centres, float64 then one rounding to float32:
 *   KAP[j] = kappa_j, Q[k][j] = kappa_j d0_k^2 + 2 d0_k,
 *   T[k][j] = 0.5 / (1 + kappa_j d0_k), PHI_LO = -pi, INVW = n_phi / (2 pi). */
typedef struct {
  float* kap; /* [n_qpt] */
  float* q;   /* [n_d0 * n_qpt] */
  float* t;   /* [n_d0 * n_qpt] */
  float phi_lo, invw;
} tables;

static int grid_ok(const or_grid* g) {
  if (!g) return 0;
  if (g->n_phi < 4 || g->n_qpt < 1 || g->n_d0 < 1) return 0;
  if ((int64_t)g->n_phi * g->n_qpt * g->n_d0 > 0x7fffffffLL) return 0;
  if (!(g->bfield > 0.0f)) return 0;
  if (!(g->qpt_hi >= g->qpt_lo) || !(g->d0_hi >= g->d0_lo)) return 0;
  return 1;
}

static double qpt_centre(const or_grid* g, int j) {
  return (double)g->qpt_lo + ((double)j + 0.5) * ((double)g->qpt_hi - (double)g->qpt_lo) / (double)g->n_qpt;
}
static double kappa_centre(const or_grid* g, int j) {
  double cb = C_LIGHT * (double)g->bfield;
  return -cb * qpt_centre(g, j);
}
static double d0_centre(const or_grid* g, int k) {
  return (double)g->d0_lo + ((double)k + 0.5) * ((double)g->d0_hi - (double)g->d0_lo) / (double)g->n_d0;
}
static double phi0_centre(const or_grid* g, int i) {
  return -OR_PI + ((double)i + 0.5) * (2.0 * OR_PI / (double)g->n_phi);
}

static int make_tables(const or_grid* g, tables* tb) {
  int nq = g->n_qpt, nd = g->n_d0;
  tb->kap = (float*)malloc(sizeof(float) * (size_t)nq);
  tb->q = (float*)malloc(sizeof(float) * (size_t)nq * nd);
  tb->t = (float*)malloc(sizeof(float) * (size_t)nq * nd);
  if (!tb->kap || !tb->q || !tb->t) return -2;
  for (int j = 0; j < nq; ++j) tb->kap[j] = (float)kappa_centre(g, j);
  for (int k = 0; k < nd; ++k) {
    double d0 = d0_centre(g, k);
    for (int j = 0; j < nq; ++j) {
      double kap = kappa_centre(g, j);
      tb->q[(size_t)k * nq + j] = (float)(kap * d0 * d0 + 2.0 * d0);
      tb->t[(size_t)k * nq + j] = (float)(0.5 / (1.0 + kap * d0));
    }
  }
  tb->phi_lo = (float)(-OR_PI);
  tb->invw = (float)((double)g->n_phi / (2.0 * OR_PI));
  return 0;
}

static void free_tables(tables* tb) {
  free(tb->kap);
  free(tb->q);
  free(tb->t);
}

int oracle_tables(const or_grid* g, float* kap, float* q, float* t, float* consts) {
  if (!grid_ok(g)) return -1;
  tables tb;
  if (make_tables(g, &tb)) { free_tables(&tb); return -2; }
  size_t nc = (size_t)g->n_qpt * g->n_d0;
  memcpy(kap, tb.kap, sizeof(float) * (size_t)g->n_qpt);
  memcpy(q, tb.q, sizeof(float) * nc);
  memcpy(t, tb.t, sizeof(float) * nc);
  consts[0] = tb.phi_lo;
  consts[1] = tb.invw;
  free_tables(&tb);
  return 0;
}

/* Hits with r outside (0, 1e4) cm, |phi| > 4 or a NaN cast no votes. */
static int hit_valid(float r, float phi) {
  return r > 0.0f && r < 1.0e4f && fabsf(phi) <= 4.0f;
}

/* The float32 vote formula, one rounding per operation in this order:
 *   a = KAP*r2; b = a + Q; c = b*ir; u = c*T  (r2 = r*r, ir = 1/r)
 *   no vote unless |u| <= 1
 *   phi0 = phi - asin_f(u); x = (phi0 - PHI_LO) * INVW.
 * Returns 0 (no vote) or 1 and the unfloored coordinate x. */
static int phi0_coord_u(float r2, float ir, float phi, float kap, float q, float t,
                        float phi_lo, float invw, float* x_out, float* u_out) {
  float a = kap * r2;
  float b = a + q;
  float c = b * ir;
  float u = c * t;
  *u_out = u;
  if (!(fabsf(u) <= 1.0f)) return 0;
  float s = oracle_asin_f(u);
  float phi0 = phi - s;
  float d = phi0 - phi_lo;
  *x_out = d * invw;
  return 1;
}

static int phi0_coord(float r2, float ir, float phi, float kap, float q, float t,
                      float phi_lo, float invw, float* x_out) {
  float u;
  return phi0_coord_u(r2, ir, phi, kap, q, t, phi_lo, invw, x_out, &u);
}

/* floor of x, then periodic wrap into [0, n) */
static int wrap_bin(float x, int n) {
  int i = (int)floorf(x);
  return ((i % n) + n) % n;
}

int oracle_phi0_coord(const or_grid* g, const float* r, const float* phi, int32_t n,
                      const int32_t* j, const int32_t* k, float* x, int32_t* bin,
                      int32_t* valid) {
  if (!grid_ok(g) || n < 0) return -1;
  tables tb;
  if (make_tables(g, &tb)) { free_tables(&tb); return -2; }
  for (int32_t h = 0; h < n; ++h) {
    valid[h] = 0;
    x[h] = 0.0f;
    bin[h] = -1;
    if (j[h] < 0 || j[h] >= g->n_qpt || k[h] < 0 || k[h] >= g->n_d0) continue;
    if (!hit_valid(r[h], phi[h])) continue;
    float r2 = r[h] * r[h];
    float ir = 1.0f / r[h];
    size_t c = (size_t)k[h] * g->n_qpt + j[h];
    float xv;
    if (phi0_coord(r2, ir, phi[h], tb.kap[j[h]], tb.q[c], tb.t[c], tb.phi_lo, tb.invw, &xv)) {
      valid[h] = 1;
      x[h] = xv;
      bin[h] = wrap_bin(xv, g->n_phi);
    }
  }
  free_tables(&tb);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Vote: acc[k][j][i] = number of valid hits whose phi0 bin in column (j,k)
 * is i -- the paper's "each instance starts at zero, each datum adds a vote
 * to every instance that would include it" (section "Hough Transform
 * Algorithm"), with one instance per (phi0, q/pT, d0) cell. */
int oracle_hough_vote(const or_grid* g, const float* r, const float* phi, int32_t n_hits,
                      int32_t* acc, uint64_t* n_votes) {
  if (!grid_ok(g) || n_hits < 0 || !acc) return -1;
  tables tb;
  if (make_tables(g, &tb)) { free_tables(&tb); return -2; }
  const int np = g->n_phi, nq = g->n_qpt, nd = g->n_d0;
  const int64_t ncol = (int64_t)nq * nd;
  uint64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
  for (int64_t col = 0; col < ncol; ++col) {
    int j = (int)(col % nq);
    int32_t* row = acc + col * np;
    for (int i = 0; i < np; ++i) row[i] = 0;
    for (int32_t h = 0; h < n_hits; ++h) {
      if (!hit_valid(r[h], phi[h])) continue;
      float r2 = r[h] * r[h];
      float ir = 1.0f / r[h];
      float x;
      if (!phi0_coord(r2, ir, phi[h], tb.kap[j], tb.q[col], tb.t[col], tb.phi_lo, tb.invw, &x))
        continue;
      row[wrap_bin(x, np)] += 1;
      total += 1;
    }
  }
  if (n_votes) *n_votes = total;
  free_tables(&tb);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Band (cell) vote, a variant of the vote above: instead of the point at
 * the column centre, a hit votes for every phi0 bin that its curve reaches
 * while (kappa, d0) range over the column's cell (the paper's instances are
 * cells of the parameter space, section "Hough Transform Algorithm").
 * Reading used: u is increasing in kappa and in d0 over the cell (true
 * while r > |d0| and kappa^2 r^2 < (1 + kappa d0)^2 + 1), so u spans
 * [u_lo, u_hi] with u_lo at (smallest kappa, lower d0 edge) and u_hi at
 * (largest kappa, upper d0 edge); kappa = -0.299792458e-2 B q/pT, so the
 * smallest kappa is at the upper q/pT edge.  Both come from the float32
 * vote formula with the corner's tables (float64, rounded once).  No vote
 * when u_lo > 1 or u_hi < -1; otherwise u is clipped to [-1, 1], the band's
 * coordinates are x_a = (phi - asin_f(u_hi) - PHI_LO) INVW and x_b =
 * (phi - asin_f(u_lo) - PHI_LO) INVW, and every bin from floor(min) to
 * floor(max) gets one vote (periodic; a band of n_phi or more bins votes
 * once in every bin). */
static double qpt_edge(const or_grid* g, int j) {
  return (double)g->qpt_lo + (double)j * ((double)g->qpt_hi - (double)g->qpt_lo) / (double)g->n_qpt;
}
static double d0_edge(const or_grid* g, int k) {
  return (double)g->d0_lo + (double)k * ((double)g->d0_hi - (double)g->d0_lo) / (double)g->n_d0;
}

int oracle_hough_vote_cell(const or_grid* g, const float* r, const float* phi, int32_t n_hits,
                           int32_t* acc, uint64_t* n_votes) {
  if (!grid_ok(g) || n_hits < 0 || !acc) return -1;
  const int np = g->n_phi, nq = g->n_qpt, nd = g->n_d0;
  const int64_t ncol = (int64_t)nq * nd;
  const double cb = C_LIGHT * (double)g->bfield;
  const float phi_lo = (float)(-OR_PI);
  const float invw = (float)((double)np / (2.0 * OR_PI));
  uint64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
  for (int64_t col = 0; col < ncol; ++col) {
    int j = (int)(col % nq), k = (int)(col / nq);
    /* corners: (smallest kappa, lower d0 edge) and (largest kappa, upper d0 edge) */
    double klo = -cb * qpt_edge(g, j + 1), khi = -cb * qpt_edge(g, j);
    double dlo = d0_edge(g, k), dhi = d0_edge(g, k + 1);
    float kl = (float)klo, kh = (float)khi;
    float ql = (float)(klo * dlo * dlo + 2.0 * dlo), tl = (float)(0.5 / (1.0 + klo * dlo));
    float qh = (float)(khi * dhi * dhi + 2.0 * dhi), th = (float)(0.5 / (1.0 + khi * dhi));
    int32_t* row = acc + col * np;
    for (int i = 0; i < np; ++i) row[i] = 0;
    for (int32_t h = 0; h < n_hits; ++h) {
      if (!hit_valid(r[h], phi[h])) continue;
      float r2 = r[h] * r[h];
      float ir = 1.0f / r[h];
      float ulo = ((kl * r2 + ql) * ir) * tl;
      float uhi = ((kh * r2 + qh) * ir) * th;
      if (ulo > 1.0f || uhi < -1.0f || ulo != ulo || uhi != uhi) continue;
      if (ulo < -1.0f) ulo = -1.0f;
      if (uhi > 1.0f) uhi = 1.0f;
      float xa = ((phi[h] - oracle_asin_f(uhi)) - phi_lo) * invw;
      float xb = ((phi[h] - oracle_asin_f(ulo)) - phi_lo) * invw;
      float lo = xa < xb ? xa : xb, hi = xa < xb ? xb : xa;
      int ia = (int)floorf(lo), ib = (int)floorf(hi);
      int m = ib - ia + 1;
      if (m >= np) {
        for (int i = 0; i < np; ++i) row[i] += 1;
        total += (uint64_t)np;
      } else {
        for (int q = 0; q < m; ++q) row[(((ia + q) % np) + np) % np] += 1;
        total += (uint64_t)m;
      }
    }
  }
  if (n_votes) *n_votes = total;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Peaks: local maxima of the accumulator (section "Hough Transform
 * Algorithm"; the same finder serves the second transform, section "Jet and
 * Black Hole Detection").  Reading used: cell c is a peak iff acc[c] >= T and,
 * for each of its 26 (3D) neighbours c+o inside the q/pT and d0 range (phi0
 * is periodic), acc[c] > acc[c+o] when o = (dk, dj, di) is lexicographically
 * negative and acc[c] >= acc[c+o] otherwise.  Output sorted by cell index. */
static int is_peak3(const int32_t* acc, int np, int nq, int nd, int k, int j, int i,
                    int32_t thr) {
  int32_t v = acc[((int64_t)k * nq + j) * np + i];
  if (v < thr) return 0;
  for (int dk = -1; dk <= 1; ++dk) {
    int kk = k + dk;
    if (kk < 0 || kk >= nd) continue;
    for (int dj = -1; dj <= 1; ++dj) {
      int jj = j + dj;
      if (jj < 0 || jj >= nq) continue;
      for (int di = -1; di <= 1; ++di) {
        if (dk == 0 && dj == 0 && di == 0) continue;
        int ii = ((i + di) % np + np) % np;
        int32_t w = acc[((int64_t)kk * nq + jj) * np + ii];
        int negative = dk < 0 || (dk == 0 && (dj < 0 || (dj == 0 && di < 0)));
        if (negative ? !(v > w) : !(v >= w)) return 0;
      }
    }
  }
  return 1;
}

int oracle_hough_peaks(const or_grid* g, const int32_t* acc, int32_t min_votes,
                       or_peak* out, int32_t capacity, int32_t* n_found) {
  if (!grid_ok(g) || !acc || capacity < 0 || !n_found) return -1;
  const int np = g->n_phi, nq = g->n_qpt, nd = g->n_d0;
  const int64_t ncol = (int64_t)nq * nd;
  /* per-column peak counts, then an in-order fill (deterministic) */
  int32_t* cnt = (int32_t*)calloc((size_t)ncol, sizeof(int32_t));
  if (!cnt) return -2;
#pragma omp parallel for schedule(static)
  for (int64_t col = 0; col < ncol; ++col) {
    int k = (int)(col / nq), j = (int)(col % nq);
    int32_t c = 0;
    for (int i = 0; i < np; ++i) c += is_peak3(acc, np, nq, nd, k, j, i, min_votes);
    cnt[col] = c;
  }
  int64_t total = 0;
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ncol + 1));
  if (!off) { free(cnt); return -2; }
  for (int64_t col = 0; col < ncol; ++col) { off[col] = total; total += cnt[col]; }
#pragma omp parallel for schedule(static)
  for (int64_t col = 0; col < ncol; ++col) {
    if (cnt[col] == 0 || off[col] >= capacity) continue;
    int k = (int)(col / nq), j = (int)(col % nq);
    int64_t o = off[col];
    for (int i = 0; i < np && o < capacity; ++i) {
      if (is_peak3(acc, np, nq, nd, k, j, i, min_votes)) {
        int64_t lin = col * np + i;
        out[o].lin = (int32_t)lin;
        out[o].votes = acc[lin];
        ++o;
      }
    }
  }
  *n_found = (int32_t)(total > 0x7fffffff ? 0x7fffffff : total);
  free(cnt);
  free(off);
  return 0;
}


/* ------------------------------------------------------------------------ */
/* Canonical sine and cosine in float64 for hit Cartesian coordinates:
 * Cody-Waite reduction by pi/2 (two-part constant, the high part holding 33
 * bits so k * high is exact for |k| <= 3) followed by Taylor series of sin
 * and cos on |r| <= pi/4 (truncation below 1e-17).  Only arithmetic, so the
 * result is reproducible bit for bit on any IEEE-754 machine with the same
 * operation order.  Valid for |a| <= 4 (valid hits). */
static const double PIO2_HI = 1.57079632673412561417e+00;
static const double PIO2_LO = 6.07710050650619224932e-11;

static void csincos(double a, double* s_out, double* c_out) {
  double t = a * 0.63661977236758134308;
  double kf = floor(t + 0.5);
  double r = a - kf * PIO2_HI;
  r = r - kf * PIO2_LO;
  double z = r * r;
  double ps = -1.0 / 355687428096000.0;            /* -1/17! */
  ps = ps * z + 1.0 / 1307674368000.0;             /*  1/15! */
  ps = ps * z - 1.0 / 6227020800.0;                /* -1/13! */
  ps = ps * z + 1.0 / 39916800.0;                  /*  1/11! */
  ps = ps * z - 1.0 / 362880.0;                    /* -1/9!  */
  ps = ps * z + 1.0 / 5040.0;                      /*  1/7!  */
  ps = ps * z - 1.0 / 120.0;                       /* -1/5!  */
  ps = ps * z + 1.0 / 6.0;                         /*  1/3!  */
  double sn = r - r * z * ps;                      /* r - r^3/3! + ... */
  double pc = 1.0 / 20922789888000.0;              /*  1/16! */
  pc = pc * z - 1.0 / 87178291200.0;               /* -1/14! */
  pc = pc * z + 1.0 / 479001600.0;                 /*  1/12! */
  pc = pc * z - 1.0 / 3628800.0;                   /* -1/10! */
  pc = pc * z + 1.0 / 40320.0;                     /*  1/8!  */
  pc = pc * z - 1.0 / 720.0;                       /* -1/6!  */
  pc = pc * z + 1.0 / 24.0;                        /*  1/4!  */
  pc = pc * z - 0.5;                               /* -1/2!  */
  double cs = 1.0 + z * pc;
  int q = ((int)kf) & 3;
  if (q == 0) { *s_out = sn; *c_out = cs; }
  else if (q == 1) { *s_out = cs; *c_out = -sn; }
  else if (q == 2) { *s_out = -sn; *c_out = -cs; }
  else { *s_out = -cs; *c_out = sn; }
}

/* Canonical float64 atan2: octant reduction to 0 <= z <= 1, then
 * atan z = pi/6 + atan((sqrt3 z - 1) / (z + sqrt3)) above tan(pi/12), then the
 * Taylor series of atan on |z| <= 2 - sqrt3 up to z^35 (truncation below
 * 1e-21).  Arithmetic only, reproducible bit for bit. */
static double catan2(double y, double x) {
  double ax = fabs(x), ay = fabs(y);
  int swap = ay > ax;
  double num = swap ? ax : ay, den = swap ? ay : ax;
  if (den == 0.0) return 0.0;
  double z = num / den;
  double base = 0.0;
  const double SQRT3 = 1.73205080756887729353;
  const double TAN_PI_12 = 0.26794919243112270647;
  if (z > TAN_PI_12) {
    z = (z * SQRT3 - 1.0) / (z + SQRT3);
    base = OR_PI / 6.0;
  }
  double w = z * z;
  double p = -1.0 / 35.0;
  p = p * w + 1.0 / 33.0;
  p = p * w - 1.0 / 31.0;
  p = p * w + 1.0 / 29.0;
  p = p * w - 1.0 / 27.0;
  p = p * w + 1.0 / 25.0;
  p = p * w - 1.0 / 23.0;
  p = p * w + 1.0 / 21.0;
  p = p * w - 1.0 / 19.0;
  p = p * w + 1.0 / 17.0;
  p = p * w - 1.0 / 15.0;
  p = p * w + 1.0 / 13.0;
  p = p * w - 1.0 / 11.0;
  p = p * w + 1.0 / 9.0;
  p = p * w - 1.0 / 7.0;
  p = p * w + 1.0 / 5.0;
  p = p * w - 1.0 / 3.0;
  double a = base + (z + z * w * p);
  if (swap) a = OR_PI / 2.0 - a;
  if (x < 0.0) a = OR_PI - a;
  if (y < 0.0) a = -a;
  return a;
}

void oracle_atan2_array(const double* y, const double* x, double* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = catan2(y[i], x[i]);
}

void oracle_sincos_array(const double* a, double* s, double* c, int64_t n) {
  for (int64_t i = 0; i < n; ++i) csincos(a[i], &s[i], &c[i]);
}

/* ------------------------------------------------------------------------ */
/* Candidate refinement (section "Jet and Black Hole Detection": candidates
 * from the peak finder are refined before the second transform; the paper
 * uses a Kalman filter, this implementation a seeded road search plus a
 * least-squares fit).  Reading used, per peak cell (i, j, k):
 *
 *  members   valid hits whose coordinate x in column (j, k), on the periodic
 *            image nearest the cell, satisfies |x - (i + 0.5)| <= w with
 *            w = 0.5 + win_bins + 1.5 INVW (hd0 / r + hk r / 2) / sqrt(1 - u^2):
 *            the cell widened by the phi0 spread of a hit across the
 *            column's d0 half-width hd0 and curvature half-width hk, to first
 *            order (du/dd0 ~ 1/r, du/dkappa ~ r/2, arcsine slope
 *            1/sqrt(1 - u^2)), with 1.5 covering the (1 + kappa d0) factors
 *            of the exact derivatives.  More than member_cap members drops
 *            the candidate.
 *  seed      among the layers with members (ascending layer index = radius),
 *            take the outer min(n, min_layers) of them; the seed layers are
 *            the innermost, middle and outermost of that span.  For every
 *            combination of the seed_k members nearest the cell centre on
 *            each seed layer, the circle through the three hits (float64,
 *            algebraic form A(x^2+y^2) + Bx + Cy + D = 0 normalised to
 *            B^2 + C^2 - 4AD = 1, oriented so the track runs from the inner to
 *            the outer hit) must have kappa = 2A and d0 = 2D / (1 + sqrt(B^2 +
 *            C^2)) within the cell widened by box_margin bins; its inliers
 *            are, per member layer, the member nearest the circle in signed
 *            distance 2f / (1 + sqrt(1 + 4Af)) if within road_sigmas *
 *            sigma_rphi.  The best seed has the most inlier layers, then the
 *            smallest sum of squared inlier distances, then comes first.
 *  candidate best seed with at least min_layers inlier layers.
 *
 * All of it is float32 vote arithmetic or float64 arithmetic and square roots
 * in a fixed order, so every decision is reproducible bit for bit. */
typedef struct {
  int32_t n_layers, n_inliers, status; /* status 0 ok, 1 too few layers/inliers, 2 member overflow */
  int32_t n_members;
  int64_t n_tests;                     /* (admissible seed circle, member) road tests */
  int32_t hit[OR_MAX_LAYERS];          /* inlier hit per layer */
  double ss;                           /* sum of squared inlier distances */
  double A, B, C, D;                   /* seed circle */
} cand_t;

typedef struct {
  int32_t h;
  int32_t layer;
  float adx;
} member_t;

static int member_less(const member_t* a, const member_t* b) {
  if (a->adx != b->adx) return a->adx < b->adx;
  return a->h < b->h;
}

/* circle through P1, P2, P3 (inner to outer); returns 0 when degenerate */
static int circle3(double x1, double y1, double x2, double y2, double x3, double y3, double* A,
                   double* B, double* C, double* D) {
  double X2 = x2 - x1, Y2 = y2 - y1, X3 = x3 - x1, Y3 = y3 - y1;
  double q2 = X2 * X2 + Y2 * Y2;
  double q3 = X3 * X3 + Y3 * Y3;
  /* circle through the origin of the shifted frame: (q, X, Y) . (a, b, c) = 0 */
  double a = X2 * Y3 - Y2 * X3;
  double b = Y2 * q3 - q2 * Y3;
  double c = q2 * X3 - X2 * q3;
  double nrm2 = b * b + c * c;
  if (!(nrm2 > 0.0)) return 0;
  double nrm = sqrt(nrm2);
  double q1 = x1 * x1 + y1 * y1;
  double AA = a;
  double BB = b - 2.0 * a * x1;
  double CC = c - 2.0 * a * y1;
  double DD = a * q1 - b * x1 - c * y1;
  AA = AA / nrm;
  BB = BB / nrm;
  CC = CC / nrm;
  DD = DD / nrm;
  /* direction of motion at the perigee is proportional to (-C, B) */
  double dir = -CC * (x3 - x1) + BB * (y3 - y1);
  if (dir == 0.0) return 0;
  if (dir < 0.0) { AA = -AA; BB = -BB; CC = -CC; DD = -DD; }
  *A = AA; *B = BB; *C = CC; *D = DD;
  return 1;
}

static double circle_dist(double A, double B, double C, double D, double x, double y, double q) {
  double f = A * q + B * x + C * y + D;
  double s = 1.0 + 4.0 * A * f;
  if (s < 0.0) s = 0.0;
  return 2.0 * f / (1.0 + sqrt(s));
}

typedef struct {
  double* x;
  double* y;
  double* q;
} hitxy_t;

typedef struct {
  float hd0, hk;          /* half column widths for the member window */
  double kbin, dbin;      /* full column widths in kappa and d0 */
} window_t;

static void refine(const or_grid* g, const tables* tb, const window_t* wd, const hitxy_t* hx,
                   const float* r, const float* phi, const uint8_t* layer, int32_t n_hits,
                   int32_t lin, const or_cluster_cfg* cfg, member_t* mem, cand_t* out) {
  const int np = g->n_phi, nq = g->n_qpt;
  out->status = 1;
  out->n_layers = 0;
  out->n_inliers = 0;
  out->ss = 0.0;
  for (int L = 0; L < OR_MAX_LAYERS; ++L) out->hit[L] = -1;
  /* a cell index outside the grid is not a candidate */
  if (lin < 0 || (int64_t)lin >= (int64_t)np * nq * g->n_d0) return;
  int i = lin % np, col = lin / np, j = col % nq, k = col / nq;
  float xi = (float)i + 0.5f;
  float half_n = 0.5f * (float)np;
  float wbase = 0.5f + (float)cfg->win_bins;
  int nm = 0;
  out->n_members = 0;
  out->n_tests = 0;
  out->status = 1;
  out->n_layers = 0;
  out->n_inliers = 0;
  out->ss = 0.0;
  for (int L = 0; L < OR_MAX_LAYERS; ++L) out->hit[L] = -1;
  for (int32_t h = 0; h < n_hits; ++h) {
    if (!hit_valid(r[h], phi[h])) continue;
    int L = layer[h];
    if (L >= OR_MAX_LAYERS) continue;
    float r2 = r[h] * r[h];
    float ir = 1.0f / r[h];
    float x, u;
    if (!phi0_coord_u(r2, ir, phi[h], tb->kap[j], tb->q[col], tb->t[col], tb->phi_lo, tb->invw,
                      &x, &u))
      continue;
    float dx = x - xi;
    if (dx > half_n) dx = (x - (float)np) - xi;
    else if (dx < -half_n) dx = (x + (float)np) - xi;
    float e1 = wd->hd0 * ir;
    float e2 = r[h] * 0.5f;
    float e3 = wd->hk * e2;
    float e4 = e1 + e3;
    float e5 = tb->invw * e4;
    float uu = u * u;
    float gg = 1.0f - uu;
    float sg = sqrtf(gg);
    float e6 = e5 * 1.5f;
    float e7 = e6 / sg;
    float w = wbase + e7;
    float adx = fabsf(dx);
    if (!(adx <= w)) continue;
    if (nm >= cfg->member_cap) { out->status = 2; out->n_members = 0; return; }
    mem[nm].h = h;
    mem[nm].layer = L;
    mem[nm].adx = adx;
    ++nm;
  }
  out->n_members = nm;
  /* member layers */
  int cntL[OR_MAX_LAYERS] = {0};
  for (int m = 0; m < nm; ++m) cntL[mem[m].layer]++;
  int S[OR_MAX_LAYERS], nS = 0;
  for (int L = 0; L < OR_MAX_LAYERS; ++L)
    if (cntL[L] > 0) S[nS++] = L;
  out->n_layers = nS;
  if (nS < cfg->min_layers || nS < 3) return;
  int span = nS < cfg->min_layers ? nS : cfg->min_layers;
  int Ls[3] = {S[nS - span], S[nS - span + (span - 1) / 2], S[nS - 1]};
  /* prompt grid (one d0 column at d0 = 0): seeds are the beam line plus the
   * middle and outer seed hits */
  const int origin_seed = (g->n_d0 == 1 && g->d0_lo == 0.0f && g->d0_hi == 0.0f);
  /* seed_k nearest-to-centre members of each seed layer (insertion order) */
  int seed[3][64];
  int ns[3];
  int kk = cfg->seed_k < 64 ? cfg->seed_k : 64;
  for (int s = 0; s < 3; ++s) {
    ns[s] = 0;
    for (int m = 0; m < nm; ++m) {
      if (mem[m].layer != Ls[s]) continue;
      /* insert m into the sorted list, keep at most kk */
      int pos = ns[s];
      while (pos > 0 && member_less(&mem[m], &mem[seed[s][pos - 1]])) --pos;
      if (pos >= kk) continue;
      int top = ns[s] < kk ? ns[s] : kk - 1;
      for (int q = top; q > pos; --q) seed[s][q] = seed[s][q - 1];
      seed[s][pos] = m;
      if (ns[s] < kk) ns[s]++;
    }
  }
  if (origin_seed) ns[0] = 1;
  const double kap_c = kappa_centre(g, j), d0_c = d0_centre(g, k);
  double ktol = (0.5 + (double)cfg->box_margin) * wd->kbin;
  if (ktol < 1e-6) ktol = 1e-6;
  const double road = (double)cfg->road_sigmas * (double)cfg->sigma_rphi;
  double dtol = (0.5 + (double)cfg->box_margin) * wd->dbin + road;
  int best_n = -1;
  double best_ss = 0.0;
  for (int a = 0; a < ns[0]; ++a) {
    double xa = 0.0, ya = 0.0;
    if (!origin_seed) {
      int ha = mem[seed[0][a]].h;
      xa = hx->x[ha];
      ya = hx->y[ha];
    }
    for (int b = 0; b < ns[1]; ++b) {
      int hb = mem[seed[1][b]].h;
      for (int c = 0; c < ns[2]; ++c) {
        int hc = mem[seed[2][c]].h;
        double A, B, C, D;
        if (!circle3(xa, ya, hx->x[hb], hx->y[hb], hx->x[hc], hx->y[hc], &A, &B, &C, &D))
          continue;
        double kap = 2.0 * A;
        double sq = sqrt(B * B + C * C);
        double d0 = 2.0 * D / (1.0 + sq);
        if (!(fabs(kap - kap_c) <= ktol) || !(fabs(d0 - d0_c) <= dtol)) continue;
        out->n_tests += nm;
        int n_in = 0;
        double ss = 0.0;
        int hit[OR_MAX_LAYERS];
        double bd[OR_MAX_LAYERS];
        for (int L = 0; L < OR_MAX_LAYERS; ++L) { hit[L] = -1; bd[L] = 0.0; }
        for (int m = 0; m < nm; ++m) {
          int h = mem[m].h;
          double dist = fabs(circle_dist(A, B, C, D, hx->x[h], hx->y[h], hx->q[h]));
          if (!(dist <= road)) continue;
          int L = mem[m].layer;
          if (hit[L] < 0 || dist < bd[L]) { hit[L] = h; bd[L] = dist; }
        }
        for (int L = 0; L < OR_MAX_LAYERS; ++L)
          if (hit[L] >= 0) { ++n_in; ss += bd[L] * bd[L]; }
        if (n_in > best_n || (n_in == best_n && ss < best_ss)) {
          best_n = n_in;
          best_ss = ss;
          out->A = A; out->B = B; out->C = C; out->D = D;
          for (int L = 0; L < OR_MAX_LAYERS; ++L) out->hit[L] = hit[L];
        }
      }
    }
  }
  if (best_n < 0) { for (int L = 0; L < OR_MAX_LAYERS; ++L) out->hit[L] = -1; return; }
  out->n_inliers = best_n;
  out->ss = best_ss;
  if (best_n >= cfg->min_layers) out->status = 0;
  else for (int L = 0; L < OR_MAX_LAYERS; ++L) out->hit[L] = -1;
}

/* Ownership (duplicate cleaning, in the spirit of the cleaning step of the
 * combinatorial track finder, section "Current Tracker and Tracking
 * Algorithm"): each inlier hit goes to the candidate with the most inlier
 * layers, then the smallest seed sum of squares (rounded to float32), then
 * the smallest cell index; a candidate survives when it owns at least
 * min_layers of its inlier hits.  Single pass. */
static int key_greater(int n_a, float ss_a, int lin_a, int n_b, float ss_b, int lin_b) {
  if (n_a != n_b) return n_a > n_b;
  if (ss_a != ss_b) return ss_a < ss_b;
  return lin_a < lin_b;
}

/* Candidates p with n_in[p] >= 0 take part, in index order; hits[p][L] is
 * the inlier hit of layer L (-1 none).  owner[h] receives the candidate that
 * owns hit h (-1 none), n_owned[p] the inlier hits p owns. */
static void ownership(int32_t n_cand, const int32_t* n_in, const float* ss, const int32_t* lin,
                      const int32_t* hits, int32_t n_hits, int32_t* owner, int32_t* n_owned) {
  for (int32_t h = 0; h < n_hits; ++h) owner[h] = -1;
  for (int32_t p = 0; p < n_cand; ++p) {
    if (n_in[p] < 0) continue;
    for (int L = 0; L < OR_MAX_LAYERS; ++L) {
      int32_t h = hits[(size_t)p * OR_MAX_LAYERS + L];
      if (h < 0 || h >= n_hits) continue;
      int32_t o = owner[h];
      if (o < 0 || key_greater(n_in[p], ss[p], lin[p], n_in[o], ss[o], lin[o])) owner[h] = p;
    }
  }
  for (int32_t p = 0; p < n_cand; ++p) {
    int own = 0;
    if (n_in[p] >= 0)
      for (int L = 0; L < OR_MAX_LAYERS; ++L) {
        int32_t h = hits[(size_t)p * OR_MAX_LAYERS + L];
        if (h >= 0 && h < n_hits && owner[h] == p) ++own;
      }
    n_owned[p] = own;
  }
}

int oracle_ownership(int32_t n_cand, const int32_t* n_in, const float* ss, const int32_t* lin,
                     const int32_t* hits, int32_t n_hits, int32_t* owner, int32_t* n_owned) {
  if (n_cand < 0 || n_hits < 0 || (n_cand > 0 && (!n_in || !ss || !lin || !hits || !n_owned)) ||
      (n_hits > 0 && !owner))
    return -1;
  ownership(n_cand, n_in, ss, lin, hits, n_hits, owner, n_owned);
  return 0;
}

/* Refit (stands in for the Kalman filter of section "Jet and Black Hole
 * Detection"): weighted least squares in float64 by Gauss-Newton from the
 * seed circle, model phi_pred(r) = phi0 + asin(u(r; kappa, d0)), residual
 * wrapped into [-pi, pi), weight r^2 (constant r-phi resolution).  kappa is
 * free when n_qpt > 1 and d0 when n_d0 > 1; otherwise they stay at the column
 * value.  Status 1 when a hit has |u| >= 1, 2 when the normal matrix is not
 * positive definite; then the cell centre is reported and chi2 = -1. */
static double wrap_pi(double a) {
  return a - 2.0 * OR_PI * floor((a + OR_PI) / (2.0 * OR_PI));
}

static void fit_track(const or_grid* g, const float* r, const float* phi, const int32_t* hits,
                      int32_t lin, const cand_t* cd, int iters, float sigma, or_track* t) {
  const int np = g->n_phi, nq = g->n_qpt;
  int i = lin % np, col = lin / np, j = col % nq, k = col / nq;
  double p[3];
  double sq0 = sqrt(cd->B * cd->B + cd->C * cd->C);
  p[0] = atan2(cd->B, -cd->C);
  p[1] = g->n_qpt > 1 ? 2.0 * cd->A : kappa_centre(g, j);
  p[2] = g->n_d0 > 1 ? 2.0 * cd->D / (1.0 + sq0) : d0_centre(g, k);
  int freep[3] = {1, g->n_qpt > 1, g->n_d0 > 1};
  int idx[3], nfree = 0;
  for (int a = 0; a < 3; ++a)
    if (freep[a]) idx[nfree++] = a;
  int status = 0;
  for (int it = 0; it < iters && status == 0; ++it) {
    double Am[3][3] = {{0}}, gv[3] = {0};
    for (int L = 0; L < OR_MAX_LAYERS; ++L) {
      int h = hits[L];
      if (h < 0) continue;
      double rr = (double)r[h], ph = (double)phi[h];
      double kap = p[1], d0 = p[2];
      double den = 1.0 + kap * d0;
      double u = (kap * (rr * rr + d0 * d0) + 2.0 * d0) / (2.0 * rr * den);
      if (!(fabs(u) < 1.0)) { status = 1; break; }
      double sq = sqrt(1.0 - u * u);
      double res = wrap_pi(ph - (p[0] + asin(u)));
      double jac[3];
      jac[0] = 1.0;
      jac[1] = (rr * rr - d0 * d0) / (2.0 * rr * den * den) / sq;
      jac[2] = (den * den + 1.0 - kap * kap * rr * rr) / (2.0 * rr * den * den) / sq;
      double w = rr * rr;
      for (int a = 0; a < nfree; ++a) {
        gv[a] += w * jac[idx[a]] * res;
        for (int b = 0; b < nfree; ++b) Am[a][b] += w * jac[idx[a]] * jac[idx[b]];
      }
    }
    if (status) break;
    /* Cholesky Am = L L^T, then L y = g, L^T d = y */
    double Lm[3][3] = {{0}};
    for (int a = 0; a < nfree && !status; ++a) {
      for (int b = 0; b <= a; ++b) {
        double s = Am[a][b];
        for (int c = 0; c < b; ++c) s -= Lm[a][c] * Lm[b][c];
        if (a == b) {
          if (!(s > 0.0)) { status = 2; break; }
          Lm[a][a] = sqrt(s);
        } else {
          Lm[a][b] = s / Lm[b][b];
        }
      }
    }
    if (status) break;
    double y[3], d[3];
    for (int a = 0; a < nfree; ++a) {
      double s = gv[a];
      for (int c = 0; c < a; ++c) s -= Lm[a][c] * y[c];
      y[a] = s / Lm[a][a];
    }
    for (int a = nfree - 1; a >= 0; --a) {
      double s = y[a];
      for (int c = a + 1; c < nfree; ++c) s -= Lm[c][a] * d[c];
      d[a] = s / Lm[a][a];
    }
    for (int a = 0; a < nfree; ++a) p[idx[a]] += d[a];
  }
  double chi2 = 0.0;
  if (status == 0) {
    for (int L = 0; L < OR_MAX_LAYERS; ++L) {
      int h = hits[L];
      if (h < 0) continue;
      double rr = (double)r[h], ph = (double)phi[h];
      double kap = p[1], d0 = p[2];
      double den = 1.0 + kap * d0;
      double u = (kap * (rr * rr + d0 * d0) + 2.0 * d0) / (2.0 * rr * den);
      if (!(fabs(u) < 1.0)) { status = 1; break; }
      double res = wrap_pi(ph - (p[0] + asin(u)));
      double z = rr * res / (double)sigma;
      chi2 += z * z;
    }
  }
  double cb = C_LIGHT * (double)g->bfield;
  if (status != 0) {
    p[0] = phi0_centre(g, i);
    p[1] = kappa_centre(g, j);
    p[2] = d0_centre(g, k);
    chi2 = -1.0;
  }
  t->status = status;
  t->phi0 = (float)wrap_pi(p[0]);
  t->qpt = (float)(-p[1] / cb);
  t->d0 = (float)p[2];
  t->chi2 = (float)chi2;
}

/* Refit by a Kalman filter (the paper refines candidates with a Kalman
 * filter on the CPU, section "Jet and Black Hole Detection"; here it runs on
 * the device as an alternative to the Gauss-Newton fit).  Reading: state
 * p = (phi0, kappa, d0) at the perigee, the free ones only (as in the
 * Gauss-Newton fit), starting from the seed circle.  Each pass filters the
 * deviation dp from a reference state (the seed, then the previous pass's
 * result), with the measurement model phi0 + asin(u(r; kappa, d0))
 * linearised at the reference, as track fits do about a reference
 * trajectory: prior dp = 0 with covariance diag(0.1^2, 0.01^2, 10^2) (rad,
 * cm^-1, cm), weak against the hits; the owned hits in increasing radius,
 * each an azimuth measurement of variance (sigma / r)^2 with innovation
 * res - H dp; no process noise (the toy detector has no material); the pass
 * ends with p += dp.  iters passes.  Status 1 when a hit has |u| >= 1, 2 when
 * an innovation variance is not positive; chi2 as for the Gauss-Newton fit. */
static void kf_track(const or_grid* g, const float* r, const float* phi, const int32_t* hits,
                     int32_t lin, const cand_t* cd, int iters, float sigma, or_track* t) {
  const int np = g->n_phi, nq = g->n_qpt;
  int i = lin % np, col = lin / np, j = col % nq, k = col / nq;
  double p[3];
  double sq0 = sqrt(cd->B * cd->B + cd->C * cd->C);
  p[0] = atan2(cd->B, -cd->C);
  p[1] = g->n_qpt > 1 ? 2.0 * cd->A : kappa_centre(g, j);
  p[2] = g->n_d0 > 1 ? 2.0 * cd->D / (1.0 + sq0) : d0_centre(g, k);
  int freep[3] = {1, g->n_qpt > 1, g->n_d0 > 1};
  const double prior[3] = {0.01, 1e-4, 100.0};
  const double s2 = (double)sigma * (double)sigma;
  int idx[3], nfree = 0;
  for (int a = 0; a < 3; ++a)
    if (freep[a]) idx[nfree++] = a;
  int status = 0;
  for (int it = 0; it < iters && status == 0; ++it) {
    double P[3][3] = {{0}};
    double dp[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < nfree; ++a) P[a][a] = prior[idx[a]];
    for (int L = 0; L < OR_MAX_LAYERS; ++L) {
      int h = hits[L];
      if (h < 0) continue;
      double rr = (double)r[h], ph = (double)phi[h];
      double kap = p[1], d0 = p[2];
      double den = 1.0 + kap * d0;
      double u = (kap * (rr * rr + d0 * d0) + 2.0 * d0) / (2.0 * rr * den);
      if (!(fabs(u) < 1.0)) { status = 1; break; }
      double sq = sqrt(1.0 - u * u);
      double res = wrap_pi(ph - (p[0] + asin(u)));
      double jac[3];
      jac[0] = 1.0;
      jac[1] = (rr * rr - d0 * d0) / (2.0 * rr * den * den) / sq;
      jac[2] = (den * den + 1.0 - kap * kap * rr * rr) / (2.0 * rr * den * den) / sq;
      double H[3], PH[3];
      for (int a = 0; a < nfree; ++a) H[a] = jac[idx[a]];
      for (int a = 0; a < nfree; ++a) {
        double s = 0.0;
        for (int b = 0; b < nfree; ++b) s += P[a][b] * H[b];
        PH[a] = s;
      }
      double S = s2 / (rr * rr);
      for (int a = 0; a < nfree; ++a) S += H[a] * PH[a];
      if (!(S > 0.0)) { status = 2; break; }
      double K[3];
      double innov = res;
      for (int a = 0; a < nfree; ++a) innov -= H[a] * dp[a];
      for (int a = 0; a < nfree; ++a) K[a] = PH[a] / S;
      for (int a = 0; a < nfree; ++a) dp[a] += K[a] * innov;
      for (int a = 0; a < nfree; ++a)
        for (int b = 0; b < nfree; ++b) P[a][b] -= K[a] * PH[b];
    }
    if (status) break;
    for (int a = 0; a < nfree; ++a) p[idx[a]] += dp[a];
  }
  double chi2 = 0.0;
  if (status == 0) {
    for (int L = 0; L < OR_MAX_LAYERS; ++L) {
      int h = hits[L];
      if (h < 0) continue;
      double rr = (double)r[h], ph = (double)phi[h];
      double kap = p[1], d0 = p[2];
      double den = 1.0 + kap * d0;
      double u = (kap * (rr * rr + d0 * d0) + 2.0 * d0) / (2.0 * rr * den);
      if (!(fabs(u) < 1.0)) { status = 1; break; }
      double res = wrap_pi(ph - (p[0] + asin(u)));
      double z = rr * res / (double)sigma;
      chi2 += z * z;
    }
  }
  double cb = C_LIGHT * (double)g->bfield;
  if (status != 0) {
    p[0] = phi0_centre(g, i);
    p[1] = kappa_centre(g, j);
    p[2] = d0_centre(g, k);
    chi2 = -1.0;
  }
  t->status = status;
  t->phi0 = (float)wrap_pi(p[0]);
  t->qpt = (float)(-p[1] / cb);
  t->d0 = (float)p[2];
  t->chi2 = (float)chi2;
}

/* ------------------------------------------------------------------------ */
/* Second transform (section "Jet and Black Hole Detection"): tracks that
 * share a displaced vertex lie on one sinusoid of the track-parameter space;
 * dually, each track votes for every vertex position it passes through.
 * Reading used: vertex cells (rho_m, theta_t) over [rho_lo, rho_hi) x
 * [-pi, pi); the lower radius bound is the paper's filter of features near
 * the interaction point.  Each track votes once for every cell its seed
 * circle passes through on the outgoing branch between its perigee radius
 * |d0| and the radius of its first owned hit (the vertex cannot lie outside
 * the first hit): in row m the crossing azimuths at the ends of
 * [max(e_m, |d0|), min(e_m+1, r_first)] span an arc of theta bins, all of
 * which get one vote.  With vtx_two_branch the track also votes on its
 * incoming branch, the part of the circle before the perigee that a track
 * sent from its vertex towards the beam line follows (an isotropic decay
 * sends half of its tracks that way): in row m the incoming crossings at the
 * ends of [max(e_m, |d0|), e_m+1] span a second arc, and each cell of the
 * union of the two arcs gets one vote.  A crossing at radius rho solves the circle's line
 * equation B x + C y = -(A rho^2 + D) on the circle of radius rho and takes
 * the point ahead of the perigee along the direction of motion; theta comes
 * from the canonical atan2; float64 arithmetic and square roots only.
 * Vertex peaks use the same local-maximum rule in 2D; members are tracks
 * whose arc comes within one cell of the peak; an object is black-hole-like
 * (section "Physics Motivation": high multiplicity, omnidirectional) when it
 * has at least bh_min_tracks members and the length of the mean member
 * direction (perigee directions) is at most bh_max_isotropy. */
static int theta_bin(double th, int nt) {
  int t = (int)floor((th + OR_PI) / (2.0 * OR_PI / (double)nt));
  return ((t % nt) + nt) % nt;
}

/* branch > 0: the crossing ahead of the perigee along the direction of
 * motion (outgoing branch); branch < 0: the one before it (incoming) */
static double crossing_theta(const cand_t* c, double sn, double rho, int branch) {
  double c0 = -(c->A * rho * rho + c->D);
  double dl = c0 / sn;
  double hh = (rho - dl) * (rho + dl);
  double h = hh > 0.0 ? sqrt(hh) : 0.0;
  if (branch < 0) h = -h;
  double px = (dl / sn) * c->B + (h / sn) * (-c->C);
  double py = (dl / sn) * c->C + (h / sn) * c->B;
  return catan2(py, px);
}

/* the arc of theta bins between the crossings at radii ra < rb of one
 * branch: the shorter way round from the bin of one end to the other */
static void branch_arc(const cand_t* c, double sn, double ra, double rb, int branch, int nt,
                       int32_t* start, int32_t* len) {
  int ta = theta_bin(crossing_theta(c, sn, ra, branch), nt);
  int tb = theta_bin(crossing_theta(c, sn, rb, branch), nt);
  int d = ((tb - ta) % nt + nt) % nt; /* steps from ta to tb going up */
  if (d <= nt / 2) { *start = ta; *len = d + 1; }
  else { *start = tb; *len = nt - d + 1; }
}

static int is_peak2(const int32_t* v, int nm, int nt, int m, int t, int32_t thr) {
  int32_t c = v[m * nt + t];
  if (c < thr) return 0;
  for (int dm = -1; dm <= 1; ++dm) {
    int mm = m + dm;
    if (mm < 0 || mm >= nm) continue;
    for (int dt = -1; dt <= 1; ++dt) {
      if (dm == 0 && dt == 0) continue;
      int tt = ((t + dt) % nt + nt) % nt;
      int32_t w = v[mm * nt + tt];
      int negative = dm < 0 || (dm == 0 && dt < 0);
      if (negative ? !(c > w) : !(c >= w)) return 0;
    }
  }
  return 1;
}

int oracle_vertex_peaks(const int32_t* v, int32_t nm, int32_t nt, int32_t thr, int32_t* out,
                        int32_t capacity, int32_t* n_found) {
  if (!v || nm < 1 || nt < 4 || capacity < 0 || (capacity > 0 && !out) || !n_found) return -1;
  int32_t n = 0;
  for (int m = 0; m < nm; ++m)
    for (int t = 0; t < nt; ++t)
      if (is_peak2(v, nm, nt, m, t, thr)) {
        if (n < capacity) out[n] = m * nt + t;
        ++n;
      }
  *n_found = n;
  return 0;
}

int oracle_assoc_cluster(const or_grid* g, const float* r, const float* phi,
                         const uint8_t* layer, int32_t n_hits, const or_peak* peaks,
                         int32_t n_peaks, const or_cluster_cfg* cfg, int32_t* hit_owner,
                         or_track* tracks, int32_t track_cap, or_object* objects,
                         int32_t object_cap, int32_t* members, int32_t member_cap,
                         int32_t* vacc_out, int32_t* counts) {
  if (!grid_ok(g) || !cfg || n_hits < 0 || n_peaks < 0 || track_cap < 0 || object_cap < 0 ||
      member_cap < 0 || !counts)
    return -1;
  if (cfg->win_bins < 0 || cfg->min_layers < 3 || cfg->min_layers > OR_MAX_LAYERS ||
      cfg->seed_k < 1 || cfg->seed_k > 64 || cfg->member_cap < 1 || !(cfg->road_sigmas > 0.0f) ||
      !(cfg->box_margin >= 0.0f) || cfg->fit_iters < 0 || cfg->n_rho < 1 || cfg->n_theta < 4 ||
      !(cfg->rho_hi > cfg->rho_lo) || !(cfg->rho_lo > 0.0f) || !(cfg->sigma_rphi > 0.0f) ||
      !(cfg->vtx_min_d0 >= 0.0f) || cfg->fit_kind < 0 || cfg->fit_kind > 1 ||
      cfg->vtx_two_branch < 0 || cfg->vtx_two_branch > 1)
    return -1;
  tables tb;
  if (make_tables(g, &tb)) { free_tables(&tb); return -2; }

  /* 0. hit Cartesian coordinates (canonical sincos, float64) */
  hitxy_t hx;
  size_t nh1 = (size_t)(n_hits > 0 ? n_hits : 1);
  hx.x = (double*)malloc(sizeof(double) * nh1);
  hx.y = (double*)malloc(sizeof(double) * nh1);
  hx.q = (double*)malloc(sizeof(double) * nh1);
  for (int32_t h = 0; h < n_hits; ++h) {
    double s, c;
    double rr = (double)r[h];
    csincos(hit_valid(r[h], phi[h]) ? (double)phi[h] : 0.0, &s, &c);
    hx.x[h] = rr * c;
    hx.y[h] = rr * s;
    hx.q[h] = hx.x[h] * hx.x[h] + hx.y[h] * hx.y[h];
  }
  window_t wd;
  double cb = C_LIGHT * (double)g->bfield;
  wd.kbin = cb * ((double)g->qpt_hi - (double)g->qpt_lo) / (double)g->n_qpt;
  wd.dbin = ((double)g->d0_hi - (double)g->d0_lo) / (double)g->n_d0;
  wd.hk = (float)(0.5 * wd.kbin);
  wd.hd0 = (float)(0.5 * wd.dbin);

  /* 1. refinement, per peak */
  cand_t* cd = (cand_t*)malloc(sizeof(cand_t) * (size_t)(n_peaks > 0 ? n_peaks : 1));
#pragma omp parallel
  {
    member_t* mem = (member_t*)malloc(sizeof(member_t) * (size_t)cfg->member_cap);
#pragma omp for schedule(dynamic, 16)
    for (int32_t p = 0; p < n_peaks; ++p)
      refine(g, &tb, &wd, &hx, r, phi, layer, n_hits, peaks[p].lin, cfg, mem, &cd[p]);
    free(mem);
  }

  /* 2. ownership among candidates */
  int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * nh1);
  int32_t n_cand = 0, n_over = 0;
  int64_t n_pairs = 0, n_tests = 0;
  size_t np1 = (size_t)(n_peaks > 0 ? n_peaks : 1);
  int32_t* c_nin = (int32_t*)calloc(np1, sizeof(int32_t));
  float* c_ss = (float*)calloc(np1, sizeof(float));
  int32_t* c_lin = (int32_t*)calloc(np1, sizeof(int32_t));
  int32_t* c_hits = (int32_t*)calloc(np1 * OR_MAX_LAYERS, sizeof(int32_t));
  int32_t* c_own = (int32_t*)calloc(np1, sizeof(int32_t));
  for (int32_t p = 0; p < n_peaks; ++p) {
    n_pairs += cd[p].n_members;
    n_tests += cd[p].n_tests;
    if (cd[p].status == 2) ++n_over;
    if (cd[p].status == 0) ++n_cand;
    c_nin[p] = cd[p].status == 0 ? cd[p].n_inliers : -1;
    c_ss[p] = (float)cd[p].ss;
    c_lin[p] = peaks[p].lin;
    for (int L = 0; L < OR_MAX_LAYERS; ++L) c_hits[(size_t)p * OR_MAX_LAYERS + L] = cd[p].hit[L];
  }
  ownership(n_peaks, c_nin, c_ss, c_lin, c_hits, n_hits, owner, c_own);

  /* 3. survivors in peak order */
  int32_t n_trk = 0;
  int32_t* trk_of_peak = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_peaks > 0 ? n_peaks : 1));
  int32_t* trk_peak = (int32_t*)malloc(sizeof(int32_t) * (size_t)(track_cap > 0 ? track_cap : 1));
  for (int32_t p = 0; p < n_peaks; ++p) {
    trk_of_peak[p] = -1;
    if (cd[p].status != 0) continue;
    int own = c_own[p];
    if (own < cfg->min_layers) continue;
    if (n_trk < track_cap) {
      or_track* t = &tracks[n_trk];
      memset(t, 0, sizeof(*t));
      t->peak = p;
      t->lin = peaks[p].lin;
      t->votes = peaks[p].votes;
      t->n_layers = cd[p].n_layers;
      t->n_inliers = cd[p].n_inliers;
      t->n_owned = own;
      t->seed_ss = (float)cd[p].ss;
      float rf = INFINITY;
      for (int L = 0; L < OR_MAX_LAYERS; ++L) {
        int32_t h = cd[p].hit[L];
        t->hits[L] = (h >= 0 && owner[h] == p) ? h : -1;
        if (t->hits[L] >= 0 && r[h] < rf) rf = r[h];
      }
      t->r_first = rf;
      trk_of_peak[p] = n_trk;
      trk_peak[n_trk] = p;
    }
    ++n_trk;
  }
  int32_t n_stored = n_trk < track_cap ? n_trk : track_cap;
  if (hit_owner)
    for (int32_t h = 0; h < n_hits; ++h) hit_owner[h] = owner[h] >= 0 ? trk_of_peak[owner[h]] : -1;

  /* 4. refit */
#pragma omp parallel for schedule(dynamic, 8)
  for (int32_t t = 0; t < n_stored; ++t) {
    if (cfg->fit_kind == 1)
      kf_track(g, r, phi, tracks[t].hits, tracks[t].lin, &cd[trk_peak[t]], cfg->fit_iters,
               cfg->sigma_rphi, &tracks[t]);
    else
      fit_track(g, r, phi, tracks[t].hits, tracks[t].lin, &cd[trk_peak[t]], cfg->fit_iters,
                cfg->sigma_rphi, &tracks[t]);
  }

  /* 5. vertex transform over the stored tracks */
  const int nm = cfg->n_rho, nt = cfg->n_theta;
  int32_t* vacc = (int32_t*)calloc((size_t)nm * nt, sizeof(int32_t));
  /* per (track, row): first bin of the arc and its length (0 = no vote), on
   * the outgoing branch (tv0, tvn) and the incoming one (ti0, tin) */
  const size_t narc = (size_t)(n_stored > 0 ? n_stored : 1) * nm;
  int32_t* tv0 = (int32_t*)malloc(sizeof(int32_t) * narc);
  int32_t* tvn = (int32_t*)malloc(sizeof(int32_t) * narc);
  int32_t* ti0 = (int32_t*)malloc(sizeof(int32_t) * narc);
  int32_t* tin = (int32_t*)malloc(sizeof(int32_t) * narc);
  const double rw = ((double)cfg->rho_hi - (double)cfg->rho_lo) / (double)nm;
  for (int32_t t = 0; t < n_stored; ++t) {
    const cand_t* c = &cd[trk_peak[t]];
    double sn = sqrt(c->B * c->B + c->C * c->C);
    double pca = fabs(2.0 * c->D / (1.0 + sn));
    double rf = (double)tracks[t].r_first;
    /* a track passing within vtx_min_d0 of the beam line is a feature at
     * the interaction point (the paper's filter near the IP): no votes */
    int votes = !(pca < (double)cfg->vtx_min_d0);
    for (int m = 0; m < nm; ++m) {
      const size_t a = (size_t)t * nm + m;
      tv0[a] = tvn[a] = ti0[a] = tin[a] = 0;
      double e0 = (double)cfg->rho_lo + (double)m * rw;
      double e1 = (double)cfg->rho_lo + (double)(m + 1) * rw;
      double ra = e0 > pca ? e0 : pca;
      if (!votes) continue;
      /* outgoing branch: between the perigee and the first hit */
      double rb = e1 < rf ? e1 : rf;
      if (ra < rb) branch_arc(c, sn, ra, rb, +1, nt, &tv0[a], &tvn[a]);
      /* incoming branch (two-branch vote): the part of the circle before the
       * perigee, which a track leaving its vertex towards the beam line
       * follows; anywhere in the row above the perigee radius */
      if (cfg->vtx_two_branch && ra < e1) branch_arc(c, sn, ra, e1, -1, nt, &ti0[a], &tin[a]);
      /* one vote per cell of the union of the two arcs */
      for (int q = 0; q < tvn[a]; ++q) vacc[m * nt + (tv0[a] + q) % nt] += 1;
      for (int q = 0; q < tin[a]; ++q) {
        int cc = (ti0[a] + q) % nt;
        int off = ((cc - tv0[a]) % nt + nt) % nt;
        if (off >= tvn[a]) vacc[m * nt + cc] += 1;
      }
    }
  }
  if (vacc_out) memcpy(vacc_out, vacc, sizeof(int32_t) * (size_t)nm * nt);

  /* 6. vertex peaks -> objects */
  int32_t n_obj = 0;
  int64_t n_mem = 0;
  for (int m = 0; m < nm; ++m) {
    for (int ti = 0; ti < nt; ++ti) {
      if (!is_peak2(vacc, nm, nt, m, ti, cfg->vtx_min_votes)) continue;
      if (n_obj < object_cap) {
        or_object* o = &objects[n_obj];
        int32_t cntm = 0;
        double sx = 0.0, sy = 0.0;
        o->member_begin = (int32_t)n_mem;
        for (int32_t t = 0; t < n_stored; ++t) {
          int hit = 0;
          for (int dm = -1; dm <= 1 && !hit; ++dm) {
            int mm = m + dm;
            if (mm < 0 || mm >= nm) continue;
            for (int br = 0; br < 2 && !hit; ++br) {
              int len = br ? tin[(size_t)t * nm + mm] : tvn[(size_t)t * nm + mm];
              if (len == 0) continue;
              int st = br ? ti0[(size_t)t * nm + mm] : tv0[(size_t)t * nm + mm];
              /* arc widened by one bin each side contains ti */
              int off = ((ti - st + 1) % nt + nt) % nt;
              if (off < len + 2) hit = 1;
            }
          }
          if (!hit) continue;
          const cand_t* c = &cd[trk_peak[t]];
          double sn = sqrt(c->B * c->B + c->C * c->C);
          sx += -c->C / sn;
          sy += c->B / sn;
          if (n_mem < member_cap) members[n_mem] = t;
          ++n_mem;
          ++cntm;
        }
        double R = cntm > 0 ? sqrt(sx * sx + sy * sy) / (double)cntm : 0.0;
        o->lin = m * nt + ti;
        o->votes = vacc[m * nt + ti];
        o->n_tracks = cntm;
        o->kind = (cntm >= cfg->bh_min_tracks && R <= (double)cfg->bh_max_isotropy) ? 1 : 0;
        o->rho = (float)((double)cfg->rho_lo + ((double)m + 0.5) * rw);
        o->theta = (float)(-OR_PI + ((double)ti + 0.5) * (2.0 * OR_PI / (double)nt));
        o->isotropy = (float)R;
      }
      ++n_obj;
    }
  }
  counts[0] = n_cand;
  counts[1] = n_trk;
  counts[2] = n_obj;
  counts[3] = (int32_t)n_mem;
  counts[4] = n_over;
  counts[5] = (int32_t)(n_pairs > 0x7fffffff ? 0x7fffffff : n_pairs);
  counts[6] = (int32_t)(n_tests > 0x7fffffff ? 0x7fffffff : n_tests);
  counts[7] = 0;

  free(cd);
  free(owner);
  free(c_nin);
  free(c_ss);
  free(c_lin);
  free(c_hits);
  free(c_own);
  free(trk_of_peak);
  free(trk_peak);
  free(vacc);
  free(tv0);
  free(tvn);
  free(ti0);
  free(tin);
  free(hx.x);
  free(hx.y);
  free(hx.q);
  free_tables(&tb);
  return 0;
}

/* One candidate's refinement (diagnostics and tests): out_i32[0..2] =
 * (status, n_layers, n_inliers), out_i32[3..18] = inlier hit per layer,
 * out_f64[0..4] = (ss, A, B, C, D). */
int oracle_refine_one(const or_grid* g, const float* r, const float* phi, const uint8_t* layer,
                      int32_t n_hits, int32_t lin, const or_cluster_cfg* cfg, int32_t* out_i32,
                      double* out_f64) {
  if (!grid_ok(g) || !cfg || cfg->member_cap < 1) return -1;
  tables tb;
  if (make_tables(g, &tb)) { free_tables(&tb); return -2; }
  hitxy_t hx;
  size_t nh1 = (size_t)(n_hits > 0 ? n_hits : 1);
  hx.x = (double*)malloc(sizeof(double) * nh1);
  hx.y = (double*)malloc(sizeof(double) * nh1);
  hx.q = (double*)malloc(sizeof(double) * nh1);
  for (int32_t h = 0; h < n_hits; ++h) {
    double s, c;
    csincos(hit_valid(r[h], phi[h]) ? (double)phi[h] : 0.0, &s, &c);
    hx.x[h] = (double)r[h] * c;
    hx.y[h] = (double)r[h] * s;
    hx.q[h] = hx.x[h] * hx.x[h] + hx.y[h] * hx.y[h];
  }
  window_t wd;
  double cb = C_LIGHT * (double)g->bfield;
  wd.kbin = cb * ((double)g->qpt_hi - (double)g->qpt_lo) / (double)g->n_qpt;
  wd.dbin = ((double)g->d0_hi - (double)g->d0_lo) / (double)g->n_d0;
  wd.hk = (float)(0.5 * wd.kbin);
  wd.hd0 = (float)(0.5 * wd.dbin);
  member_t* mem = (member_t*)malloc(sizeof(member_t) * (size_t)cfg->member_cap);
  cand_t cd;
  refine(g, &tb, &wd, &hx, r, phi, layer, n_hits, lin, cfg, mem, &cd);
  out_i32[0] = cd.status;
  out_i32[1] = cd.n_layers;
  out_i32[2] = cd.n_inliers;
  for (int L = 0; L < OR_MAX_LAYERS; ++L) out_i32[3 + L] = cd.hit[L];
  out_f64[0] = cd.ss;
  out_f64[1] = cd.A; out_f64[2] = cd.B; out_f64[3] = cd.C; out_f64[4] = cd.D;
  free(mem);
  free(hx.x); free(hx.y); free(hx.q);
  free_tables(&tb);
  return 0;
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
