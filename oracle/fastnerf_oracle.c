/*
 * FP64 reference renderer for FastNeRF's cached path -- TEST INFRASTRUCTURE.
 *
 * Plain, slow and single-threaded on purpose: every pixel and every sample is
 * computed from the definition, in double precision, with no tiling, no
 * empty-space skipping and no reordering. It shares no code with the HIP
 * library. Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.
 *
 * Paper passages followed (FastNeRF, Garbin et al. 2021):
 *   ray per pixel from the camera parameters ........ Sec. 3.1, Sec. 4
 *   samples between near and far bounds ............. Sec. 3.1
 *   position cache over k^3, direction cache over
 *     l values of theta in [0,pi] and phi in [0,2pi] . Sec. 3.3
 *   nearest-neighbour position lookup, interpolated
 *     direction lookup ............................. Sec. 4
 *   colour = beta . (u, v, w) ........................ Sec. 3.2, Eq. 5
 *   front-to-back quadrature with transmittance ...... Sec. 3.1, Eq. 1
 *   termination once the remaining contribution falls
 *     to a threshold ............................... supplementary S3
 *
 * Readings where the paper is silent or garbled:
 *   R1 pinhole K, pixel centres at +1/2, OpenCV camera axes (x right, y down,
 *      z forward), unit ray direction so t is a Euclidean distance.
 *   R2 delta_i is printed as a vector difference (Eq. 1): read as the constant
 *      spacing (t1 - t0)/N with midpoints t_i = t0 + (i + 1/2) delta; there is no
 *      special last interval.
 *   R3 "samples within the bounding box": [near,far] intersected with the box.
 *   R4 the direction cache is l x l over (theta, phi); the interpolated lookup
 *      is bilinear over cell centres, periodic in phi, clamped in theta.
 *   R5 theta is measured from +z, phi = atan2(y, x) in [0, 2pi).
 *   R6 position-cache values sit at cell centres; the nearest voxel of g is
 *      the cell that contains it, floor(g) (a point on a face goes to the upper
 *      cell, the far box face to the last cell); outside the box density is 0.
 *   R7 trilinear lookups clamp corner indices to the grid inside the box.
 *   R8 termination: stop before sample i once T_i < eps, i.e. once the
 *      accumulated optical depth exceeds ln(1/eps); the background is then
 *      composited with the remaining transmittance.
 *   R9/R11 RGB includes the background times the final transmittance; A = 1 - T.
 *   R10 no activation is applied to the colour of Eq. 5.
 *   R13 a sample whose grid coordinate lies within gamma (voxels) of a voxel
 *      face may take either neighbour (except one on the face, R6b), and a stop
 *      point within tau_band of ln(1/eps) may be taken or not: all such
 *      variants are admissible results (the FP32 kernel cannot resolve them),
 *      and they are enumerated.
 *   R6b faces hit exactly: when the sample spacing is commensurate with the
 *      grid (k/N voxels per sample along an axis that the ray crosses from
 *      face to face, e.g. k = 768, N = 192) every sample lies on a voxel face.
 *      R6 puts such a point in the upper cell; so that FP64 rounding of the
 *      sample position cannot flip that choice, a grid coordinate within
 *      ORC_ON_FACE (1e-9 voxel, far below any FP32 resolution) of a face counts
 *      as lying on it. Everywhere else the nearest voxel is floor(g).
 *   R17 the transmittance sum of Eq. 1 runs over the samples before i.
 *   R18 voxel traversal (N = 0): the rendering procedure of Sec. 4 visits every
 *      voxel a ray crosses. The ray inside [near, far] intersected with the box
 *      is cut at every crossing of a voxel face; each
 *      piece is one sample, of length delta_i equal to the piece's length and
 *      value that of the nearest voxel of its midpoint (nearest lookups only).
 *      The nearest-lookup field is constant on each piece, so this evaluates
 *      Eq. 1 exactly for the cached field, and the midpoint rule with N
 *      samples converges to it as N grows.
 */
#include "fastnerf_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Rays (Sec. 4; reading R1)                                                 */
/* ------------------------------------------------------------------------- */

static void inverse3(const double *m, double *r) {
  double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5], g = m[6], h = m[7],
         i = m[8];
  double c00 = e * i - f * h, c01 = -(d * i - f * g), c02 = d * h - e * g;
  double det = a * c00 + b * c01 + c * c02;
  r[0] = c00 / det;
  r[1] = -(b * i - c * h) / det;
  r[2] = (b * f - c * e) / det;
  r[3] = c01 / det;
  r[4] = (a * i - c * g) / det;
  r[5] = -(a * f - c * d) / det;
  r[6] = c02 / det;
  r[7] = -(a * h - b * g) / det;
  r[8] = (a * e - b * d) / det;
}

void orc_pixel_ray(const orc_view *v, double x, double y, double o[3], double d[3]) {
  double Ki[9], q[3], w[3];
  inverse3(v->K, Ki);
  double px = x + 0.5, py = y + 0.5;
  for (int r = 0; r < 3; r++) q[r] = Ki[3 * r + 0] * px + Ki[3 * r + 1] * py + Ki[3 * r + 2];
  for (int r = 0; r < 3; r++)
    w[r] = v->c2w[4 * r + 0] * q[0] + v->c2w[4 * r + 1] * q[1] + v->c2w[4 * r + 2] * q[2];
  double n = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  for (int r = 0; r < 3; r++) {
    d[r] = w[r] / n;
    o[r] = v->c2w[4 * r + 3];
  }
}

/* Sample interval (readings R2, R3). Returns 1 when it is non-empty. */
int orc_interval(const orc_scene *s, const orc_view *v, const double o[3], const double d[3],
                 double *t0, double *t1) {
  double a = v->near, b = v->far;
  if (s->in_box) {
    for (int ax = 0; ax < 3; ax++) {
      if (d[ax] == 0.0) {
        if (o[ax] < s->bmin[ax] || o[ax] > s->bmax[ax]) return 0;
      } else {
        double ta = (s->bmin[ax] - o[ax]) / d[ax];
        double tb = (s->bmax[ax] - o[ax]) / d[ax];
        double lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
        if (lo > a) a = lo;
        if (hi < b) b = hi;
      }
    }
  }
  *t0 = a;
  *t1 = b;
  return b > a;
}

/* ------------------------------------------------------------------------- */
/* Position cache (Sec. 3.3, Sec. 4; readings R6, R7)                         */
/* ------------------------------------------------------------------------- */

/* Reads voxel (x, y, z); any negative coordinate means "outside the box". */
static void fetch_voxel(const orc_scene *s, int x, int y, int z, double *sig, double *uu) {
  int n3 = 3 * s->D;
  if (x < 0 || y < 0 || z < 0) {
    *sig = 0.0;
    for (int j = 0; j < n3; j++) uu[j] = 0.0;
    return;
  }
  int64_t k = s->k;
  if (s->sigma) {
    int64_t idx = ((int64_t)z * k + y) * k + x;
    *sig = s->sigma[idx];
    for (int j = 0; j < n3; j++) uu[j] = s->u[idx * n3 + j];
    return;
  }
  int64_t sb = s->sb, nb = k / sb;
  int64_t b = ((int64_t)(z / sb) * nb + y / sb) * nb + x / sb;
  int32_t sl = s->slot[b];
  if (sl < 0) {
    *sig = 0.0;
    for (int j = 0; j < n3; j++) uu[j] = 0.0;
    return;
  }
  int64_t loc = ((int64_t)(z % sb) * sb + y % sb) * sb + x % sb;
  int64_t idx = (int64_t)sl * sb * sb * sb + loc;
  *sig = s->ssigma[idx];
  for (int j = 0; j < n3; j++) uu[j] = s->su[idx * n3 + j];
}

/* Continuous grid coordinate of world position p along one axis: cell i spans
   [i, i+1), its centre is at i + 1/2. */
static double grid_coord(const orc_scene *s, int ax, double p) {
  return (p - s->bmin[ax]) * (double)s->k / (s->bmax[ax] - s->bmin[ax]);
}

/* A grid coordinate this close (in voxels) to a face lies on it (reading R6b):
   FP64 rounding of a sample position is about 1e-12 voxel at k <= 1024. */
#define ORC_ON_FACE 1e-9

/* Nearest voxel along one axis (reading R6: the cell containing g, the upper
   one on a face), -1 outside the box. */
static int nn_coord(double g, int k) {
  if (g < 0.0 || g > (double)k) return -1;
  int c = (int)floor(g + ORC_ON_FACE);
  return c > k - 1 ? k - 1 : c;
}

static void lookup_nn(const orc_scene *s, const double p[3], double *sig, double *uu) {
  int c[3];
  for (int ax = 0; ax < 3; ax++) c[ax] = nn_coord(grid_coord(s, ax, p[ax]), s->k);
  if (c[0] < 0 || c[1] < 0 || c[2] < 0)
    fetch_voxel(s, -1, -1, -1, sig, uu);
  else
    fetch_voxel(s, c[0], c[1], c[2], sig, uu);
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static void lookup_trilinear(const orc_scene *s, const double p[3], double *sig, double *uu) {
  int n3 = 3 * s->D, k = s->k;
  int i0[3];
  double w[3];
  *sig = 0.0;
  for (int j = 0; j < n3; j++) uu[j] = 0.0;
  for (int ax = 0; ax < 3; ax++) {
    double g = grid_coord(s, ax, p[ax]);
    if (g < 0.0 || g > (double)k) return; /* outside the box */
    double gc = g - 0.5;
    double f = floor(gc);
    i0[ax] = (int)f;
    w[ax] = gc - f;
  }
  double cs, cu[3 * 16];
  for (int corner = 0; corner < 8; corner++) {
    int bx = corner & 1, by = (corner >> 1) & 1, bz = (corner >> 2) & 1;
    double wt = (bx ? w[0] : 1.0 - w[0]) * (by ? w[1] : 1.0 - w[1]) * (bz ? w[2] : 1.0 - w[2]);
    fetch_voxel(s, clampi(i0[0] + bx, 0, k - 1), clampi(i0[1] + by, 0, k - 1),
                clampi(i0[2] + bz, 0, k - 1), &cs, cu);
    *sig += wt * cs;
    for (int j = 0; j < n3; j++) uu[j] += wt * cu[j];
  }
}

void orc_lookup_pos(const orc_scene *s, int64_t n, const double *pts, double *sigma_out,
                    double *u_out) {
  int n3 = 3 * s->D;
  for (int64_t i = 0; i < n; i++) {
    if (s->pos_linear)
      lookup_trilinear(s, pts + 3 * i, sigma_out + i, u_out + i * n3);
    else
      lookup_nn(s, pts + 3 * i, sigma_out + i, u_out + i * n3);
  }
}

/* ------------------------------------------------------------------------- */
/* Direction cache (Sec. 3.3, Sec. 4; readings R4, R5)                        */
/* ------------------------------------------------------------------------- */

static void dir_angles(const double d[3], double *th, double *ph) {
  double z = d[2];
  if (z > 1.0) z = 1.0;
  if (z < -1.0) z = -1.0;
  *th = acos(z);
  double p = atan2(d[1], d[0]);
  if (p < 0.0) p += 2.0 * PI;
  *ph = p;
}

static int modl(int m, int l) {
  int r = m % l;
  return r < 0 ? r + l : r;
}

static void beta_cell(const orc_scene *s, int j, int m, double *out) {
  const float *b = s->beta + ((int64_t)j * s->l + m) * s->D;
  for (int c = 0; c < s->D; c++) out[c] = b[c];
}

static void nn_dir_cell(const orc_scene *s, double th, double ph, int *j, int *m) {
  int l = s->l;
  int jj = (int)floor(th * l / PI);
  *j = jj > l - 1 ? l - 1 : jj;
  *m = modl((int)floor(ph * l / (2.0 * PI)), l);
}

static void lookup_dir_cells(const orc_scene *s, const double d[3], int j, int m,
                             double *beta) {
  if (!s->dir_linear) {
    beta_cell(s, j, m, beta);
    return;
  }
  int l = s->l, D = s->D;
  double th, ph;
  dir_angles(d, &th, &ph);
  double gt = th * l / PI - 0.5, gp = ph * l / (2.0 * PI) - 0.5;
  double ft = floor(gt), fp = floor(gp);
  double wt = gt - ft, wp = gp - fp;
  int ja = clampi((int)ft, 0, l - 1), jb = clampi((int)ft + 1, 0, l - 1);
  int ma = modl((int)fp, l), mb = modl((int)fp + 1, l);
  double b00[16], b01[16], b10[16], b11[16];
  beta_cell(s, ja, ma, b00);
  beta_cell(s, ja, mb, b01);
  beta_cell(s, jb, ma, b10);
  beta_cell(s, jb, mb, b11);
  for (int c = 0; c < D; c++)
    beta[c] = (1 - wt) * (1 - wp) * b00[c] + (1 - wt) * wp * b01[c] + wt * (1 - wp) * b10[c] +
              wt * wp * b11[c];
}

void orc_lookup_dir(const orc_scene *s, int64_t n, const double *dirs, double *beta_out) {
  for (int64_t i = 0; i < n; i++) {
    double th, ph;
    int j, m;
    dir_angles(dirs + 3 * i, &th, &ph);
    nn_dir_cell(s, th, ph, &j, &m);
    lookup_dir_cells(s, dirs + 3 * i, j, m, beta_out + i * s->D);
  }
}

/* ------------------------------------------------------------------------- */
/* Per-pixel rendering with admissible variants (Eq. 1, Eq. 5; R8, R13)       */
/* ------------------------------------------------------------------------- */

typedef struct {
  int smp;  /* sample index, -1 for a direction-cell choice */
  int axis; /* 0..2 position axes, 3 theta row, 4 phi column */
  int alt;  /* alternative coordinate */
} choice_t;

typedef struct {
  int n;       /* samples */
  int cap;
  int (*c)[3]; /* primary voxel coordinates per sample */
  double (*p)[3];
  double *t;
  double *dl;  /* per-sample length (voxel traversal); unused with N samples */
  int var_dl;  /* 1: use dl[i], 0: the constant spacing */
} ray_work;

static int work_reserve(ray_work *w, int n) {
  if (n <= w->cap) return 0;
  free(w->c);
  free(w->p);
  free(w->t);
  free(w->dl);
  w->c = malloc(sizeof(int[3]) * (size_t)n);
  w->p = malloc(sizeof(double[3]) * (size_t)n);
  w->t = malloc(sizeof(double) * (size_t)n);
  w->dl = malloc(sizeof(double) * (size_t)n);
  if (!w->c || !w->p || !w->t || !w->dl) return -1;
  w->cap = n;
  return 0;
}

static void work_free(ray_work *w) {
  free(w->c);
  free(w->p);
  free(w->t);
  free(w->dl);
}

/* Alternative nearest-voxel coordinate across the nearest voxel face (or box
   face), if the grid coordinate is within gamma voxels of it but not on it
   (reading R13; a point on an interior face takes the upper cell, R6b). */
static int nn_alternative(double g, int k, double gamma, int prim, int *alt) {
  if (fabs(g) < gamma) { /* lower box face */
    *alt = prim == -1 ? 0 : -1;
    return 1;
  }
  if (fabs(g - k) < gamma) { /* upper box face */
    *alt = prim == -1 ? k - 1 : -1;
    return 1;
  }
  double n = floor(g + 0.5);
  if (n < 1.0 || n > (double)(k - 1) || fabs(g - n) >= gamma || fabs(g - n) <= ORC_ON_FACE ||
      prim < 0)
    return 0;
  *alt = prim == (int)n ? (int)n - 1 : (int)n;
  return *alt != prim;
}

static int records_differ(const orc_scene *s, const int a[3], const int b[3]) {
  double sa, sb2, ua[48], ub[48];
  int outa = a[0] < 0 || a[1] < 0 || a[2] < 0, outb = b[0] < 0 || b[1] < 0 || b[2] < 0;
  if (outa) fetch_voxel(s, -1, -1, -1, &sa, ua); else fetch_voxel(s, a[0], a[1], a[2], &sa, ua);
  if (outb) fetch_voxel(s, -1, -1, -1, &sb2, ub); else fetch_voxel(s, b[0], b[1], b[2], &sb2, ub);
  if (sa == 0.0 && sb2 == 0.0) return 0; /* neither contributes anything */
  if (sa != sb2) return 1;
  for (int j = 0; j < 3 * s->D; j++)
    if (ua[j] != ub[j]) return 1;
  return 0;
}

static int brick_occupied(const orc_scene *s, int x, int y, int z) {
  int nb = (s->k + s->ob - 1) / s->ob;
  return s->occ[((int64_t)(z / s->ob) * nb + y / s->ob) * nb + x / s->ob] != 0;
}

/* Does sample i need cache data under the brick occupancy? (for the byte count) */
static int sample_occupied(const orc_scene *s, const int c[3], const double p[3]) {
  if (!s->occ || s->ob <= 0) return 0;
  if (!s->pos_linear) {
    if (c[0] < 0 || c[1] < 0 || c[2] < 0) return 0;
    return brick_occupied(s, c[0], c[1], c[2]);
  }
  int k = s->k, i0[3];
  for (int ax = 0; ax < 3; ax++) {
    double g = grid_coord(s, ax, p[ax]);
    if (g < 0.0 || g > (double)k) return 0;
    i0[ax] = (int)floor(g - 0.5);
  }
  for (int corner = 0; corner < 8; corner++)
    if (brick_occupied(s, clampi(i0[0] + (corner & 1), 0, k - 1),
                       clampi(i0[1] + ((corner >> 1) & 1), 0, k - 1),
                       clampi(i0[2] + ((corner >> 2) & 1), 0, k - 1)))
      return 1;
  return 0;
}

static void sample_value(const orc_scene *s, const int c[3], const double p[3], double *sig,
                         double *uu) {
  if (s->pos_linear)
    lookup_trilinear(s, p, sig, uu);
  else if (c[0] < 0 || c[1] < 0 || c[2] < 0)
    fetch_voxel(s, -1, -1, -1, sig, uu);
  else
    fetch_voxel(s, c[0], c[1], c[2], sig, uu);
}

typedef struct {
  double rgba[ORC_MAXCAND][4];
  int n;
  int overflow;
} cand_list;

static void cand_push(cand_list *cl, const double C[3], double tau, const double bg[3]) {
  if (cl->n >= ORC_MAXCAND) {
    cl->overflow = 1;
    return;
  }
  double T = exp(-tau);
  for (int c = 0; c < 3; c++) cl->rgba[cl->n][c] = C[c] + T * bg[c];
  cl->rgba[cl->n][3] = -expm1(-tau);
  cl->n++;
}

/* Front-to-back quadrature of one variant (Eq. 1 with the colour of Eq. 5).
   Pushes every admissible stop point; writes the primary one to prim. */
static void composite(const orc_scene *s, const orc_view *v, const orc_tol *tol,
                      const ray_work *w, const double *beta, double delta, cand_list *cl,
                      double prim[4], orc_counts *cnt) {
  int D = s->D;
  double C[3] = {0, 0, 0}, tau = 0.0;
  double lim = v->eps > 0.0 ? log(1.0 / v->eps) : INFINITY;
  double band = tol ? tol->tau_band : 0.0;
  int primary_done = 0;
  int changed = 1; /* (C, tau) moved since the last admissible stop was recorded */
  double uu[48];
  for (int i = 0; i < w->n; i++) {
    /* stopping before an empty sample gives the same result as stopping after
       it, so only distinct stop points are recorded */
    if (tau > lim - band && changed) {
      cand_push(cl, C, tau, s->bg);
      changed = 0;
    }
    if (!primary_done && tau > lim) {
      double T = exp(-tau);
      for (int c = 0; c < 3; c++) prim[c] = C[c] + T * s->bg[c];
      prim[3] = -expm1(-tau);
      primary_done = 1;
    }
    if (tau > lim + band) return;
    double sig;
    sample_value(s, w->c[i], w->p[i], &sig, uu);
    if (cnt && !primary_done) {
      int inside = 1;
      for (int ax = 0; ax < 3; ax++) {
        double g = grid_coord(s, ax, w->p[i][ax]);
        if (g < 0.0 || g > (double)s->k) inside = 0;
      }
      cnt->samples += inside;
      cnt->occ_samples += sample_occupied(s, w->c[i], w->p[i]);
      cnt->nonzero_samples += sig > 0.0;
    }
    double col[3];
    for (int c = 0; c < 3; c++) {
      double acc = 0.0;
      for (int d = 0; d < D; d++) acc += beta[d] * uu[3 * d + c];
      col[c] = acc;
    }
    double dli = w->var_dl ? w->dl[i] : delta;
    double alpha = -expm1(-sig * dli);
    double T = exp(-tau);
    for (int c = 0; c < 3; c++) C[c] += T * alpha * col[c];
    tau += sig * dli;
    if (sig != 0.0) changed = 1;
  }
  if (changed) cand_push(cl, C, tau, s->bg);
  if (!primary_done) {
    double T = exp(-tau);
    for (int c = 0; c < 3; c++) prim[c] = C[c] + T * s->bg[c];
    prim[3] = -expm1(-tau);
  }
}

/* Places the samples of one ray (R2) and their nearest voxels; collects the
   admissible alternative lookups (R13). Returns the number of choices found
   (possibly more than were stored). */
static int place_samples(const orc_scene *s, const orc_view *v, const orc_tol *tol,
                         const double o[3], const double d[3], double t0, double delta,
                         ray_work *w, choice_t *ch) {
  int k = s->k, nch = 0;
  w->n = v->N;
  for (int i = 0; i < v->N; i++) {
    double t = t0 + (i + 0.5) * delta;
    w->t[i] = t;
    double g[3];
    for (int ax = 0; ax < 3; ax++) {
      w->p[i][ax] = o[ax] + t * d[ax];
      g[ax] = grid_coord(s, ax, w->p[i][ax]);
      w->c[i][ax] = nn_coord(g[ax], k);
    }
    if (s->pos_linear || !tol || tol->gamma <= 0.0) continue;
    int amb = 0, alts[3], has[3];
    for (int ax = 0; ax < 3; ax++) {
      has[ax] = nn_alternative(g[ax], k, tol->gamma, w->c[i][ax], &alts[ax]);
      amb += has[ax];
    }
    for (int ax = 0; ax < 3; ax++) {
      if (!has[ax]) continue;
      int alt[3] = {w->c[i][0], w->c[i][1], w->c[i][2]};
      alt[ax] = alts[ax];
      if (amb > 1 || records_differ(s, w->c[i], alt)) {
        if (nch < ORC_MAXCHOICE_LIMIT + 1) ch[nch] = (choice_t){i, ax, alts[ax]};
        nch++;
      }
    }
  }
  return nch;
}

static int cmp_double(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return x < y ? -1 : (x > y);
}

/* Voxel traversal (R18): cuts [t0, t1] at every crossing of an interior voxel
   face (grid coordinate i) and makes each piece of positive
   length a sample at its midpoint, with the nearest voxel of the midpoint and
   the piece's length. ts holds 3(k+1)+2 doubles. */
static void place_segments(const orc_scene *s, const double o[3], const double d[3], double t0,
                           double t1, double *ts, ray_work *w) {
  int k = s->k, n = 0;
  ts[n++] = t0;
  for (int ax = 0; ax < 3; ax++) {
    if (d[ax] == 0.0) continue;
    double h = (s->bmax[ax] - s->bmin[ax]) / k;
    for (int i = 1; i < k; i++) {
      double t = (s->bmin[ax] + i * h - o[ax]) / d[ax];
      if (t > t0 && t < t1) ts[n++] = t;
    }
  }
  ts[n++] = t1;
  qsort(ts, (size_t)n, sizeof(double), cmp_double);
  w->n = 0;
  w->var_dl = 1;
  for (int q = 0; q + 1 < n; q++) {
    double a = ts[q], b = ts[q + 1];
    if (!(b > a)) continue;
    double mid = 0.5 * (a + b);
    int i = w->n;
    w->t[i] = mid;
    w->dl[i] = b - a;
    for (int ax = 0; ax < 3; ax++) {
      w->p[i][ax] = o[ax] + mid * d[ax];
      w->c[i][ax] = nn_coord(grid_coord(s, ax, w->p[i][ax]), k);
    }
    w->n++;
  }
}

static int dir_choices(const orc_scene *s, const orc_tol *tol, double th, double ph, int j,
                       int m, choice_t *ch, int nch) {
  if (s->dir_linear || !tol || tol->gamma_dir <= 0.0) return nch;
  int l = s->l;
  double gt = th * l / PI, nt = floor(gt + 0.5);
  if (nt >= 1.0 && nt <= l - 1 && fabs(gt - nt) * (PI / l) < tol->gamma_dir) {
    int below = (int)nt - 1, above = (int)nt;
    int alt = j == below ? above : below;
    if (alt != j) {
      if (nch < ORC_MAXCHOICE_LIMIT + 1) ch[nch] = (choice_t){-1, 3, alt};
      nch++;
    }
  }
  double gp = ph * l / (2.0 * PI), np_ = floor(gp + 0.5);
  if (fabs(gp - np_) * (2.0 * PI / l) < tol->gamma_dir) {
    int below = modl((int)np_ - 1, l), above = modl((int)np_, l);
    int alt = m == below ? above : below;
    if (alt != m) {
      if (nch < ORC_MAXCHOICE_LIMIT + 1) ch[nch] = (choice_t){-1, 4, alt};
      nch++;
    }
  }
  return nch;
}

/* Enclosure of every admissible result of a pixel (reading R13) without
   enumerating them: per sample the interval of density and of each colour
   channel over its candidate voxels (both sides of every face within gamma)
   and candidate direction cells; then, from the last sample to the first,
   V_i = a_i c_i + (1 - a_i) V_{i+1} (V = the background past the stop) and
   W_i = a_i + (1 - a_i) W_{i+1} (W = 0 past the stop), so RGB = V_0 and
   A = W_0. V_i is bilinear in (a, c, V_{i+1}) with a, 1 - a >= 0, so its bounds
   are at c and V_{i+1} at their own bounds and a at an end of its interval.
   A stop before sample i is possible once the largest optical depth before it
   exceeds ln(1/eps) - tau_band and certain once the smallest exceeds
   ln(1/eps) + tau_band; where possible the bounds take in the background. */
static void enclose(const orc_scene *s, const orc_view *v, const orc_tol *tol,
                    const ray_work *w, const double d[3], double th, double ph, int j0, int m0,
                    double delta, double lo[4], double hi[4]) {
  int D = s->D, k = s->k, n = w->n;
  double gamma = tol ? tol->gamma : 0.0, band = tol ? tol->tau_band : 0.0;
  double lim = v->eps > 0.0 ? log(1.0 / v->eps) : INFINITY;
  /* candidate direction weights */
  double betas[4][16];
  int nb = 0;
  if (s->dir_linear) {
    lookup_dir_cells(s, d, j0, m0, betas[0]);
    nb = 1;
  } else {
    choice_t chd[ORC_MAXCHOICE_LIMIT + 1];
    int nd = dir_choices(s, tol, th, ph, j0, m0, chd, 0);
    int js[2] = {j0, j0}, ms[2] = {m0, m0}, njs = 1, nms = 1;
    for (int q = 0; q < nd && q < 2; q++) {
      if (chd[q].axis == 3) js[njs++] = chd[q].alt;
      else ms[nms++] = chd[q].alt;
    }
    for (int a = 0; a < njs; a++)
      for (int b = 0; b < nms; b++) lookup_dir_cells(s, d, js[a], ms[b], betas[nb++]);
  }
  double *slo = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 8);
  if (!slo) {
    for (int c = 0; c < 4; c++) {
      lo[c] = -INFINITY;
      hi[c] = INFINITY;
    }
    return;
  }
  double *shi = slo + n, *clo = slo + 2 * n, *chi = slo + 5 * n;
  for (int i = 0; i < n; i++) {
    int cand[3][2], nc[3];
    for (int ax = 0; ax < 3; ax++) {
      cand[ax][0] = w->c[i][ax];
      nc[ax] = 1;
      int alt;
      if (!s->pos_linear && gamma > 0.0 &&
          nn_alternative(grid_coord(s, ax, w->p[i][ax]), k, gamma, w->c[i][ax], &alt))
        cand[ax][nc[ax]++] = alt;
    }
    slo[i] = INFINITY;
    shi[i] = -INFINITY;
    for (int c = 0; c < 3; c++) {
      clo[3 * i + c] = INFINITY;
      chi[3 * i + c] = -INFINITY;
    }
    for (int a = 0; a < nc[0]; a++)
      for (int b = 0; b < nc[1]; b++)
        for (int e = 0; e < nc[2]; e++) {
          int cc[3] = {cand[0][a], cand[1][b], cand[2][e]};
          double sig, uu[48];
          if (s->pos_linear)
            lookup_trilinear(s, w->p[i], &sig, uu);
          else if (cc[0] < 0 || cc[1] < 0 || cc[2] < 0)
            fetch_voxel(s, -1, -1, -1, &sig, uu);
          else
            fetch_voxel(s, cc[0], cc[1], cc[2], &sig, uu);
          if (sig < slo[i]) slo[i] = sig;
          if (sig > shi[i]) shi[i] = sig;
          for (int q = 0; q < nb; q++)
            for (int c = 0; c < 3; c++) {
              double acc = 0.0;
              for (int dd = 0; dd < D; dd++) acc += betas[q][dd] * uu[3 * dd + c];
              if (acc < clo[3 * i + c]) clo[3 * i + c] = acc;
              if (acc > chi[3 * i + c]) chi[3 * i + c] = acc;
            }
        }
  }
  /* optical depth before each sample: smallest and largest */
  double *tlo = malloc(sizeof(double) * (size_t)(n + 1) * 2);
  if (!tlo) {
    free(slo);
    for (int c = 0; c < 4; c++) {
      lo[c] = -INFINITY;
      hi[c] = INFINITY;
    }
    return;
  }
  double *thi = tlo + n + 1;
  tlo[0] = thi[0] = 0.0;
  for (int i = 0; i < n; i++) {
    double dl = w->var_dl ? w->dl[i] : delta;
    tlo[i + 1] = tlo[i] + slo[i] * dl;
    thi[i + 1] = thi[i] + shi[i] * dl;
  }
  double Vlo[3], Vhi[3], Wlo = 0.0, Whi = 0.0;
  for (int c = 0; c < 3; c++) Vlo[c] = Vhi[c] = s->bg[c];
  for (int i = n - 1; i >= 0; i--) {
    if (tlo[i] > lim + band) { /* stopped before sample i in every variant */
      for (int c = 0; c < 3; c++) Vlo[c] = Vhi[c] = s->bg[c];
      Wlo = Whi = 0.0;
      continue;
    }
    double dl = w->var_dl ? w->dl[i] : delta;
    double al = -expm1(-slo[i] * dl), ah = -expm1(-shi[i] * dl);
    for (int c = 0; c < 3; c++) {
      double l1 = al * clo[3 * i + c] + (1.0 - al) * Vlo[c];
      double l2 = ah * clo[3 * i + c] + (1.0 - ah) * Vlo[c];
      double h1 = al * chi[3 * i + c] + (1.0 - al) * Vhi[c];
      double h2 = ah * chi[3 * i + c] + (1.0 - ah) * Vhi[c];
      Vlo[c] = l1 < l2 ? l1 : l2;
      Vhi[c] = h1 > h2 ? h1 : h2;
    }
    double wl1 = al + (1.0 - al) * Wlo, wl2 = ah + (1.0 - ah) * Wlo;
    double wh1 = al + (1.0 - al) * Whi, wh2 = ah + (1.0 - ah) * Whi;
    Wlo = wl1 < wl2 ? wl1 : wl2;
    Whi = wh1 > wh2 ? wh1 : wh2;
    if (thi[i] > lim - band) { /* a stop before sample i is possible */
      for (int c = 0; c < 3; c++) {
        if (s->bg[c] < Vlo[c]) Vlo[c] = s->bg[c];
        if (s->bg[c] > Vhi[c]) Vhi[c] = s->bg[c];
      }
      if (0.0 < Wlo) Wlo = 0.0;
    }
  }
  for (int c = 0; c < 3; c++) {
    lo[c] = Vlo[c];
    hi[c] = Vhi[c];
  }
  lo[3] = Wlo;
  hi[3] = Whi;
  free(slo);
  free(tlo);
}

static void render_pixel(const orc_scene *s, const orc_view *v, const orc_tol *tol, int x,
                         int y, ray_work *w, double *ts, double rgba[4], cand_list *cl,
                         int32_t *flag, double env[8], orc_counts *cnt) {
  double o[3], d[3], t0, t1;
  int maxch = !tol || tol->max_choice == 0 ? ORC_MAXCHOICE
                                            : (tol->max_choice < 0 ? 0 : tol->max_choice);
  if (maxch > ORC_MAXCHOICE_LIMIT) maxch = ORC_MAXCHOICE_LIMIT;
  cl->n = 0;
  cl->overflow = 0;
  *flag = 0;
  orc_pixel_ray(v, x, y, o, d);
  if (cnt) cnt->rays++;
  orc_scene clipped = *s; /* voxel traversal always stays inside the box (R18) */
  clipped.in_box = 1;
  if (!orc_interval(v->N == 0 ? &clipped : s, v, o, d, &t0, &t1)) {
    for (int c = 0; c < 3; c++) rgba[c] = s->bg[c];
    rgba[3] = 0.0;
    cand_push(cl, (double[3]){0, 0, 0}, 0.0, s->bg);
    if (env)
      for (int c = 0; c < 4; c++) env[c] = env[4 + c] = rgba[c];
    return;
  }
  *flag |= ORC_HIT;
  if (cnt) cnt->hit++;
  double delta = 0.0;
  choice_t ch[ORC_MAXCHOICE_LIMIT + 1];
  int nch = 0;
  if (v->N == 0) {
    place_segments(s, o, d, t0, t1, ts, w);
  } else {
    delta = (t1 - t0) / v->N;
    w->var_dl = 0;
    nch = place_samples(s, v, tol, o, d, t0, delta, w, ch);
  }
  double th, ph;
  int j0, m0;
  dir_angles(d, &th, &ph);
  nn_dir_cell(s, th, ph, &j0, &m0);
  nch = dir_choices(s, tol, th, ph, j0, m0, ch, nch);
  if (nch > maxch) {
    *flag |= ORC_UNCHECKED;
    nch = 0;
  }
  double beta[16];
  for (int var = 0; var < (1 << nch); var++) {
    int j = j0, m = m0;
    int saved[ORC_MAXCHOICE_LIMIT];
    for (int q = 0; q < nch; q++) {
      if (!(var >> q & 1)) continue;
      if (ch[q].smp >= 0) {
        saved[q] = w->c[ch[q].smp][ch[q].axis];
        w->c[ch[q].smp][ch[q].axis] = ch[q].alt;
      } else if (ch[q].axis == 3) {
        j = ch[q].alt;
      } else {
        m = ch[q].alt;
      }
    }
    lookup_dir_cells(s, d, j, m, beta);
    double prim[4];
    composite(s, v, tol, w, beta, delta, cl, prim, var == 0 ? cnt : NULL);
    if (var == 0)
      for (int c = 0; c < 4; c++) rgba[c] = prim[c];
    for (int q = nch - 1; q >= 0; q--)
      if ((var >> q & 1) && ch[q].smp >= 0) w->c[ch[q].smp][ch[q].axis] = saved[q];
  }
  if (cl->overflow) *flag |= ORC_UNCHECKED;
  if (nch > 0 || cl->n > 1) *flag |= ORC_AMBIG;
  if (!env) return;
  if (*flag & ORC_UNCHECKED) {
    enclose(s, v, tol, w, d, th, ph, j0, m0, delta, env, env + 4);
  } else {
    for (int c = 0; c < 4; c++) {
      env[c] = INFINITY;
      env[4 + c] = -INFINITY;
    }
    for (int q = 0; q < cl->n; q++)
      for (int c = 0; c < 4; c++) {
        if (cl->rgba[q][c] < env[c]) env[c] = cl->rgba[q][c];
        if (cl->rgba[q][c] > env[4 + c]) env[4 + c] = cl->rgba[q][c];
      }
  }
}

int orc_render(const orc_scene *s, const orc_view *v, const orc_tol *tol, int64_t npix,
               const int64_t *pix, double *rgba, double *cand, int32_t *ncand,
               int32_t *flags, double *env, orc_counts *counts) {
  if (!s || !v || !rgba || s->k <= 0 || s->D <= 0 || s->D > 16 || s->l <= 0 || v->N < 0 ||
      (v->N == 0 && s->pos_linear) || v->H <= 0 || v->W <= 0 || !s->beta ||
      (!s->sigma && (!s->slot || s->sb <= 0)))
    return -1;
  if (counts) memset(counts, 0, sizeof *counts);
  ray_work w = {0};
  int nseg = 3 * (s->k + 1) + 2;
  if (work_reserve(&w, v->N > nseg ? v->N : nseg)) return -1;
  double *ts = malloc(sizeof(double) * (size_t)nseg);
  cand_list *cl = malloc(sizeof *cl);
  if (!cl || !ts) {
    free(cl);
    free(ts);
    work_free(&w);
    return -1;
  }
  int64_t total = (int64_t)v->H * v->W;
  for (int64_t q = 0; q < npix; q++) {
    int64_t id = pix ? pix[q] : q;
    if (id < 0 || id >= total) {
      free(cl);
      free(ts);
      work_free(&w);
      return -1;
    }
    int x = (int)(id % v->W), y = (int)(id / v->W);
    int32_t f;
    render_pixel(s, v, tol, x, y, &w, ts, rgba + 4 * q, cl, &f, env ? env + 8 * q : NULL,
                 counts);
    if (flags) flags[q] = f;
    if (counts) {
      counts->ambiguous_pixels += (f & ORC_AMBIG) != 0;
      counts->unchecked_pixels += (f & ORC_UNCHECKED) != 0;
    }
    if (cand) {
      for (int c = 0; c < cl->n; c++)
        for (int j = 0; j < 4; j++) cand[(q * ORC_MAXCAND + c) * 4 + j] = cl->rgba[c][j];
    }
    if (ncand) ncand[q] = cl->n;
  }
  free(cl);
  free(ts);
  work_free(&w);
  return 0;
}

/* The same render split into contiguous bands of the pixel list (row bands
   when the list is in row order), one thread per band. Pixels are independent,
   so the result is bitwise that of orc_render; the counts are summed. */
typedef struct {
  const orc_scene *s;
  const orc_view *v;
  const orc_tol *tol;
  int64_t n;
  int64_t *pix; /* the band's pixel ids */
  double *rgba, *cand, *env;
  int32_t *ncand, *flags;
  orc_counts counts;
  int rc;
} orc_band;

static void *band_main(void *arg) {
  orc_band *b = arg;
  b->rc = orc_render(b->s, b->v, b->tol, b->n, b->pix, b->rgba, b->cand, b->ncand, b->flags,
                     b->env, &b->counts);
  return NULL;
}

int orc_render_mt(const orc_scene *s, const orc_view *v, const orc_tol *tol, int64_t npix,
                  const int64_t *pix, double *rgba, double *cand, int32_t *ncand,
                  int32_t *flags, double *env, orc_counts *counts, int32_t nthreads) {
  if (nthreads < 1 || npix < 0 || !v) return -1;
  if ((int64_t)nthreads > npix) nthreads = npix > 0 ? (int32_t)npix : 1;
  orc_band *bands = calloc((size_t)nthreads, sizeof *bands);
  pthread_t *th = calloc((size_t)nthreads, sizeof *th);
  int64_t *ids = malloc(sizeof(int64_t) * (size_t)(npix > 0 ? npix : 1));
  int rc = 0;
  if (!bands || !th || !ids) {
    free(bands);
    free(th);
    free(ids);
    return -1;
  }
  for (int64_t q = 0; q < npix; q++) ids[q] = pix ? pix[q] : q;
  int started = 0;
  for (int b = 0; b < nthreads; b++) {
    int64_t lo = npix * b / nthreads, hi = npix * (b + 1) / nthreads;
    orc_band *B = &bands[b];
    B->s = s;
    B->v = v;
    B->tol = tol;
    B->n = hi - lo;
    B->pix = ids + lo;
    B->rgba = rgba ? rgba + 4 * lo : NULL;
    B->cand = cand ? cand + lo * ORC_MAXCAND * 4 : NULL;
    B->ncand = ncand ? ncand + lo : NULL;
    B->flags = flags ? flags + lo : NULL;
    B->env = env ? env + 8 * lo : NULL;
    if (pthread_create(&th[b], NULL, band_main, B) != 0) {
      rc = -1;
      break;
    }
    started++;
  }
  for (int b = 0; b < started; b++) pthread_join(th[b], NULL);
  if (counts) memset(counts, 0, sizeof *counts);
  for (int b = 0; b < started; b++) {
    if (bands[b].rc != 0) rc = -1;
    if (counts) {
      counts->rays += bands[b].counts.rays;
      counts->hit += bands[b].counts.hit;
      counts->samples += bands[b].counts.samples;
      counts->occ_samples += bands[b].counts.occ_samples;
      counts->nonzero_samples += bands[b].counts.nonzero_samples;
      counts->ambiguous_pixels += bands[b].counts.ambiguous_pixels;
      counts->unchecked_pixels += bands[b].counts.unchecked_pixels;
    }
  }
  free(bands);
  free(th);
  free(ids);
  return rc;
}

int orc_trace(const orc_scene *s, const orc_view *v, int32_t x, int32_t y, double *t,
              double *sigma, double *rgb, double *delta) {
  double o[3], d[3], t0, t1;
  if (v->N <= 0) return -1;
  orc_pixel_ray(v, x, y, o, d);
  if (!orc_interval(s, v, o, d, &t0, &t1)) return 0;
  ray_work w = {0};
  if (work_reserve(&w, v->N)) return -1;
  double dl = (t1 - t0) / v->N;
  place_samples(s, v, NULL, o, d, t0, dl, &w, NULL);
  double beta[16], uu[48];
  orc_lookup_dir(s, 1, d, beta);
  for (int i = 0; i < v->N; i++) {
    t[i] = w.t[i];
    sample_value(s, w.c[i], w.p[i], sigma + i, uu);
    for (int c = 0; c < 3; c++) {
      double acc = 0.0;
      for (int dd = 0; dd < s->D; dd++) acc += beta[dd] * uu[3 * dd + c];
      rgb[3 * i + c] = acc;
    }
  }
  *delta = dl;
  work_free(&w);
  return v->N;
}

void orc_occupancy(const orc_scene *s, int32_t ob, uint8_t *occ) {
  int k = s->k, nb = (k + ob - 1) / ob;
  double sig, uu[48];
  memset(occ, 0, (size_t)nb * nb * nb);
  for (int z = 0; z < k; z++)
    for (int y = 0; y < k; y++)
      for (int x = 0; x < k; x++) {
        int64_t b = ((int64_t)(z / ob) * nb + y / ob) * nb + x / ob;
        if (occ[b]) continue;
        if (!s->sigma && s->slot[((int64_t)(z / s->sb) * (k / s->sb) + y / s->sb) * (k / s->sb) +
                                 x / s->sb] < 0)
          continue;
        fetch_voxel(s, x, y, z, &sig, uu);
        if (sig > 0.0) occ[b] = 1;
      }
}

/* ------------------------------------------------------------------------- */
/* Storage formats (reading R12): IEEE-754 binary16 and bfloat16, OCP E4M3    */
/* ------------------------------------------------------------------------- */

double orc_round_to(int32_t fmt, double x) {
  int p, emin;
  double maxv;
  switch (fmt) {
    case 1: p = 11; emin = -14; maxv = 65504.0; break;
    case 2: p = 8; emin = -126; maxv = ldexp(2.0 - ldexp(1.0, -7), 127); break;
    case 3: p = 4; emin = -6; maxv = 448.0; break;
    default: return x;
  }
  if (fmt == 3 && isinf(x)) return x < 0 ? -maxv : maxv; /* saturating */
  if (x == 0.0 || !isfinite(x)) return x;
  double a = fabs(x);
  int e;
  frexp(a, &e);
  e -= 1; /* a = m 2^e with m in [1,2) */
  if (e < emin) e = emin;
  double quantum = ldexp(1.0, e - (p - 1));
  double r = rint(a / quantum) * quantum; /* nearest, ties to even */
  if (r > maxv) r = fmt == 3 ? maxv : INFINITY;
  return x < 0 ? -r : r;
}

double orc_e4m3_decode(uint32_t code) {
  int sgn = (code >> 7) & 1, e = (code >> 3) & 15, m = code & 7;
  double v;
  if (e == 15 && m == 7) return NAN;
  if (e == 0)
    v = ldexp((double)m, -9);
  else
    v = ldexp(1.0 + m / 8.0, e - 7);
  return sgn ? -v : v;
}

uint32_t orc_e4m3_encode(float y) {
  uint32_t sgn = signbit(y) ? 0x80u : 0u;
  if (isnan(y)) return sgn | 0x7Fu;
  double a = fabs(orc_round_to(3, (double)y));
  if (a == 0.0) return sgn;
  int e;
  frexp(a, &e);
  e -= 1;
  if (e < -6) return sgn | (uint32_t)(a / ldexp(1.0, -9)); /* subnormal */
  uint32_t mant = (uint32_t)((a / ldexp(1.0, e) - 1.0) * 8.0);
  return sgn | (uint32_t)(e + 7) << 3 | mant;
}

void orc_dequant_cache(int32_t fmt, int64_t nvox, int32_t D, const float *sigma, const float *u,
                       float *sigma_q, float *u_q, float *scales) {
  int n3 = 3 * D;
  if (fmt == 0 || fmt == 1 || fmt == 2) {
    for (int64_t i = 0; i < nvox; i++) sigma_q[i] = (float)orc_round_to(fmt, sigma[i]);
    for (int64_t i = 0; i < nvox * n3; i++) u_q[i] = (float)orc_round_to(fmt, u[i]);
    if (scales)
      for (int c = 0; c <= n3; c++) scales[c] = 1.0f;
    return;
  }
  /* E4M3 with one absmax scale per channel: channel 0 is sigma, 1 + j is u[.][j]. */
  float sc[1 + 48];
  for (int c = 0; c <= n3; c++) {
    float amax = 0.0f;
    for (int64_t i = 0; i < nvox; i++) {
      float xv = c == 0 ? sigma[i] : u[i * n3 + (c - 1)];
      float ax = fabsf(xv);
      if (ax > amax) amax = ax;
    }
    sc[c] = amax > 0.0f ? amax / 448.0f : 1.0f;
    if (scales) scales[c] = sc[c];
  }
  for (int64_t i = 0; i < nvox; i++) {
    float yv = sigma[i] / sc[0];
    sigma_q[i] = (float)orc_e4m3_decode(orc_e4m3_encode(yv)) * sc[0];
    for (int j = 0; j < n3; j++) {
      float yu = u[i * n3 + j] / sc[1 + j];
      u_q[i * n3 + j] = (float)orc_e4m3_decode(orc_e4m3_encode(yu)) * sc[1 + j];
    }
  }
}
