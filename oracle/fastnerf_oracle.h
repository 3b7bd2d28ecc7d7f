/*
 * FP64 reference renderer for FastNeRF's cached path -- TEST INFRASTRUCTURE.
 *
 * This header belongs to the oracle alone. The HIP library shares no code,
 * header, table or constant with it. Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load the oracle; the product path never
 * does.
 *
 * What is computed (paper, Sec. 3.1 Eq. 1, Sec. 3.2 Eq. 5, Sec. 3.3, Sec. 4,
 * supplementary S3): for every pixel a ray is cast from the camera, N samples
 * are placed between its near and far bounds, each sample reads density and the
 * D-component deep radiance map from the k^3 position cache, the ray reads the
 * D weights beta once from the l x l direction cache, the colour of a sample is
 * the inner product of beta with the radiance map, and the samples are
 * composited front to back with the transmittance, stopping once it falls
 * below eps. Readings where the paper is silent are listed next to the code.
 */
#ifndef FASTNERF_ORACLE_H
#define FASTNERF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXCAND 32        /* candidate results kept per pixel */
#define ORC_MAXCHOICE 3       /* ambiguous lookups enumerated per pixel (default) */
#define ORC_MAXCHOICE_LIMIT 5 /* the most that orc_tol.max_choice may ask for */

/* Pixel flags. */
#define ORC_HIT 1        /* the ray's sample interval is non-empty */
#define ORC_AMBIG 2      /* more than one admissible result */
#define ORC_UNCHECKED 4  /* too many ambiguous lookups to enumerate */

typedef struct {
  int32_t k, D, l;
  double bmin[3], bmax[3];
  int32_t pos_linear;   /* 0: nearest voxel; 1: trilinear over voxel centres */
  int32_t dir_linear;   /* 0: nearest cell;  1: bilinear over cell centres   */
  int32_t in_box;       /* 0: samples span [near,far]; 1: [near,far] clipped to the box */
  double bg[3];         /* background colour */
  /* Dense position cache (NULL when the brick-sparse source below is used). */
  const float *sigma;   /* [k][k][k], x fastest: index (z*k + y)*k + x */
  const float *u;       /* [k][k][k][D][3] */
  /* Brick-sparse position cache: bricks of sb^3 voxels, absent bricks read as 0. */
  int32_t sb;
  const int32_t *slot;  /* [(k/sb)^3] slot index or -1, brick index (bz*nb + by)*nb + bx */
  const float *ssigma;  /* [nslot][sb^3], brick-local x fastest */
  const float *su;      /* [nslot][sb^3][D][3] */
  /* Direction cache. */
  const float *beta;    /* [l][l][D]: theta row, phi column */
  /* Per-brick occupancy used only to count samples in occupied bricks
     (the byte count of the measurement); NULL = do not count. */
  int32_t ob;
  const uint8_t *occ;   /* [(k/ob)^3] */
} orc_scene;

typedef struct {
  double K[9];          /* 3x3 intrinsics, row-major */
  double c2w[12];       /* 3x4 camera-to-world, row-major, columns right, down, forward, eye */
  int32_t H, W;
  double near, far;
  int32_t N;            /* samples per ray; 0 = every voxel the ray crosses (nearest only) */
  double eps;           /* termination threshold on transmittance; 0 = never stop */
} orc_view;

typedef struct {
  double gamma;         /* voxels: samples this close to a cell boundary may take either voxel */
  double gamma_dir;     /* radians: same for nearest direction cells */
  double tau_band;      /* log-transmittance: stop points this close to ln(1/eps) are both admissible */
  int32_t max_choice;   /* ambiguous lookups enumerated per pixel: 0 = ORC_MAXCHOICE, < 0 =
                           none, at most ORC_MAXCHOICE_LIMIT */
} orc_tol;

typedef struct {
  int64_t rays, hit, samples, occ_samples, nonzero_samples, ambiguous_pixels, unchecked_pixels;
} orc_counts;

/* Renders the listed pixels (pix = linear index y*W + x; NULL = all H*W pixels in
   order). rgba receives the primary result, cand/ncand (may be NULL) every
   admissible result, flags (may be NULL) the ORC_* bits, env (may be NULL; 8
   doubles per pixel: RGBA lower bounds, then upper bounds) an enclosure of
   every admissible result: the hull of the enumerated ones, or for an
   ORC_UNCHECKED pixel interval bounds over all its variants. Returns 0, or -1
   on a bad argument. */
int orc_render(const orc_scene *s, const orc_view *v, const orc_tol *tol, int64_t npix,
               const int64_t *pix, double *rgba, double *cand, int32_t *ncand,
               int32_t *flags, double *env, orc_counts *counts);

/* orc_render split into nthreads contiguous bands of the pixel list, one
   thread each; bitwise the same results, counts summed. */
int orc_render_mt(const orc_scene *s, const orc_view *v, const orc_tol *tol, int64_t npix,
                  const int64_t *pix, double *rgba, double *cand, int32_t *ncand,
                  int32_t *flags, double *env, orc_counts *counts, int32_t nthreads);

/* Pieces of the definition, exposed for the pins. */
void orc_pixel_ray(const orc_view *v, double x, double y, double o[3], double d[3]);
int orc_interval(const orc_scene *s, const orc_view *v, const double o[3], const double d[3],
                 double *t0, double *t1);
void orc_lookup_pos(const orc_scene *s, int64_t n, const double *pts, double *sigma_out,
                    double *u_out);
void orc_lookup_dir(const orc_scene *s, int64_t n, const double *dirs, double *beta_out);
/* All N samples of one pixel with no termination: t, sigma, colour, and delta. */
int orc_trace(const orc_scene *s, const orc_view *v, int32_t x, int32_t y, double *t,
              double *sigma, double *rgb, double *delta);
/* Per-brick occupancy (any sigma > 0) of the scene's source, edge ob. */
void orc_occupancy(const orc_scene *s, int32_t ob, uint8_t *occ);

/* Storage formats, written from the IEEE-754 binary16, bfloat16 and OCP 8-bit
   (E4M3, "fn") definitions. fmt: 1 = binary16, 2 = bfloat16 (round to nearest
   even, overflow to infinity); 3 = E4M3 (round to nearest even, saturating at
   +-448). */
double orc_round_to(int32_t fmt, double x);
double orc_e4m3_decode(uint32_t code);
uint32_t orc_e4m3_encode(float y);
/* Dequantised copy of a position cache in storage format fmt (0 = FP32 copy).
   E4M3 uses one scale per channel (sigma, then the 3D radiance channels):
   s = absmax/448 in FP32 (1 when absmax is 0), code = E4M3(x/s in FP32),
   value = code*s in FP32. scales (1+3D floats) may be NULL. */
void orc_dequant_cache(int32_t fmt, int64_t nvox, int32_t D, const float *sigma, const float *u,
                       float *sigma_q, float *u_q, float *scales);

#ifdef __cplusplus
}
#endif
#endif
