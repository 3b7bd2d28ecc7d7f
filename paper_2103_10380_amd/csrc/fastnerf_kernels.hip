// gfx950 kernels of the FastNeRF cached renderer.
//
//   k_render      the hot path: rays of 8x8 pixel tiles (one tile per wave,
//                 tiles taken from persistent queues), empty-space skipping on
//                 the brick bitgrid and distance field, record gathers, Eq. 5
//                 colour, Eq. 1 compositing in optical depth with early
//                 termination.
//   k_render_step the same over a serving step's views and scenes.
//   k_absmax      per-channel |max| for FP8 scales.
//   k_pack        FP32 slab -> padded brick-linear records in the storage format.
//   k_occupancy   brick bitgrid from the stored densities.
//   k_dist_*      per-brick Chebyshev distance to the nearest occupied brick.
//   k_readback    records -> FP32 arrays (test hook).
//   k_lookup      the render kernel's own lookups at given points (test hook).
#include "fastnerf_device.h"
#include "fastnerf_kernels.h"

namespace fnr {

// ------------------------------------------------------------------ render

// Samples in flight per lane between loads and compositing. Tuning
// (compile-time, measured on the paper-scale orbit): samples whose occupancy
// bits are fetched together, and records requested together per lane for each
// storage format -- one 128-byte FP32 record keeps the kernel at 4 waves per
// SIMD, which beat two records at 3 waves; two 64-byte FP16 records beat four.
#ifndef FNR_WIN
#define FNR_WIN 16
#endif
#ifndef FNR_BATCH_F32
#define FNR_BATCH_F32 1
#endif
#ifndef FNR_BATCH_F16
#define FNR_BATCH_F16 2
#endif
#ifndef FNR_BATCH_F8
#define FNR_BATCH_F8 4
#endif
constexpr int kWin = FNR_WIN;
// Wave priority raised while a gather round issues its record loads (0: off).
#ifndef FNR_PRIO
#define FNR_PRIO 1
#endif

template <int FMT, bool LIN> struct Batch {
  static constexpr int value =
      LIN ? 1 : (FMT == 0 ? FNR_BATCH_F32 : (FMT == 3 ? FNR_BATCH_F8 : FNR_BATCH_F16));
};

// Records in flight per lane of the wide kernel, for launches too small to
// fill the chip (a single view): more requests per ray at fewer waves per
// SIMD shorten the dependency chain of the heaviest rays, which bounds such a
// launch.
#ifndef FNR_WIDE_F32
#define FNR_WIDE_F32 4
#endif
#ifndef FNR_WIDE_F16
#define FNR_WIDE_F16 4
#endif
#ifndef FNR_WIDE_F8
#define FNR_WIDE_F8 8
#endif
template <int FMT, bool LIN> struct WideBatch {
  static constexpr int value =
      LIN ? 2 : (FMT == 0 ? FNR_WIDE_F32 : (FMT == 3 ? FNR_WIDE_F8 : FNR_WIDE_F16));
};

// Marching state of one ray (one lane): the interval start and direction in
// grid coordinates, the sample spacing, the next window's first sample, the
// composite so far and the per-ray colour weights.
template <int FMT, int MAXD> struct Ray {
  float og[3];   // grid coordinates of the interval start
  float gd[3];   // grid coordinates per unit distance
  float dt;      // sample spacing (distance)
  float inv_step;  // 1 / (voxels advanced per sample in the max norm)
  int i, N;      // first sample of the next window, samples per ray
  float lim;     // ln(1/eps)
  float tau, cr, cg, cb;
  float cw[ColourWeights<FMT, MAXD>::n];
  float4 *out;   // the pixel
};

// Ray set-up, once per ray, in FP64: the direction's small components and the
// box-entry distance are sensitive to rounding (near-grazing rays), and every
// sample position depends on them. Reading: pixel centres, OpenCV axes, unit
// direction. Fills everything but the colour weights, and beta (the direction
// lookup, once per ray) when the ray has samples to march; returns false for
// a ray whose sample interval is empty.
template <int FMT, int MAXD>
__device__ __forceinline__ bool ray_setup(const DevCache &c, const DevView &V, int px, int py,
                                          Ray<FMT, MAXD> &r, float *beta) {
  const double qx = (double)px + 0.5, qy = (double)py + 0.5;
  double ddx = fma(V.M[0], qx, fma(V.M[1], qy, V.M[2]));
  double ddy = fma(V.M[3], qx, fma(V.M[4], qy, V.M[5]));
  double ddz = fma(V.M[6], qx, fma(V.M[7], qy, V.M[8]));
  const double rn = 1.0 / sqrt(fma(ddx, ddx, fma(ddy, ddy, ddz * ddz)));
  ddx *= rn;
  ddy *= rn;
  ddz *= rn;
  r.out = reinterpret_cast<float4 *>(V.out) + ((size_t)py * V.W + px);
  r.tau = r.cr = r.cg = r.cb = 0.0f;
  r.i = 0;
  r.N = V.N;
  r.lim = V.lim;
  // sample interval
  double t0 = V.near_, t1 = V.far_;
  if (c.in_box) {
    const double d3[3] = {ddx, ddy, ddz};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double lo = c.bmin[ax], hi = c.bmax[ax];
      if (d3[ax] == 0.0) {
        if (V.o[ax] < lo || V.o[ax] > hi) t1 = -1.0;
      } else {
        const double ta = (lo - V.o[ax]) / d3[ax], tb = (hi - V.o[ax]) / d3[ax];
        t0 = fmax(t0, fmin(ta, tb));
        t1 = fmin(t1, fmax(ta, tb));
      }
    }
  }
  if (!(t1 > t0)) return false;
  dir_lookup<MAXD>(c, (float)ddx, (float)ddy, (float)ddz, beta);
  r.dt = (float)((t1 - t0) / (double)V.N);
  // grid coordinates of the interval start and the per-distance step;
  // sample i sits at distance (i + 1/2) dt past the start
  r.og[0] = (float)((fma(t0, ddx, V.o[0]) - c.bmin[0]) * c.inv_h[0]);
  r.og[1] = (float)((fma(t0, ddy, V.o[1]) - c.bmin[1]) * c.inv_h[1]);
  r.og[2] = (float)((fma(t0, ddz, V.o[2]) - c.bmin[2]) * c.inv_h[2]);
  r.gd[0] = (float)(ddx * c.inv_h[0]);
  r.gd[1] = (float)(ddy * c.inv_h[1]);
  r.gd[2] = (float)(ddz * c.inv_h[2]);
  const float vstep = r.dt * fmaxf(fabsf(r.gd[0]), fmaxf(fabsf(r.gd[1]), fabsf(r.gd[2])));
  r.inv_step = 1.0f / vstep;
  return true;
}

// Per-ray colour weights from beta: beta itself, or for E4M3 records beta
// times the channel scales (Eq. 5 with the dequantisation folded in).
template <int FMT, int MAXD>
__device__ __forceinline__ void ray_weights(const DevCache &c, const float *beta,
                                            Ray<FMT, MAXD> &r) {
#pragma unroll
  for (int d = 0; d < MAXD; ++d) {
    if (FMT == 3) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) r.cw[3 * d + ch] = beta[d] * c.scales[1 + 3 * d + ch];
    } else {
      r.cw[d] = beta[d];
    }
  }
}

// Brick distance (bricks, max norm, to the nearest occupied brick; the
// distance field's bricks) at sample i of a ray, at the same position and
// clamped voxel as the window scan computes for it.
template <int FMT, int MAXD>
__device__ __forceinline__ uint32_t sample_distance(const DevCache &c, const Ray<FMT, MAXD> &r,
                                                    int i) {
  const float kmax = (float)(c.k - 1);
  const float t = ((float)i + 0.5f) * r.dt;
  const float gx = fmaf(t, r.gd[0], r.og[0]), gy = fmaf(t, r.gd[1], r.og[1]),
              gz = fmaf(t, r.gd[2], r.og[2]);
  const int x = voxel_of(gx, kmax), y = voxel_of(gy, kmax), z = voxel_of(gz, kmax);
  return __ldg(c.dist + grid3((uint32_t)x >> c.dshift, (uint32_t)y >> c.dshift,
                              (uint32_t)z >> c.dshift, (uint32_t)c.nbd));
}

// The first sample to scan after sample i, given its brick distance d: d >= 2
// proves every point within (d - 1) brick edges of the sample empty, so the
// samples i .. i + run are skipped (the window scan's rule); otherwise i.
__device__ __forceinline__ int skip_from(uint32_t d, int i, float bedge, float inv_step, int N) {
  if (d < 2u) return i;
  const float run = fminf(((float)(d - 1u) * bedge - 0.5f) * inv_step, (float)N);
  return i + 1 + (int)run;
}

// Jumps taken at ray set-up, before the first window: the first distance is
// loaded beside the direction cells, each later one after the previous jump.
// Skipped samples lie in empty bricks, so the image is the same with any
// count; the count trades window scans for dependent loads.
#ifndef FNR_SETUP_JUMPS
#define FNR_SETUP_JUMPS 4
#endif
constexpr int kSetupJumps = FNR_SETUP_JUMPS;

// The pixel: RGB = C + T bg, A = 1 - T (T = exp(-tau)).
__device__ __forceinline__ float4 pixel_value(const DevCache &c, float tau, float cr, float cg,
                                              float cb) {
  const float T = expf(-tau);
  float4 res;
  res.x = fmaf(T, c.bg[0], cr);
  res.y = fmaf(T, c.bg[1], cg);
  res.z = fmaf(T, c.bg[2], cb);
  res.w = -expm1f(-tau);
  return res;
}
template <int FMT, int MAXD>
__device__ __forceinline__ void ray_finish(const DevCache &c, const Ray<FMT, MAXD> &r) {
  *r.out = pixel_value(c, r.tau, r.cr, r.cg, r.cb);
}

// Pixel of lane (lx, ly) in tile lt (edge T) of view V's render rectangle.
template <int T>
__device__ __forceinline__ void tile_pixel(const DevView &V, int lt, int lx, int ly, int &px,
                                           int &py) {
  const int ntx = (V.cx1 + T - 1) / T - V.cx0 / T;
  px = (V.cx0 / T + lt % ntx) * T + lx;
  py = (V.cy0 / T + lt / ntx) * T + ly;
}

// The pixels of the launch's views outside their render rectangles: rays that
// cannot meet the box, whose pixel is the background (the value a ray with no
// composited sample gets). All threads of the grid share the work before
// they take tiles.
__device__ __forceinline__ void fill_outside(const RenderArgs &a) {
  const float4 bgp = pixel_value(a.c, 0.0f, 0.0f, 0.0f, 0.0f);
  const int nv = a.views ? a.nviews : 1;
  const long long nt = (long long)gridDim.x * blockDim.x;
  const long long gt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (int vi = 0; vi < nv; ++vi) {
    const DevView *V = a.views ? a.views + vi : &a.v0;
    const int W = V->W, H = V->H, x0 = V->cx0, y0 = V->cy0, x1 = V->cx1, y1 = V->cy1;
    if (x0 == 0 && y0 == 0 && x1 >= W && y1 >= H) continue;
    float4 *out = reinterpret_cast<float4 *>(V->out);
    const long long n = (long long)W * H;
    if (gt >= n) continue;
    // (x, y) of pixel p, stepped by nt pixels without a division per step
    const long long sy = nt / W;
    const int sx = (int)(nt - sy * W);
    long long yy = gt / W;
    int x = (int)(gt - yy * W);
    for (long long p = gt; p < n; p += nt) {
      const int y = (int)yy;
      if (x < x0 || x >= x1 || y < y0 || y >= y1) out[p] = bgp;
      x += sx;
      yy += sy;
      if (x >= W) {
        x -= W;
        ++yy;
      }
    }
  }
}

// One window of kWin samples of a live ray: the occupancy bits of the window
// are fetched with independent loads and one wait, then its occupied samples
// are gathered and composited in order, B records in flight at a time. With
// the same wait, the brick distance d of the window's last sample is read:
// d >= 2 (bricks, max norm, to the nearest occupied brick) proves that every
// point within (d - 1) brick edges of that sample lies in an empty brick, so
// the next window starts past the last sample so proven empty. Samples advance
// vstep voxels each in the max norm; half a voxel of margin covers FP32
// position rounding. alive turns false when the ray stops (optical depth past
// ln(1/eps)) or runs out of samples. Lanes enter with alive false and do
// nothing (the wave runs the window for its live lanes).
// SPARSE: a brick-sparse cache (bitgrid brick = storage brick = 8^3); the
// stored brick of a flagged sample is its rank among the set bitgrid bits,
// found from the bitgrid word already loaded by the window scan and the count
// of set bits before that word (one more independent load), so the gather
// needs no dependent table lookup.
template <int FMT, int MAXD, bool LIN, bool SPARSE, int B = Batch<FMT, LIN>::value,
          bool OL = false>
__device__ __forceinline__ void ray_window(const DevCache &c, Ray<FMT, MAXD> &r, bool &alive,
                                           float s0, const uint32_t *locc = nullptr) {
  using RW = RecWords<FMT, MAXD>;
  const int k = c.k;
  const float kf = c.kf;
  const float kmax = (float)(k - 1);
  const int N = r.N;
  const float dt = r.dt;
  const float bedge = (float)(1 << c.dshift);
  // sample i + j sits at distance (i + j + 1/2) dt: fi + (j + 1/2) is exact,
  // so the scan and the gather below compute the same positions
  const float fi = (float)r.i;
  uint32_t mask = 0u;
  int next = r.i + kWin;
  uint32_t sslot[SPARSE ? kWin : 1];  // stored brick of each sample (SPARSE)
  if (alive) {
    // a cache without a bitgrid has one all-ones word and one zero
    // distance, with oshift past every coordinate bit
    uint32_t word[kWin], bitpos[kWin], rk[SPARSE ? kWin : 1], dlast = 0u;
    bool in[kWin];
#pragma unroll
    for (int j = 0; j < kWin; ++j) {
      const float t = (fi + ((float)j + 0.5f)) * dt;
      const float gx = fmaf(t, r.gd[0], r.og[0]), gy = fmaf(t, r.gd[1], r.og[1]),
                  gz = fmaf(t, r.gd[2], r.og[2]);
      // inside the box: 0 <= g <= k on every axis
      in[j] = (r.i + j < N) && fminf(fminf(gx, gy), gz) >= 0.0f &&
              fmaxf(fmaxf(gx, gy), gz) <= kf;
      // clamped voxel: always a valid address, even when not inside
      const int x = voxel_of(gx, kmax), y = voxel_of(gy, kmax), z = voxel_of(gz, kmax);
      const uint32_t bit = grid3((uint32_t)x >> c.oshift, (uint32_t)y >> c.oshift,
                                 (uint32_t)z >> c.oshift, (uint32_t)c.nbo);
      // OL: the occupancy words are held in LDS (locc), a copy of c.occ
      word[j] = OL ? locc[bit >> 5] : __ldg(c.occ + (bit >> 5));
      bitpos[j] = bit & 31u;
      if (SPARSE) rk[(SPARSE ? j : 0)] = __ldg(c.rank + (bit >> 5));
      if (j == kWin - 1)
        dlast = __ldg(c.dist + grid3((uint32_t)x >> c.dshift, (uint32_t)y >> c.dshift,
                                     (uint32_t)z >> c.dshift, (uint32_t)c.nbd));
    }
#pragma unroll
    for (int j = 0; j < kWin; ++j)
      mask |= (uint32_t)(in[j] && ((word[j] >> bitpos[j]) & 1u)) << j;
    if (SPARSE) {
#pragma unroll
      for (int j = 0; j < kWin; ++j)
        sslot[(SPARSE ? j : 0)] = 1u + rk[(SPARSE ? j : 0)] +
                                  (uint32_t)__builtin_popcount(word[j] & ((1u << bitpos[j]) - 1u));
    }
    if (dlast >= 2u) {
      const float run = fminf(((float)(dlast - 1u) * bedge - 0.5f) * r.inv_step, (float)N);
      next += (int)run;
    }
  }
  // record registers: loaded only by lanes with a sample in the slot; the
  // others keep earlier (defined) values, which the composite selects away
  uint32_t w[B][RW::nwords];
#pragma unroll
  for (int b = 0; b < B; ++b)
#pragma unroll
    for (int q = 0; q < RW::nwords; ++q) w[b][q] = 0u;
  while (mask != 0u && alive) {
    // the next B occupied samples; slots past the last one repeat the
    // first sample's voxel, so every load has a valid (cached) address
    int vx[B], vy[B], vz[B];
    float wx[B], wy[B], wz[B];
    uint32_t sb[B];
    bool have[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      have[b] = mask != 0u;
      sb[b] = 0u;
      if (have[b]) {
        const int j = __builtin_ctz(mask);
        mask &= mask - 1u;
        if (SPARSE) {  // j varies across lanes: a select chain
          uint32_t v = sslot[0];
#pragma unroll
          for (int q = 1; q < kWin; ++q) v = q == j ? sslot[(SPARSE ? q : 0)] : v;
          sb[b] = v;
        }
        const float t = (fi + ((float)j + 0.5f)) * dt;
        const float gx = fmaf(t, r.gd[0], r.og[0]), gy = fmaf(t, r.gd[1], r.og[1]),
                    gz = fmaf(t, r.gd[2], r.og[2]);
        if (LIN) {
          const float hx = gx - 0.5f, hy = gy - 0.5f, hz = gz - 0.5f;
          const float fx0 = floorf(hx), fy0 = floorf(hy), fz0 = floorf(hz);
          vx[b] = (int)fx0;
          vy[b] = (int)fy0;
          vz[b] = (int)fz0;
          wx[b] = hx - fx0;
          wy[b] = hy - fy0;
          wz[b] = hz - fz0;
        } else {
          vx[b] = voxel_of(gx, kmax);
          vy[b] = voxel_of(gy, kmax);
          vz[b] = voxel_of(gz, kmax);
          wx[b] = wy[b] = wz[b] = 0.0f;
        }
      } else {
        vx[b] = vx[0];
        vy[b] = vy[0];
        vz[b] = vz[0];
        wx[b] = wy[b] = wz[b] = 0.0f;
        sb[b] = sb[0];
      }
    }
    if (!LIN) {
      uint64_t off[B];
#pragma unroll
      for (int b = 0; b < B; ++b)
        off[b] = SPARSE ? record_offset_in(c, sb[b], vx[b], vy[b], vz[b])
                        : record_offset(c, vx[b], vy[b], vz[b]);
      // the loads go out at a raised wave priority, so that a wave about to
      // wait on memory issues them ahead of waves busy with scans or
      // composites on the same SIMD (measured: FP32 launches 1.5-2% faster)
      if (FNR_PRIO) __builtin_amdgcn_s_setprio(2);
#pragma unroll
      for (int b = 0; b < B; ++b)
        if (have[b] && alive) load_record<FMT, MAXD>(c, off[b], w[b]);
      if (FNR_PRIO) __builtin_amdgcn_s_setprio(0);
      // all B records are requested before the first is used, each only
      // by the lanes that have a sample in its slot (the others issue no
      // memory request); an unused slot (past the window's last occupied
      // sample, or after the stop) adds zero optical depth and zero colour
#pragma unroll
      for (int b = 0; b < B; ++b) {
        // no contraction of sigma*dt into the optical-depth sum: every
        // slot, and every occupancy setting, rounds alike
#pragma clang fp contract(off)
        const bool use = have[b] && alive;
        const float s = rec_sigma<FMT>(w[b], s0);
        float cr, cg, cb;
        rec_colour<FMT, MAXD>(w[b], r.cw, cr, cg, cb);
        cr = use ? cr : 0.0f;
        cg = use ? cg : 0.0f;
        cb = use ? cb : 0.0f;
        const float sd = use ? s * dt : 0.0f;
        const float wgt = exp_neg(r.tau) * opacity(sd);
        r.cr = fmaf(wgt, cr, r.cr);
        r.cg = fmaf(wgt, cg, r.cg);
        r.cb = fmaf(wgt, cb, r.cb);
        r.tau = r.tau + sd;
        alive = alive && !(r.tau > r.lim);  // every later sample would be stopped
      }
    } else {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if (!have[b] || !alive) continue;
        uint32_t wq[8][RW::nwords];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int x = min(max(vx[b] + (q & 1), 0), k - 1);
          const int y = min(max(vy[b] + ((q >> 1) & 1), 0), k - 1);
          const int z = min(max(vz[b] + ((q >> 2) & 1), 0), k - 1);
          load_record<FMT, MAXD>(c, record_offset(c, x, y, z), wq[q]);
        }
        float s = 0.f, cr = 0.f, cg = 0.f, cb = 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float wt = ((q & 1) ? wx[b] : 1.0f - wx[b]) *
                           (((q >> 1) & 1) ? wy[b] : 1.0f - wy[b]) *
                           (((q >> 2) & 1) ? wz[b] : 1.0f - wz[b]);
          float rq, gq, bq;
          rec_colour<FMT, MAXD>(wq[q], r.cw, rq, gq, bq);
          s = fmaf(wt, rec_sigma<FMT>(wq[q], s0), s);
          cr = fmaf(wt, rq, cr);
          cg = fmaf(wt, gq, cg);
          cb = fmaf(wt, bq, cb);
        }
        const float sd = s * dt;
        const float wgt = exp_neg(r.tau) * opacity(sd);
        r.cr = fmaf(wgt, cr, r.cr);
        r.cg = fmaf(wgt, cg, r.cg);
        r.cb = fmaf(wgt, cb, r.cb);
        r.tau = r.tau + sd;
        if (r.tau > r.lim) alive = false;
      }
    }
  }
  if (alive) {
    r.i = next;
    if (r.i >= N) alive = false;
  }
}

// Renders the rays of one 8x8 tile (one ray per lane) of view V with cache c:
// set-up, windows until the ray stops, the pixel.
template <int FMT, int MAXD, bool LIN, bool SPARSE = false, int B = Batch<FMT, LIN>::value,
          bool OL = false>
__device__ __forceinline__ void render_tile(const RenderArgs &a, const DevCache &c,
                                            const DevView &V, int lt, int lane,
                                            const uint32_t *locc = nullptr) {
  (void)a;
  int px, py;
  tile_pixel<8>(V, lt, lane & 7, lane >> 3, px, py);
  if (px >= V.W || py >= V.H) return;
  Ray<FMT, MAXD> r;
  float beta[MAXD];
  bool alive = ray_setup<FMT, MAXD>(c, V, px, py, r, beta);
  if (alive) {
    uint32_t d = kSetupJumps > 0 ? sample_distance<FMT, MAXD>(c, r, 0) : 0u;
    ray_weights<FMT, MAXD>(c, beta, r);
    const float bedge = (float)(1 << c.dshift);
#pragma unroll
    for (int q = 0; q < kSetupJumps; ++q) {
      const int nx = skip_from(d, r.i, bedge, r.inv_step, r.N);
      d = 0u;
      if (nx != r.i) {
        r.i = nx;
        if (q + 1 < kSetupJumps && nx < r.N) d = sample_distance<FMT, MAXD>(c, r, nx);
      }
    }
    alive = r.i < r.N;
    const float s0 = FMT == 3 ? c.scales[0] : 1.0f;
    while (alive) ray_window<FMT, MAXD, LIN, SPARSE, B, OL>(c, r, alive, s0, locc);
  }
  ray_finish<FMT, MAXD>(c, r);
}

// ------------------------------------------------------------------ voxel traversal

// Pieces of a ray generated per window of the voxel traversal.
#ifndef FNR_VWIN
#define FNR_VWIN 8
#endif
constexpr int kVWin = FNR_VWIN;
constexpr float kVInf = 3.0e38f;

// Distance (from the interval start, in t) to the next crossing of a voxel
// face along one axis from cell c, moving by step (+1/-1); interior faces sit
// at grid coordinates i = 1..k-1 (the first and last cells end at the box
// faces, where the interval ends).
__device__ __forceinline__ float vox_next(int c, int step, int k, float og, float igd) {
  if (step == 0) return kVInf;
  const int b = step > 0 ? c + 1 : c;  // face index
  if (b < 1 || b > k - 1) return kVInf;
  return ((float)b - og) * igd;
}

// Renders the rays of one 8x8 tile by visiting every voxel each ray crosses
// inside [near, far] and the box (N = 0): each piece between consecutive cell
// boundaries is one sample with delta = its length (Eq. 1 with the piece
// lengths; nearest lookups). Pieces are produced kVWin at a time by stepping
// from boundary to boundary (each crossing computed directly from its index,
// not accumulated), their bricks tested with independent loads, and the
// occupied ones gathered and composited in order. The brick distance of the
// last piece lets the traversal restart past the space it proves empty.
template <int FMT, int MAXD>
__device__ __forceinline__ void render_tile_vox(const RenderArgs &a, const DevCache &c,
                                                const DevView &V, int lt, int lane) {
  using RW = RecWords<FMT, MAXD>;
  constexpr int B = Batch<FMT, false>::value;
  const int W = V.W, H = V.H;
  int px, py;
  tile_pixel<8>(V, lt, lane & 7, lane >> 3, px, py);
  if (px >= W || py >= H) return;
  const int k = c.k;
  // FP64 ray set-up, as in render_tile; the interval is always clipped to the box
  const double qx = (double)px + 0.5, qy = (double)py + 0.5;
  double ddx = fma(V.M[0], qx, fma(V.M[1], qy, V.M[2]));
  double ddy = fma(V.M[3], qx, fma(V.M[4], qy, V.M[5]));
  double ddz = fma(V.M[6], qx, fma(V.M[7], qy, V.M[8]));
  const double rn = 1.0 / sqrt(fma(ddx, ddx, fma(ddy, ddy, ddz * ddz)));
  ddx *= rn;
  ddy *= rn;
  ddz *= rn;
  double t0 = V.near_, t1 = V.far_;
  {
    const double d3[3] = {ddx, ddy, ddz};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double lo = c.bmin[ax], hi = c.bmax[ax];
      if (d3[ax] == 0.0) {
        if (V.o[ax] < lo || V.o[ax] > hi) t1 = -1.0;
      } else {
        const double ta = (lo - V.o[ax]) / d3[ax], tb = (hi - V.o[ax]) / d3[ax];
        t0 = fmax(t0, fmin(ta, tb));
        t1 = fmin(t1, fmax(ta, tb));
      }
    }
  }
  float tau = 0.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
  if (t1 > t0) {
    float cw[ColourWeights<FMT, MAXD>::n];
    float s0 = 1.0f;
    {
      float beta[MAXD];
      dir_lookup<MAXD>(c, (float)ddx, (float)ddy, (float)ddz, beta);
#pragma unroll
      for (int d = 0; d < MAXD; ++d) {
        if (FMT == 3) {
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) cw[3 * d + ch] = beta[d] * c.scales[1 + 3 * d + ch];
        } else {
          cw[d] = beta[d];
        }
      }
      if (FMT == 3) s0 = c.scales[0];
    }
    const float L = (float)(t1 - t0);
    const float og[3] = {(float)((fma(t0, ddx, V.o[0]) - c.bmin[0]) * c.inv_h[0]),
                         (float)((fma(t0, ddy, V.o[1]) - c.bmin[1]) * c.inv_h[1]),
                         (float)((fma(t0, ddz, V.o[2]) - c.bmin[2]) * c.inv_h[2])};
    const float gd[3] = {(float)(ddx * c.inv_h[0]), (float)(ddy * c.inv_h[1]),
                         (float)(ddz * c.inv_h[2])};
    int step[3];
    float igd[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      step[ax] = gd[ax] > 0.0f ? 1 : (gd[ax] < 0.0f ? -1 : 0);
      igd[ax] = step[ax] != 0 ? 1.0f / gd[ax] : 0.0f;
    }
    const float gmax = fmaxf(fabsf(gd[0]), fmaxf(fabsf(gd[1]), fabsf(gd[2])));
    const float bedge = (float)(1 << c.dshift);
    // traversal state: position s along [0, L], current cell, next crossings
    float sc = 0.0f;
    int cell[3];
    float sn[3];
    bool restart = true;
    bool alive = true;
    while (alive && sc < L) {
      if (restart) {  // (re)enter the grid at sc
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const float g = fmaf(sc, gd[ax], og[ax]);
          cell[ax] = min(max((int)floorf(g), 0), k - 1);
          sn[ax] = vox_next(cell[ax], step[ax], k, og[ax], igd[ax]);
          if (sn[ax] <= sc) {  // on (or rounded past) the face: the next cell
            cell[ax] = min(max(cell[ax] + step[ax], 0), k - 1);
            sn[ax] = vox_next(cell[ax], step[ax], k, og[ax], igd[ax]);
          }
        }
        restart = false;
      }
      // the window's pieces: record index, bitgrid bit, length
      uint32_t rec[kVWin], bit[kVWin], dbrick = 0u;
      float len[kVWin];
      uint32_t valid = 0u;
#pragma unroll
      for (int j = 0; j < kVWin; ++j) {
        const float se = fminf(fminf(sn[0], sn[1]), fminf(sn[2], L));
        const bool v = sc < L;
        len[j] = v ? se - sc : 0.0f;
        valid |= (uint32_t)v << j;
        const int x = cell[0], y = cell[1], z = cell[2];
        const uint32_t lb = ((uint32_t)(z >> 3) * (uint32_t)c.nbl + (uint32_t)(y >> 3)) *
                                (uint32_t)c.nbl + (uint32_t)(x >> 3);
        rec[j] = (lb << 9) | ((uint32_t)(z & 7) << 6) | ((uint32_t)(y & 7) << 3) | (uint32_t)(x & 7);
        bit[j] = ((uint32_t)(z >> c.oshift) * (uint32_t)c.nbo + (uint32_t)(y >> c.oshift)) *
                     (uint32_t)c.nbo + (uint32_t)(x >> c.oshift);
        if (j == kVWin - 1)
          dbrick = grid3((uint32_t)x >> c.dshift, (uint32_t)y >> c.dshift,
                         (uint32_t)z >> c.dshift, (uint32_t)c.nbd);
        // advance every axis whose boundary is crossed at se
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          if (v && sn[ax] <= se) {
            cell[ax] = min(max(cell[ax] + step[ax], 0), k - 1);
            sn[ax] = vox_next(cell[ax], step[ax], k, og[ax], igd[ax]);
          }
        }
        sc = v ? se : sc;
      }
      uint32_t word[kVWin];
#pragma unroll
      for (int j = 0; j < kVWin; ++j) word[j] = __ldg(c.occ + (bit[j] >> 5));
      const uint32_t dlast = __ldg(c.dist + dbrick);
      uint32_t mask = 0u;
#pragma unroll
      for (int j = 0; j < kVWin; ++j) mask |= ((word[j] >> (bit[j] & 31u)) & 1u) << j;
      mask &= valid;
      if (c.slot) {
        // brick-sparse (bitgrid brick = storage brick): the stored brick of a
        // set bit is 1 + the set bits before it; only set pieces are read
        uint32_t rk[kVWin];
#pragma unroll
        for (int j = 0; j < kVWin; ++j) rk[j] = __ldg(c.rank + (bit[j] >> 5));
#pragma unroll
        for (int j = 0; j < kVWin; ++j) {
          const uint32_t sb =
              1u + rk[j] + (uint32_t)__builtin_popcount(word[j] & ((1u << (bit[j] & 31u)) - 1u));
          rec[j] = (sb << 9) | (rec[j] & 511u);
        }
      }
      while (mask != 0u && alive) {
        uint32_t ri[B];
        float li[B];
        bool have[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
          have[b] = mask != 0u;
          ri[b] = ri[0];
          li[b] = 0.0f;
          if (have[b]) {
            const int j = __builtin_ctz(mask);
            mask &= mask - 1u;
            // select the j-th piece (j is lane-varying: a short select chain)
            uint32_t r = rec[0];
            float l = len[0];
#pragma unroll
            for (int q = 1; q < kVWin; ++q) {
              r = q == j ? rec[q] : r;
              l = q == j ? len[q] : l;
            }
            ri[b] = r;
            li[b] = l;
          }
        }
        uint32_t w[B][RW::nwords];
#pragma unroll
        for (int b = 0; b < B; ++b)
          load_record<FMT, MAXD>(c, (uint64_t)ri[b] << c.rec_shift, w[b]);
#pragma unroll
        for (int b = 0; b < B; ++b) {
#pragma clang fp contract(off)
          const bool use = have[b] && alive;
          const float sg = rec_sigma<FMT>(w[b], s0);
          float r, g, bl;
          rec_colour<FMT, MAXD>(w[b], cw, r, g, bl);
          const float sd = use ? sg * li[b] : 0.0f;
          const float wgt = expf(-tau) * -expm1f(-sd);
          cr = fmaf(wgt, r, cr);
          cg = fmaf(wgt, g, cg);
          cb = fmaf(wgt, bl, cb);
          tau = tau + sd;
          alive = alive && !(tau > V.lim);
        }
      }
      // every point within (d - 1) brick edges (max norm) of the window's end
      // lies in an unset brick: restart past it
      if (alive && dlast >= 2u && sc < L) {
        const float run = (((float)(dlast - 1u) * bedge - 0.5f)) / gmax;
        if (run > 0.0f) {
          sc = fminf(sc + run, L);
          restart = true;
        }
      }
    }
  }
  const float T = expf(-tau);
  float4 res;
  res.x = fmaf(T, c.bg[0], cr);
  res.y = fmaf(T, c.bg[1], cg);
  res.z = fmaf(T, c.bg[2], cb);
  res.w = -expm1f(-tau);
  reinterpret_cast<float4 *>(V.out)[(size_t)py * W + px] = res;
}

// Independent tile queues: all waves fetching from one counter serialise on
// that address, so tiles are dealt round-robin to kQueues counters 128 bytes
// apart; the waves of block b take tiles q, q + R, q + 2R, ... with
// q = b mod R.
constexpr int kQueues = 32;
constexpr int kQueueStride = 32;

struct Queue {
  unsigned *ctr;  // [0] tiles handed out, [1] waves retired
  int q, R, total;
};

__device__ __forceinline__ Queue make_queue(const RenderArgs &a, int total) {
  Queue Q;
  Q.R = min(kQueues, (int)gridDim.x);
  Q.q = (int)(blockIdx.x % (unsigned)Q.R);
  Q.ctr = a.counter + Q.q * kQueueStride;
  Q.total = total;
  return Q;
}

// Next tile of the wave's queue (uniform), -1 when it is empty.
__device__ __forceinline__ int queue_fetch(const Queue &Q, int lane) {
  unsigned got = 0;
  if (lane == 0) got = atomicAdd(Q.ctr, 1u);
  const int n = (int)__builtin_amdgcn_readfirstlane(got);
  const long long t = (long long)Q.q + (long long)n * Q.R;
  return t < Q.total ? (int)t : -1;
}

// The last wave of a queue to leave resets it for the next launch on this
// stream (every wave of the queue has made its final fetch before it retires).
__device__ __forceinline__ void queue_retire(const Queue &Q, int lane) {
  if (lane == 0) {
    const unsigned nb = (gridDim.x - (unsigned)Q.q + (unsigned)Q.R - 1u) / (unsigned)Q.R;
    const unsigned nw = nb * (blockDim.x / kWave);
    const unsigned done = atomicAdd(Q.ctr + 1, 1u);
    if (done == nw - 1u) {
      atomicExch(Q.ctr, 0u);
      atomicExch(Q.ctr + 1, 0u);
    }
  }
}

__device__ __forceinline__ int view_of_tile(const RenderArgs &a, int tile, int nviews) {
  int lo = 0, hi = nviews - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.views[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// View of launch tile `tile` in a batch, and its tile lt within that view:
// views one after another (tile_begin ascending), or, when every view of the
// batch has the same tiles, groups of `interleave` consecutive views one after
// another with the tiles of a group's views interleaved (tile r of a group of
// n views: view r % n, its tile r / n), so that the launch works through the
// same part of the group's views at once and its end holds their last rows
// rather than one view's heaviest tiles.
__device__ __forceinline__ int batch_tile(const RenderArgs &a, int tile, int &lt) {
  if (a.interleave > 0) {
    const int tpv = a.total_tiles / a.nviews;
    const int span = a.interleave * tpv;
    const int grp = tile / span;
    const int g0 = grp * a.interleave;
    const int n = min(a.interleave, a.nviews - g0);
    const int r = tile - grp * span;
    lt = r / n;
    return g0 + (r - lt * n);
  }
  const int v = view_of_tile(a, tile, a.nviews);
  lt = tile - a.views[v].tile_begin + a.views[v].tile_offset;
  return v;
}

// One cache, one storage format: single views (inline descriptor) or a batch
// of views in one launch. Each wave renders one 8x8 tile at a time, one ray
// per lane, taking tiles from its queue until the queue is empty.
template <int FMT, int MAXD, bool LIN, bool SPARSE, int B = Batch<FMT, LIN>::value,
          bool OL = false>
__device__ __forceinline__ void render_queue(const RenderArgs &a,
                                             const uint32_t *locc = nullptr) {
  const int lane = threadIdx.x & (kWave - 1);
  fill_outside(a);
  const Queue Q = make_queue(a, a.total_tiles);
  for (;;) {
    const int tile = queue_fetch(Q, lane);
    if (tile < 0) break;
    if (a.views) {
      int lt;
      const DevView V = a.views[batch_tile(a, tile, lt)];
      render_tile<FMT, MAXD, LIN, SPARSE, B, OL>(a, a.c, V, lt, lane, locc);
    } else {
      render_tile<FMT, MAXD, LIN, SPARSE, B, OL>(a, a.c, a.v0, tile, lane, locc);
    }
  }
  queue_retire(Q, lane);
}

// ------------------------------------------------------------------ split rays

#ifndef FNR_SPLIT_JUMPS
#define FNR_SPLIT_JUMPS FNR_SETUP_JUMPS
#endif
constexpr int kSplitJumps = FNR_SPLIT_JUMPS;
#ifndef FNR_SPLIT_WAVES
#define FNR_SPLIT_WAVES 0
#endif
#ifndef FNR_SPLIT_WIN
#define FNR_SPLIT_WIN FNR_WIN
#endif
constexpr int kSplitWin = FNR_SPLIT_WIN;  // samples per window of a split ray
static_assert(kSplitWin % 4 == 0 && kSplitWin <= 32, "split windows: 4 to 32 samples");

// Quad (four-lane group) exchanges through DPP: the value of lane Q of each
// quad to every lane of the quad, and the OR over a quad. Every lane of a
// quad holds the same ray and takes the same branches around these calls.
template <int Q>
__device__ __forceinline__ uint32_t quad_from(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, Q * 0x55, 0xF, 0xF, true);
}
template <int Q>
__device__ __forceinline__ float quad_from(float v) {
  return __uint_as_float(quad_from<Q>(__float_as_uint(v)));
}
__device__ __forceinline__ uint32_t quad_or(uint32_t v) {
  v |= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);  // lanes 1 0 3 2
  v |= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);  // lanes 2 3 0 1
  return v;
}

// One window of a ray held by a quad (lane sub = 0..3 of the quad): the scan
// of the window's kSplitWin samples is shared (lane sub tests samples sub, sub + 4,
// ...; the quad ORs the bits; lane 3 reads the last sample's brick distance),
// and each gather round fetches the window's next four occupied samples, one
// per lane, one record each. Every lane then steps the ray through the
// round's samples in order, each lane computing the weight of its own sample,
// with the same operations as ray_window, so the ray state stays the same in
// all four lanes and the image equals the tile schedule's bitwise.
template <int FMT, int MAXD>
__device__ __forceinline__ void split_window(const DevCache &c, Ray<FMT, MAXD> &r, bool &alive,
                                             float s0, int sub) {
  using RW = RecWords<FMT, MAXD>;
  const float kf = c.kf;
  const float kmax = (float)(c.k - 1);
  const int N = r.N;
  const float dt = r.dt;
  const float bedge = (float)(1 << c.dshift);
  const float fi = (float)r.i;
  uint32_t part = 0u, dl = 0u;
  if (alive) {
    uint32_t word[kSplitWin / 4], bitpos[kSplitWin / 4];
    bool in[kSplitWin / 4];
#pragma unroll
    for (int q = 0; q < kSplitWin / 4; ++q) {
      const int j = sub + 4 * q;
      const float t = (fi + ((float)j + 0.5f)) * dt;
      const float gx = fmaf(t, r.gd[0], r.og[0]), gy = fmaf(t, r.gd[1], r.og[1]),
                  gz = fmaf(t, r.gd[2], r.og[2]);
      in[q] = (r.i + j < N) && fminf(fminf(gx, gy), gz) >= 0.0f &&
              fmaxf(fmaxf(gx, gy), gz) <= kf;
      const int x = voxel_of(gx, kmax), y = voxel_of(gy, kmax), z = voxel_of(gz, kmax);
      const uint32_t bit = grid3((uint32_t)x >> c.oshift, (uint32_t)y >> c.oshift,
                                 (uint32_t)z >> c.oshift, (uint32_t)c.nbo);
      word[q] = __ldg(c.occ + (bit >> 5));
      bitpos[q] = bit & 31u;
      if (q == kSplitWin / 4 - 1 && sub == 3)
        dl = __ldg(c.dist + grid3((uint32_t)x >> c.dshift, (uint32_t)y >> c.dshift,
                                  (uint32_t)z >> c.dshift, (uint32_t)c.nbd));
    }
#pragma unroll
    for (int q = 0; q < kSplitWin / 4; ++q)
      part |= (uint32_t)(in[q] && ((word[q] >> bitpos[q]) & 1u)) << (sub + 4 * q);
  }
  uint32_t mask = quad_or(part);
  const uint32_t dlast = quad_from<3>(dl);
  int next = r.i + kSplitWin;
  if (dlast >= 2u) {
    const float run = fminf(((float)(dlast - 1u) * bedge - 0.5f) * r.inv_step, (float)N);
    next += (int)run;
  }
  uint32_t w[RW::nwords];
#pragma unroll
  for (int q = 0; q < RW::nwords; ++q) w[q] = 0u;
  while (mask != 0u && alive) {
    // this lane's sample: the (sub + 1)-th lowest set bit of the mask
    uint32_t m = mask;
#pragma unroll
    for (int q = 0; q < 3; ++q)
      if (q < sub) m &= m - 1u;
    const bool have = m != 0u;
    const int j = have ? __builtin_ctz(m) : 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) mask &= mask - 1u;
    float sd = 0.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    if (have) {
#pragma clang fp contract(off)
      const float t = (fi + ((float)j + 0.5f)) * dt;
      const float gx = fmaf(t, r.gd[0], r.og[0]), gy = fmaf(t, r.gd[1], r.og[1]),
                  gz = fmaf(t, r.gd[2], r.og[2]);
      load_record<FMT, MAXD>(c, record_offset(c, voxel_of(gx, kmax), voxel_of(gy, kmax),
                                              voxel_of(gz, kmax)),
                             w);
      const float sg = rec_sigma<FMT>(w, s0);
      rec_colour<FMT, MAXD>(w, r.cw, cr, cg, cb);
      sd = sg * dt;
    }
    // The round's transmittance steps first: every lane of the quad runs the
    // same optical-depth prefix over the four samples (a lane without a
    // sample sends -1), then each lane weighs only its own sample and the
    // weights and colours are gathered into the running sums in order. Each
    // value is the same expression as in ray_window, so the pixel is too.
    const float sdh = have ? sd : -1.0f;
    const float sdq[4] = {quad_from<0>(sdh), quad_from<1>(sdh), quad_from<2>(sdh),
                          quad_from<3>(sdh)};
    bool uq[4];
    float tq[4];
    {
#pragma clang fp contract(off)
      float tau = r.tau;
      bool al = alive;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uq[q] = !(sdq[q] < 0.0f) && al;
        tq[q] = tau;
        tau = tau + (uq[q] ? sdq[q] : 0.0f);
        al = al && !(tau > r.lim);
      }
      r.tau = tau;
      alive = al;
    }
    float wown;
    {
#pragma clang fp contract(off)
      const bool use = sub == 0 ? uq[0] : sub == 1 ? uq[1] : sub == 2 ? uq[2] : uq[3];
      const float t0 = sub == 0 ? tq[0] : sub == 1 ? tq[1] : sub == 2 ? tq[2] : tq[3];
      wown = exp_neg(t0) * opacity(use ? sd : 0.0f);
    }
    const float wq[4] = {quad_from<0>(wown), quad_from<1>(wown), quad_from<2>(wown),
                         quad_from<3>(wown)};
    const float crq[4] = {quad_from<0>(cr), quad_from<1>(cr), quad_from<2>(cr),
                          quad_from<3>(cr)};
    const float cgq[4] = {quad_from<0>(cg), quad_from<1>(cg), quad_from<2>(cg),
                          quad_from<3>(cg)};
    const float cbq[4] = {quad_from<0>(cb), quad_from<1>(cb), quad_from<2>(cb),
                          quad_from<3>(cb)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma clang fp contract(off)
      r.cr = fmaf(wq[q], uq[q] ? crq[q] : 0.0f, r.cr);
      r.cg = fmaf(wq[q], uq[q] ? cgq[q] : 0.0f, r.cg);
      r.cb = fmaf(wq[q], uq[q] ? cbq[q] : 0.0f, r.cb);
    }
  }
  if (alive) {
    r.i = next;
    if (r.i >= N) alive = false;
  }
}

// Renders the 16 rays of one 4x4 tile of a single view, four lanes per ray
// (lane l: ray l / 4, quarter l % 4): set-up (the same in the four lanes),
// the set-up jumps, split windows until the ray stops, the pixel (lane 0 of
// the quad). Dense caches with nearest lookups.
template <int FMT, int MAXD>
__device__ __forceinline__ void render_tile_split(const DevCache &c, const DevView &V, int lt,
                                                  int lane) {
  const int ray = lane >> 2, sub = lane & 3;
  int px, py;
  tile_pixel<4>(V, lt, ray & 3, ray >> 2, px, py);
  if (px >= V.W || py >= V.H) return;  // the whole quad
  Ray<FMT, MAXD> r;
  float beta[MAXD];
  bool alive = ray_setup<FMT, MAXD>(c, V, px, py, r, beta);
  if (alive) {
    uint32_t d = kSplitJumps > 0 ? sample_distance<FMT, MAXD>(c, r, 0) : 0u;
    ray_weights<FMT, MAXD>(c, beta, r);
    const float bedge = (float)(1 << c.dshift);
#pragma unroll
    for (int q = 0; q < kSplitJumps; ++q) {
      const int nx = skip_from(d, r.i, bedge, r.inv_step, r.N);
      d = 0u;
      if (nx != r.i) {
        r.i = nx;
        if (q + 1 < kSplitJumps && nx < r.N) d = sample_distance<FMT, MAXD>(c, r, nx);
      }
    }
    alive = r.i < r.N;
  }
  const float s0 = FMT == 3 ? c.scales[0] : 1.0f;
  while (alive) split_window<FMT, MAXD>(c, r, alive, s0, sub);
  if (sub == 0) ray_finish<FMT, MAXD>(c, r);
}

// Single views with split rays: each wave takes 4x4 tiles from its queue.
// FP32 and E4M3 are compiled for 4 waves per SIMD (single views 4-5% faster
// than at the 3 their registers would give); FP16 and BF16 reach 4 without
// the hint and were measured slower with it.
constexpr int split_waves(int fmt) {
  return FNR_SPLIT_WAVES > 0 ? FNR_SPLIT_WAVES : (fmt == 0 || fmt == 3 ? 4 : 1);
}
template <int FMT, int MAXD>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(split_waves(FMT)))) k_render_split(RenderArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  fill_outside(a);
  const Queue Q = make_queue(a, a.total_tiles);
  for (;;) {
    const int tile = queue_fetch(Q, lane);
    if (tile < 0) break;
    render_tile_split<FMT, MAXD>(a.c, a.v0, tile, lane);
  }
  queue_retire(Q, lane);
}

// Ray refill (the wave-level ray queue): a wave keeps its lanes busy across
// tiles instead of holding a tile until its slowest ray stops. After every
// window the wave takes a ballot of its live lanes; once at least kRefillMin
// lanes have retired their rays, it hands them rays from a per-wave pool in
// LDS, and when the pool is empty it takes the next tile from its queue, sets
// up that tile's 64 rays (one per lane, in parallel), writes the pixels of
// rays that miss the box, and compacts the others into the pool (ballot and
// prefix count). A ray is computed by one lane from set-up to pixel with the
// same arithmetic as in render_tile, so the image is bitwise the same; only
// the lane and the time at which a ray runs change.
#ifndef FNR_REFILL_MIN
#define FNR_REFILL_MIN 16
#endif
constexpr int kRefillMin = FNR_REFILL_MIN;

// Pool fields of a set-up ray (32-bit words): og[3], gd[3], dt, inv_step, N,
// lim, the pixel address (two words), beta[MAXD].
template <int MAXD> struct PoolFields {
  static constexpr int n = 12 + MAXD;
};

template <int FMT, int MAXD>
__device__ __forceinline__ void pool_put(uint32_t (*P)[kWave], int e, const Ray<FMT, MAXD> &r,
                                         const float *beta) {
  P[0][e] = __float_as_uint(r.og[0]);
  P[1][e] = __float_as_uint(r.og[1]);
  P[2][e] = __float_as_uint(r.og[2]);
  P[3][e] = __float_as_uint(r.gd[0]);
  P[4][e] = __float_as_uint(r.gd[1]);
  P[5][e] = __float_as_uint(r.gd[2]);
  P[6][e] = __float_as_uint(r.dt);
  P[7][e] = __float_as_uint(r.inv_step);
  P[8][e] = (uint32_t)r.N;
  P[9][e] = __float_as_uint(r.lim);
  const uint64_t op = reinterpret_cast<uint64_t>(r.out);
  P[10][e] = (uint32_t)op;
  P[11][e] = (uint32_t)(op >> 32);
#pragma unroll
  for (int d = 0; d < MAXD; ++d) P[12 + d][e] = __float_as_uint(beta[d]);
}

template <int FMT, int MAXD>
__device__ __forceinline__ void pool_get(const DevCache &c, uint32_t (*P)[kWave], int e,
                                         Ray<FMT, MAXD> &r) {
  r.og[0] = __uint_as_float(P[0][e]);
  r.og[1] = __uint_as_float(P[1][e]);
  r.og[2] = __uint_as_float(P[2][e]);
  r.gd[0] = __uint_as_float(P[3][e]);
  r.gd[1] = __uint_as_float(P[4][e]);
  r.gd[2] = __uint_as_float(P[5][e]);
  r.dt = __uint_as_float(P[6][e]);
  r.inv_step = __uint_as_float(P[7][e]);
  r.N = (int)P[8][e];
  r.lim = __uint_as_float(P[9][e]);
  r.out = reinterpret_cast<float4 *>((uint64_t)P[10][e] | ((uint64_t)P[11][e] << 32));
  float beta[MAXD];
#pragma unroll
  for (int d = 0; d < MAXD; ++d) beta[d] = __uint_as_float(P[12 + d][e]);
  ray_weights<FMT, MAXD>(c, beta, r);
  r.i = 0;
  r.tau = r.cr = r.cg = r.cb = 0.0f;
}

template <int FMT, int MAXD, bool LIN, bool SPARSE>
__device__ __forceinline__ void render_refill(const RenderArgs &a) {
  __shared__ uint32_t pool[kBlock / kWave][PoolFields<MAXD>::n][kWave];
  const int lane = threadIdx.x & (kWave - 1);
  uint32_t(*P)[kWave] = pool[threadIdx.x / kWave];
  const DevCache &c = a.c;
  fill_outside(a);
  const Queue Q = make_queue(a, a.total_tiles);
  const float s0 = FMT == 3 ? c.scales[0] : 1.0f;
  const uint64_t below = (1ull << lane) - 1ull;  // the lanes before this one
  Ray<FMT, MAXD> r;
  bool alive = false;
  int pend = 0;        // set-up rays waiting in the pool (wave-uniform)
  bool qdone = false;  // the wave's tile queue is empty (wave-uniform)
  for (;;) {
    uint64_t freem = __ballot(!alive);
    if (__popcll(freem) >= kRefillMin) {
      for (;;) {
        const int nfree = __popcll(freem);
        if (nfree == 0) break;
        if (pend == 0) {
          if (qdone) break;
          const int tile = queue_fetch(Q, lane);
          if (tile < 0) {
            qdone = true;
            break;
          }
          int lt = tile;
          const DevView V = a.views ? a.views[batch_tile(a, tile, lt)] : a.v0;
          int px, py;
          tile_pixel<8>(V, lt, lane & 7, lane >> 3, px, py);
          bool march = false;
          Ray<FMT, MAXD> nr;
          float beta[MAXD];
          if (px < V.W && py < V.H) {
            march = ray_setup<FMT, MAXD>(c, V, px, py, nr, beta);
            if (!march) ray_finish<FMT, MAXD>(c, nr);  // the background
          }
          const uint64_t m = __ballot(march);
          if (march) pool_put<FMT, MAXD>(P, __popcll(m & below), nr, beta);
          pend = __popcll(m);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          continue;
        }
        // free lanes take the pool's last entries
        const int take = min(nfree, pend);
        const int rank = __popcll(freem & below);
        if (!alive && rank < take) {
          pool_get<FMT, MAXD>(c, P, pend - 1 - rank, r);
          alive = true;
        }
        pend -= take;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        freem = __ballot(!alive);
      }
    }
    if (__ballot(alive) == 0ull) break;  // queue empty, pool empty, every ray done
    const bool was = alive;
    ray_window<FMT, MAXD, LIN, SPARSE>(c, r, alive, s0);
    if (was && !alive) ray_finish<FMT, MAXD>(c, r);
  }
  queue_retire(Q, lane);
}

// Waves per SIMD of the LDS-staged tile kernel and its records in flight per
// lane: FP32 holds two records at 3 waves per SIMD (with the loads issued at
// raised priority, 3-4% faster than one record at 4 waves); the others as
// k_render.
#ifndef FNR_LDS_WAVES_F32
#define FNR_LDS_WAVES_F32 3
#endif
#ifndef FNR_LOCC_BATCH_F32
#define FNR_LOCC_BATCH_F32 2
#endif
#ifndef FNR_LOCC_BATCH_F16
#define FNR_LOCC_BATCH_F16 FNR_BATCH_F16
#endif
#ifndef FNR_LOCC_BATCH_F8
#define FNR_LOCC_BATCH_F8 FNR_BATCH_F8
#endif
template <int FMT, bool LIN> struct LoccBatch {
  static constexpr int value =
      LIN ? Batch<FMT, LIN>::value
          : (FMT == 0 ? FNR_LOCC_BATCH_F32 : (FMT == 3 ? FNR_LOCC_BATCH_F8 : FNR_LOCC_BATCH_F16));
};
#ifndef FNR_LDS_WAVES_F16
#define FNR_LDS_WAVES_F16 4
#endif
#ifndef FNR_LDS_WAVES_F8
#define FNR_LDS_WAVES_F8 3
#endif
constexpr int lds_waves(int fmt) {
  return fmt == 0 ? FNR_LDS_WAVES_F32 : (fmt == 3 ? FNR_LDS_WAVES_F8 : FNR_LDS_WAVES_F16);
}

// Waves per SIMD asked of the compiler for the dense render kernel: FP32,
// FP16 and BF16 nearest lookups with up to 8 components keep 4 (FP16 9%
// faster for batched launches than the 3 it would get; FP32 needs two
// registers fewer than its unconstrained build), E4M3 keeps 3; the others are
// left to the compiler.
constexpr int render_waves(int fmt, int maxd, bool lin) {
  return maxd <= 8 && !lin ? (fmt == 3 ? 3 : 4) : 1;
}

template <int FMT, int MAXD, bool LIN>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(render_waves(FMT, MAXD, LIN))))
    k_render(RenderArgs a) {
  render_queue<FMT, MAXD, LIN, false>(a);
}

// The same with more records in flight per lane (WideBatch), for launches
// with few tiles.
template <int FMT, int MAXD, bool LIN>
__global__ void __launch_bounds__(kBlock) k_render_wide(RenderArgs a) {
  render_queue<FMT, MAXD, LIN, false, WideBatch<FMT, LIN>::value>(a);
}

// The tile kernel with the occupancy bitgrid staged in LDS: one block of
// lds_waves waves per SIMD fills a CU, copies the bitgrid words (at most
// kOccLdsWords, checked by the host; the buffer is padded to 16 bytes) into
// LDS once, then takes tiles from its queues as k_render does. The sixteen
// occupancy tests of every window become LDS reads instead of vector-memory
// loads, which leaves the memory pipeline to the record gathers. (Measured:
// 3-6% faster batched launches for FP32 and FP16, 2% for E4M3; the wide
// kernel of single views was slower with it, so it reads the bitgrid from
// memory.)
template <int FMT, int MAXD, bool LIN>
__global__ void __launch_bounds__(kWave * 4 * lds_waves(FMT))
    __attribute__((amdgpu_waves_per_eu(lds_waves(FMT), lds_waves(FMT))))
    k_render_locc(RenderArgs a) {
  __shared__ uint4 locc4[kOccLdsWords / 4];
  const int n4 = (a.c.occ_words + 3) >> 2;
  const uint4 *src = reinterpret_cast<const uint4 *>(a.c.occ);
  const int nt = (int)blockDim.x;
  for (int i0 = (int)threadIdx.x; i0 < n4; i0 += 4 * nt) {
    uint4 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (i0 + q * nt < n4) v[q] = src[i0 + q * nt];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (i0 + q * nt < n4) locc4[i0 + q * nt] = v[q];
  }
  __syncthreads();
  render_queue<FMT, MAXD, LIN, false, LoccBatch<FMT, LIN>::value, true>(
      a, reinterpret_cast<const uint32_t *>(locc4));
}

// The same over the refill schedule (wave-level ray queue), compiled for 4
// waves per SIMD with nearest lookups in FP32/FP16/BF16 and up to 8 components
// and 3 in E4M3 (as the tile kernel runs).
constexpr int refill_waves(int fmt, int maxd, bool lin) {
  return maxd <= 8 && !lin ? (fmt == 3 ? 3 : 4) : 1;
}
template <int FMT, int MAXD, bool LIN>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(refill_waves(FMT, MAXD, LIN))))
    k_render_refill(RenderArgs a) {
  render_refill<FMT, MAXD, LIN, false>(a);
}

// The brick-sparse render kernel. Its slot arithmetic holds one more register
// per window sample; W waves per SIMD are asked of the compiler so that it
// keeps the dense kernel's occupancy (a few spilled bytes at most), which
// measured faster for batched launches and no slower for single views than
// the unconstrained build.
template <int FMT, int MAXD, int W>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(W, W)))
k_render_sparse(RenderArgs a) {
  render_queue<FMT, MAXD, false, true>(a);
}
template <int FMT, int MAXD, int W>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(W, W)))
k_render_sparse_refill(RenderArgs a) {
  render_refill<FMT, MAXD, false, true>(a);
}
template <int FMT, int MAXD>
__global__ void __launch_bounds__(kBlock) k_render_sparse_wide(RenderArgs a) {
  render_queue<FMT, MAXD, false, true, WideBatch<FMT, false>::value>(a);
}
constexpr int sparse_waves(int fmt, int maxd) { return maxd == 16 ? 2 : (fmt == 3 ? 3 : 4); }

// Voxel traversal (N = 0) over single views or a batch of views.
template <int FMT, int MAXD>
__global__ void __launch_bounds__(kBlock) k_render_vox(RenderArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  fill_outside(a);
  const Queue Q = make_queue(a, a.total_tiles);
  for (;;) {
    const int tile = queue_fetch(Q, lane);
    if (tile < 0) break;
    if (a.views) {
      int lt;
      const DevView V = a.views[batch_tile(a, tile, lt)];
      render_tile_vox<FMT, MAXD>(a, a.c, V, lt, lane);
    } else {
      render_tile_vox<FMT, MAXD>(a, a.c, a.v0, tile, lane);
    }
  }
  queue_retire(Q, lane);
}

// Serving step: tile ranges of many views over several resident caches of one
// storage format, in one launch (one per format present); the step's size is
// read from device memory so the launch can be replayed from a captured graph.
// Compiled for the waves per SIMD of the batched kernel of the same format.
template <int FMT, int MAXD, bool LIN>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(render_waves(FMT, MAXD, LIN))))
    k_render_step(RenderArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int total = __builtin_amdgcn_readfirstlane(a.dyn_total[0]);
  const int nviews = __builtin_amdgcn_readfirstlane(a.dyn_total[1]);
  const Queue Q = make_queue(a, total);
  for (;;) {
    const int tile = queue_fetch(Q, lane);
    if (tile < 0) break;
    const DevView V = a.views[view_of_tile(a, tile, nviews)];
    const DevCache c = a.caches[V.scene];
    render_tile<FMT, MAXD, LIN>(a, c, V, tile - V.tile_begin + V.tile_offset, lane);
  }
  queue_retire(Q, lane);
}

// ------------------------------------------------------------------ cache build

__device__ inline uint32_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7F800000u) == 0x7F800000u) return (u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return u >> 16;
}

// OCP E4M3 ("fn": bias 7, no infinities, 0x7F is NaN), round to nearest even,
// saturating at 448.
__device__ inline uint32_t f32_to_e4m3_sat(float y) {
  const uint32_t sgn = (__float_as_uint(y) >> 24) & 0x80u;
  const float a = fabsf(y);
  if (!(a < 448.0f)) return sgn | (a != a ? 0x7Fu : 0x7Eu);
  if (a < 0.015625f) {  // below 2^-6: multiples of 2^-9 (q = 8 carries into the first normal)
    return sgn | (uint32_t)rintf(a * 512.0f);
  }
  const int e = (int)((__float_as_uint(a) >> 23) & 0xFF) - 127;  // 2^e <= a < 2^(e+1)
  const uint32_t q = (uint32_t)rintf(ldexpf(a, 3 - e));          // 8..16, exact scaling
  return sgn | ((uint32_t)(e + 7) << 3) + (q - 8u);
}

__global__ void k_absmax(const float *__restrict__ sigma, const float *__restrict__ u,
                         int64_t nvox, int D, unsigned *__restrict__ amax) {
  const int nch = 1 + 3 * D;
  float m[kMaxCh];
#pragma unroll
  for (int j = 0; j < kMaxCh; ++j) m[j] = 0.0f;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox;
       v += (int64_t)gridDim.x * blockDim.x) {
    m[0] = fmaxf(m[0], fabsf(sigma[v]));
#pragma unroll
    for (int j = 1; j < kMaxCh; ++j)
      if (j < nch) m[j] = fmaxf(m[j], fabsf(u[v * (nch - 1) + (j - 1)]));
  }
  __shared__ float red[kBlock / kWave][kMaxCh];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
  for (int j = 0; j < kMaxCh; ++j) {
    if (j >= nch) break;
    float x = m[j];
    for (int off = kWave / 2; off > 0; off >>= 1) x = fmaxf(x, __shfl_xor(x, off));
    if (lane == 0) red[wv][j] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < nch) {
    float x = 0.0f;
    for (int q = 0; q < kBlock / kWave; ++q) x = fmaxf(x, red[q][threadIdx.x]);
    atomicMax(amax + threadIdx.x, __float_as_uint(x));  // non-negative floats order as ints
  }
}

// Sets n words to v (queue counters that must start at zero; a kernel rather
// than a memset so that a captured graph replays it reliably).
__global__ void k_fill_u32(unsigned *p, int n, unsigned v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_make_scales(const unsigned *amax, int nch, float *scales) {
  const int j = threadIdx.x;
  if (j < nch) {
    const float a = __uint_as_float(amax[j]);
    scales[j] = a > 0.0f ? __fdiv_rn(a, 448.0f) : 1.0f;
  }
}

// Brick-sparse caches: flags[b] = 1 for every 8^3 brick b holding a voxel of
// the slab with sigma > 0 (a brick without one is empty to the bitgrid too).
__global__ void k_brick_flags(const float *__restrict__ sigma, int z0, int nz, int k, int nbl,
                              uint32_t *__restrict__ flags) {
  const int64_t nvox = (int64_t)nz * k * k;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox;
       v += (int64_t)gridDim.x * blockDim.x) {
    if (!(sigma[v] > 0.0f)) continue;
    const int x = (int)(v % k), y = (int)((v / k) % k), z = z0 + (int)(v / ((int64_t)k * k));
    flags[((uint32_t)(z >> 3) * (uint32_t)nbl + (uint32_t)(y >> 3)) * (uint32_t)nbl +
          (uint32_t)(x >> 3)] = 1u;
  }
}

template <int FMT>
__global__ void k_pack(const float *__restrict__ sigma, const float *__restrict__ u, int z0,
                       int nz, DevCache c, float *scales_unused) {
  (void)scales_unused;
  const int k = c.k, D = c.D, nch = 1 + 3 * D;
  const int64_t nvox = (int64_t)nz * k * k;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(v % k), y = (int)((v / k) % k), z = z0 + (int)(v / ((int64_t)k * k));
    if (c.slot && c.slot[((uint32_t)(z >> 3) * (uint32_t)c.nbl + (uint32_t)(y >> 3)) *
                             (uint32_t)c.nbl + (uint32_t)(x >> 3)] == 0)
      continue;  // brick-sparse: the brick is not stored (it reads as zero)
    uint32_t w[(kMaxCh * 4 + 15) / 16 * 4];
#pragma unroll
    for (int q = 0; q < (int)(sizeof(w) / 4); ++q) w[q] = 0u;
#pragma unroll
    for (int j = 0; j < kMaxCh; ++j) {
      if (j >= nch) break;
      const float x32 = j == 0 ? sigma[v] : u[v * (nch - 1) + (j - 1)];
      if (FMT == 0) {
        w[j] = __float_as_uint(x32);
      } else if (FMT == 1) {
        const uint32_t h = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x32);
        w[j >> 1] |= h << ((j & 1) * 16);
      } else if (FMT == 2) {
        w[j >> 1] |= f32_to_bf16_rne(x32) << ((j & 1) * 16);
      } else {
        const uint32_t q8 = f32_to_e4m3_sat(__fdiv_rn(x32, c.scales[j]));
        w[j >> 2] |= q8 << ((j & 3) * 8);
      }
    }
    u32x4 *dst = reinterpret_cast<u32x4 *>(const_cast<uint8_t *>(c.rec) +
                                           record_offset(c, x, y, z));
#pragma unroll
    for (int q = 0; q < (int)(sizeof(w) / 16); ++q)
      if (q < c.nchunk) dst[q] = u32x4{w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]};
  }
}

template <int FMT>
__device__ inline float stored_sigma(const DevCache &c, int x, int y, int z) {
  const uint32_t *p = reinterpret_cast<const uint32_t *>(c.rec + record_offset(c, x, y, z));
  uint32_t w[1] = {p[0]};
  return Fmt<FMT>::get(w, 0);  // sign and zero test only: the scale is positive
}

// one thread per brick; dilate = 1 widens the brick by one voxel on every side
template <int FMT>
__global__ void k_occupancy(DevCache c, int dilate, uint32_t *__restrict__ words) {
  const int nb = c.nbo, e = 1 << c.oshift, k = c.k;
  const int64_t nbr = (int64_t)nb * nb * nb;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nbr;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int bx = (int)(b % nb), by = (int)((b / nb) % nb), bz = (int)(b / ((int64_t)nb * nb));
    const int x0 = max(bx * e - dilate, 0), x1 = min(bx * e + e + dilate, k);
    const int y0 = max(by * e - dilate, 0), y1 = min(by * e + e + dilate, k);
    const int z0 = max(bz * e - dilate, 0), z1 = min(bz * e + e + dilate, k);
    bool any = false;
    for (int z = z0; z < z1 && !any; ++z)
      for (int y = y0; y < y1 && !any; ++y)
        for (int x = x0; x < x1; ++x)
          if (stored_sigma<FMT>(c, x, y, z) > 0.0f) {
            any = true;
            break;
          }
    if (any) atomicOr(words + (b >> 5), 1u << (b & 31));
  }
}

// Brick distance field, step 1: 0 for occupied bricks, kDistCap otherwise.
// Initial distance of each distance brick: 0 when any of the ratio^3 bitgrid
// bricks it holds is set, kDistCap otherwise (nbo = nbd * ratio).
__global__ void k_dist_init(const uint32_t *__restrict__ words, int nbd, int nbo, int ratio,
                            uint8_t *__restrict__ out) {
  const int64_t nbr = (int64_t)nbd * nbd * nbd;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nbr;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int bx = (int)(b % nbd), by = (int)((b / nbd) % nbd), bz = (int)(b / ((int64_t)nbd * nbd));
    bool any = false;
    for (int dz = 0; dz < ratio && !any; ++dz)
      for (int dy = 0; dy < ratio && !any; ++dy)
        for (int dx = 0; dx < ratio && !any; ++dx) {
          const int64_t f = ((int64_t)(bz * ratio + dz) * nbo + (by * ratio + dy)) * nbo +
                            (bx * ratio + dx);
          any = (words[f >> 5] >> (f & 31)) & 1u;
        }
    out[b] = any ? 0 : kDistCap;
  }
}

// One axis of the Chebyshev (max-norm) distance transform, which separates:
// out(i) = min over |i - j| <= kDistCap of max(|i - j|, in(j)) along the axis.
// Applied along x, y and z in turn to the step-1 field it yields, for every
// brick, min(kDistCap, max-norm distance in bricks to the nearest occupied one).
__global__ void k_dist_axis(const uint8_t *__restrict__ in, uint8_t *__restrict__ out, int nb,
                            int axis) {
  const int64_t nbr = (int64_t)nb * nb * nb;
  const int64_t stride = axis == 0 ? 1 : (axis == 1 ? nb : (int64_t)nb * nb);
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nbr;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)((b / stride) % nb);
    const int64_t base = b - (int64_t)i * stride;
    int best = in[b];
    for (int dd = 1; dd < best; ++dd) {  // offsets >= best cannot lower it
      if (i - dd >= 0) best = min(best, max(dd, (int)in[base + (int64_t)(i - dd) * stride]));
      if (i + dd < nb) best = min(best, max(dd, (int)in[base + (int64_t)(i + dd) * stride]));
    }
    out[b] = (uint8_t)best;
  }
}

template <int FMT, int MAXD>
__global__ void k_readback(DevCache c, float *__restrict__ sigma, float *__restrict__ u) {
  using RW = RecWords<FMT, MAXD>;
  const int k = c.k, D = c.D;
  const int64_t nvox = (int64_t)k * k * k;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(v % k), y = (int)((v / k) % k), z = (int)(v / ((int64_t)k * k));
    uint32_t w[RW::nwords];
    load_record<FMT, MAXD>(c, record_offset(c, x, y, z), w);
#pragma unroll
    for (int j = 0; j < 1 + 3 * MAXD; ++j) {
      if (j >= 1 + 3 * D) break;
      float val = Fmt<FMT>::get(w, j);
      if (FMT == 3) val *= c.scales[j];
      if (j == 0) sigma[v] = val; else u[v * 3 * D + (j - 1)] = val;
    }
  }
}

template <int FMT, int MAXD, bool LIN>
__global__ void k_lookup(DevCache c, int n, const float *__restrict__ pts,
                         const float *__restrict__ dirs, float *__restrict__ su,
                         float *__restrict__ bo) {
  using RW = RecWords<FMT, MAXD>;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int D = c.D, k = c.k;
  float sc[kMaxCh];
#pragma unroll
  for (int j = 0; j < kMaxCh; ++j) sc[j] = (FMT == 3 && j < 1 + 3 * D) ? c.scales[j] : 1.0f;
  if (dirs && bo) {
    float beta[MAXD];
    dir_lookup<MAXD>(c, dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2], beta);
#pragma unroll
    for (int d = 0; d < MAXD; ++d)
      if (d < D) bo[(size_t)q * D + d] = beta[d];
  }
  if (!pts || !su) return;
  float g[3];
  bool inside = true;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    g[ax] = (pts[3 * q + ax] - c.bmin[ax]) * c.inv_h[ax];
    inside = inside && g[ax] >= 0.0f && g[ax] <= c.kf;
  }
  float acc[kMaxCh];
#pragma unroll
  for (int j = 0; j < kMaxCh; ++j) acc[j] = 0.0f;
  if (inside) {
    for (int corner = 0; corner < (LIN ? 8 : 1); ++corner) {
      int v[3];
      float wt = 1.0f;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        if (LIN) {
          const float h = g[ax] - 0.5f, f = floorf(h);
          const int bit = (corner >> ax) & 1;
          v[ax] = min(max((int)f + bit, 0), k - 1);
          wt *= bit ? h - f : 1.0f - (h - f);
        } else {
          v[ax] = min((int)(g[ax] + kTie), k - 1);
        }
      }
      uint32_t w[RW::nwords];
      load_record<FMT, MAXD>(c, record_offset(c, v[0], v[1], v[2]), w);
#pragma unroll
      for (int j = 0; j < 1 + 3 * MAXD; ++j) acc[j] = fmaf(wt, Fmt<FMT>::get(w, j) * sc[j], acc[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < 1 + 3 * MAXD; ++j)
    if (j < 1 + 3 * D) su[(size_t)q * (1 + 3 * D) + j] = acc[j];
}

// ------------------------------------------------------------------ launchers

namespace {

// The render kernel of a launch: schedule (kSchedTiles, kSchedRefill,
// kSchedWide), cache kind (dense or brick-sparse) and, for the tile schedule,
// whether the bitgrid is staged in LDS (locc).
template <int FMT, int MAXD, bool LIN>
const void *render_kernel(int sched, bool sparse, bool locc = false) {
  if constexpr (!LIN && MAXD <= 8) {
    if (locc && !sparse && sched == kSchedTiles)
      return (const void *)k_render_locc<FMT, MAXD, LIN>;
  }
  if constexpr (!LIN) {
    if (sparse) {
      if (sched == kSchedRefill)
        return (const void *)k_render_sparse_refill<FMT, MAXD, sparse_waves(FMT, MAXD)>;
      if (sched == kSchedWide) return (const void *)k_render_sparse_wide<FMT, MAXD>;
      return (const void *)k_render_sparse<FMT, MAXD, sparse_waves(FMT, MAXD)>;
    }
  }
  if constexpr (!LIN && MAXD <= 8) {
    if (sched == kSchedSplit && !sparse) return (const void *)k_render_split<FMT, MAXD>;
  }
  if (sched == kSchedRefill) return (const void *)k_render_refill<FMT, MAXD, LIN>;
  if (sched == kSchedWide) return (const void *)k_render_wide<FMT, MAXD, LIN>;
  return (const void *)k_render<FMT, MAXD, LIN>;
}

template <int FMT, int MAXD, bool LIN>
hipError_t launch_render_t(const RenderArgs &a, int grid, int block, bool locc, hipStream_t s) {
  const void *k = render_kernel<FMT, MAXD, LIN>(a.sched, a.c.slot != nullptr, locc);
  RenderArgs arg = a;
  void *args[] = {&arg};
  return hipLaunchKernel(k, dim3(grid), dim3(block), args, 0, s);
}

// Resident blocks per CU of the render kernel of a schedule and cache kind.
template <int FMT, int MAXD, bool LIN>
int occupancy_t(bool sparse, int sched, int block, bool locc) {
  int nb = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &nb, render_kernel<FMT, MAXD, LIN>(sched, sparse, locc), block, 0);
  return (e != hipSuccess || nb < 1) ? 1 : nb;
}

template <int FMT, bool LIN>
hipError_t dispatch_maxd(int D, const RenderArgs *a, int grid, int block, bool locc,
                         hipStream_t s, bool sparse, int sched, int *occ) {
  if (D <= 4) return a ? launch_render_t<FMT, 4, LIN>(*a, grid, block, locc, s) : (*occ = occupancy_t<FMT, 4, LIN>(sparse, sched, block, locc), hipSuccess);
  if (D <= 8) return a ? launch_render_t<FMT, 8, LIN>(*a, grid, block, locc, s) : (*occ = occupancy_t<FMT, 8, LIN>(sparse, sched, block, locc), hipSuccess);
  return a ? launch_render_t<FMT, 16, LIN>(*a, grid, block, locc, s) : (*occ = occupancy_t<FMT, 16, LIN>(sparse, sched, block, locc), hipSuccess);
}

template <int FMT>
hipError_t dispatch_lin(bool lin, int D, const RenderArgs *a, int grid, int block, bool locc,
                        hipStream_t s, bool sparse, int sched, int *occ) {
  return lin ? dispatch_maxd<FMT, true>(D, a, grid, block, locc, s, sparse, sched, occ)
             : dispatch_maxd<FMT, false>(D, a, grid, block, locc, s, sparse, sched, occ);
}

hipError_t dispatch(int fmt, bool lin, int D, const RenderArgs *a, int grid, int block,
                    bool locc, hipStream_t s, bool sparse, int sched, int *occ) {
  switch (fmt) {
    case 0: return dispatch_lin<0>(lin, D, a, grid, block, locc, s, sparse, sched, occ);
    case 1: return dispatch_lin<1>(lin, D, a, grid, block, locc, s, sparse, sched, occ);
    case 2: return dispatch_lin<2>(lin, D, a, grid, block, locc, s, sparse, sched, occ);
    default: return dispatch_lin<3>(lin, D, a, grid, block, locc, s, sparse, sched, occ);
  }
}

template <int FMT>
hipError_t launch_lookup_f(const DevCache &c, bool lin, int n, const float *pts,
                           const float *dirs, float *su, float *bo, hipStream_t s) {
  const int grid = (n + kBlock - 1) / kBlock;
  if (c.D <= 4) {
    if (lin) hipLaunchKernelGGL((k_lookup<FMT, 4, true>), dim3(grid), dim3(kBlock), 0, s, c, n, pts, dirs, su, bo);
    else hipLaunchKernelGGL((k_lookup<FMT, 4, false>), dim3(grid), dim3(kBlock), 0, s, c, n, pts, dirs, su, bo);
  } else if (c.D <= 8) {
    if (lin) hipLaunchKernelGGL((k_lookup<FMT, 8, true>), dim3(grid), dim3(kBlock), 0, s, c, n, pts, dirs, su, bo);
    else hipLaunchKernelGGL((k_lookup<FMT, 8, false>), dim3(grid), dim3(kBlock), 0, s, c, n, pts, dirs, su, bo);
  } else {
    if (lin) hipLaunchKernelGGL((k_lookup<FMT, 16, true>), dim3(grid), dim3(kBlock), 0, s, c, n, pts, dirs, su, bo);
    else hipLaunchKernelGGL((k_lookup<FMT, 16, false>), dim3(grid), dim3(kBlock), 0, s, c, n, pts, dirs, su, bo);
  }
  return hipGetLastError();
}

template <int FMT>
hipError_t launch_readback_f(const DevCache &c, float *sigma, float *u, hipStream_t s) {
  const int grid = 2048;
  if (c.D <= 4) hipLaunchKernelGGL((k_readback<FMT, 4>), dim3(grid), dim3(kBlock), 0, s, c, sigma, u);
  else if (c.D <= 8) hipLaunchKernelGGL((k_readback<FMT, 8>), dim3(grid), dim3(kBlock), 0, s, c, sigma, u);
  else hipLaunchKernelGGL((k_readback<FMT, 16>), dim3(grid), dim3(kBlock), 0, s, c, sigma, u);
  return hipGetLastError();
}

}  // namespace

namespace {

template <int FMT, int MAXD>
hipError_t launch_step_t(bool lin, const RenderArgs &a, int grid, hipStream_t s) {
  if (lin) hipLaunchKernelGGL((k_render_step<FMT, MAXD, true>), dim3(grid), dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((k_render_step<FMT, MAXD, false>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int FMT, int MAXD>
int step_occupancy_t(bool lin) {
  int nb = 0;
  const hipError_t e =
      lin ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_render_step<FMT, MAXD, true>,
                                                         kBlock, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_render_step<FMT, MAXD, false>,
                                                         kBlock, 0);
  return (e != hipSuccess || nb < 1) ? 1 : nb;
}

// The kernel for (format, lookup, component-count class); a null launch
// argument asks for the resident blocks per CU instead.
template <int FMT>
hipError_t step_dispatch(bool lin, int D, const RenderArgs *a, int grid, hipStream_t s, int *occ) {
  switch (maxd_class(D)) {
    case 4: return a ? launch_step_t<FMT, 4>(lin, *a, grid, s) : (*occ = step_occupancy_t<FMT, 4>(lin), hipSuccess);
    case 8: return a ? launch_step_t<FMT, 8>(lin, *a, grid, s) : (*occ = step_occupancy_t<FMT, 8>(lin), hipSuccess);
    default: return a ? launch_step_t<FMT, 16>(lin, *a, grid, s) : (*occ = step_occupancy_t<FMT, 16>(lin), hipSuccess);
  }
}

hipError_t step_dispatch_fmt(int fmt, bool lin, int D, const RenderArgs *a, int grid,
                             hipStream_t s, int *occ) {
  switch (fmt) {
    case 0: return step_dispatch<0>(lin, D, a, grid, s, occ);
    case 1: return step_dispatch<1>(lin, D, a, grid, s, occ);
    case 2: return step_dispatch<2>(lin, D, a, grid, s, occ);
    default: return step_dispatch<3>(lin, D, a, grid, s, occ);
  }
}

}  // namespace

// fmt and D select the kernel's storage format and component-count class
// (maxd_class), which must be those of every cache of the step.
hipError_t launch_render_step(int fmt, bool lin, int D, const RenderArgs &a, int grid,
                              hipStream_t s) {
  return step_dispatch_fmt(fmt, lin, D, &a, grid, s, nullptr);
}

int render_step_occupancy(int fmt, bool lin, int D) {
  int occ = 1;
  (void)step_dispatch_fmt(fmt, lin, D, nullptr, 0, nullptr, &occ);
  return occ;
}

#ifndef FNR_LOCC
#define FNR_LOCC 1
#endif

bool render_locc(int fmt, bool lin, int D, bool sparse, int sched, int occ_words) {
  (void)fmt;
  return FNR_LOCC && !lin && !sparse && D <= 8 && sched == kSchedTiles &&
         occ_words <= kOccLdsWords;
}

int render_block(int fmt, bool lin, int D, bool sparse, int sched, int occ_words) {
  return render_locc(fmt, lin, D, sparse, sched, occ_words) ? kWave * 4 * lds_waves(fmt)
                                                            : kBlock;
}

int render_occupancy(int fmt, bool lin, int D, bool sparse, int sched, int occ_words) {
  int occ = 0;
  (void)dispatch(fmt, lin, D, nullptr, 0, render_block(fmt, lin, D, sparse, sched, occ_words),
                 render_locc(fmt, lin, D, sparse, sched, occ_words), nullptr, sparse, sched,
                 &occ);
  return occ;
}

hipError_t launch_render(int fmt, bool lin, const RenderArgs &a, int grid, hipStream_t s) {
  const bool sparse = a.c.slot != nullptr;
  const int block = render_block(fmt, lin, a.c.D, sparse, a.sched, a.c.occ_words);
  const bool locc = render_locc(fmt, lin, a.c.D, sparse, a.sched, a.c.occ_words);
  return dispatch(fmt, lin, a.c.D, &a, grid, block, locc, s, sparse, a.sched, nullptr);
}

namespace {

template <int FMT, int MAXD>
hipError_t vox_t(const RenderArgs *a, int grid, hipStream_t s, int *occ) {
  if (a) {
    hipLaunchKernelGGL((k_render_vox<FMT, MAXD>), dim3(grid), dim3(kBlock), 0, s, *a);
    return hipGetLastError();
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_render_vox<FMT, MAXD>, kBlock, 0) !=
      hipSuccess)
    nb = 1;
  *occ = nb < 1 ? 1 : nb;
  return hipSuccess;
}

template <int FMT>
hipError_t vox_d(int D, const RenderArgs *a, int grid, hipStream_t s, int *occ) {
  switch (maxd_class(D)) {
    case 4: return vox_t<FMT, 4>(a, grid, s, occ);
    case 8: return vox_t<FMT, 8>(a, grid, s, occ);
    default: return vox_t<FMT, 16>(a, grid, s, occ);
  }
}

hipError_t vox_dispatch(int fmt, int D, const RenderArgs *a, int grid, hipStream_t s, int *occ) {
  switch (fmt) {
    case 0: return vox_d<0>(D, a, grid, s, occ);
    case 1: return vox_d<1>(D, a, grid, s, occ);
    case 2: return vox_d<2>(D, a, grid, s, occ);
    default: return vox_d<3>(D, a, grid, s, occ);
  }
}

}  // namespace

int render_vox_occupancy(int fmt, int D) {
  int occ = 1;
  (void)vox_dispatch(fmt, D, nullptr, 0, nullptr, &occ);
  return occ;
}

hipError_t launch_render_vox(int fmt, const RenderArgs &a, int grid, hipStream_t s) {
  return vox_dispatch(fmt, a.c.D, &a, grid, s, nullptr);
}

hipError_t launch_absmax(const float *sigma, const float *u, int64_t nvox, int D, unsigned *amax,
                         hipStream_t s) {
  int64_t blocks = (nvox + kBlock - 1) / kBlock;
  const int grid = (int)(blocks < 1024 ? (blocks < 1 ? 1 : blocks) : 1024);
  hipLaunchKernelGGL(k_absmax, dim3(grid), dim3(kBlock), 0, s, sigma, u, nvox, D, amax);
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, int n, unsigned v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_make_scales(const unsigned *amax, int nch, float *scales, hipStream_t s) {
  hipLaunchKernelGGL(k_make_scales, dim3(1), dim3(64), 0, s, amax, nch, scales);
  return hipGetLastError();
}

hipError_t launch_pack(int fmt, const float *sigma, const float *u, int z0, int nz,
                       const DevCache &c, hipStream_t s) {
  const int64_t nvox = (int64_t)nz * c.k * c.k;
  int64_t blocks = (nvox + kBlock - 1) / kBlock;
  const int grid = (int)(blocks < 65536 ? (blocks < 1 ? 1 : blocks) : 65536);
  switch (fmt) {
    case 0: hipLaunchKernelGGL(k_pack<0>, dim3(grid), dim3(kBlock), 0, s, sigma, u, z0, nz, c, nullptr); break;
    case 1: hipLaunchKernelGGL(k_pack<1>, dim3(grid), dim3(kBlock), 0, s, sigma, u, z0, nz, c, nullptr); break;
    case 2: hipLaunchKernelGGL(k_pack<2>, dim3(grid), dim3(kBlock), 0, s, sigma, u, z0, nz, c, nullptr); break;
    default: hipLaunchKernelGGL(k_pack<3>, dim3(grid), dim3(kBlock), 0, s, sigma, u, z0, nz, c, nullptr); break;
  }
  return hipGetLastError();
}

hipError_t launch_occupancy(int fmt, const DevCache &c, int dilate, uint32_t *words,
                            hipStream_t s) {
  const int64_t nbr = (int64_t)c.nbo * c.nbo * c.nbo;
  int64_t blocks = (nbr + kBlock - 1) / kBlock;
  const int grid = (int)(blocks < 65536 ? (blocks < 1 ? 1 : blocks) : 65536);
  switch (fmt) {
    case 0: hipLaunchKernelGGL(k_occupancy<0>, dim3(grid), dim3(kBlock), 0, s, c, dilate, words); break;
    case 1: hipLaunchKernelGGL(k_occupancy<1>, dim3(grid), dim3(kBlock), 0, s, c, dilate, words); break;
    case 2: hipLaunchKernelGGL(k_occupancy<2>, dim3(grid), dim3(kBlock), 0, s, c, dilate, words); break;
    default: hipLaunchKernelGGL(k_occupancy<3>, dim3(grid), dim3(kBlock), 0, s, c, dilate, words); break;
  }
  return hipGetLastError();
}

hipError_t launch_brick_flags(const float *sigma, int z0, int nz, int k, int nbl,
                              uint32_t *flags, hipStream_t s) {
  const int64_t nvox = (int64_t)nz * k * k;
  int64_t blocks = (nvox + kBlock - 1) / kBlock;
  const int grid = (int)(blocks < 65536 ? (blocks < 1 ? 1 : blocks) : 65536);
  hipLaunchKernelGGL(k_brick_flags, dim3(grid), dim3(kBlock), 0, s, sigma, z0, nz, k, nbl, flags);
  return hipGetLastError();
}

hipError_t launch_distance(const DevCache &c, const uint32_t *words, uint8_t *dist, uint8_t *tmp,
                           hipStream_t s) {
  const int nb = c.nbd;
  const int64_t nbr = (int64_t)nb * nb * nb;
  int64_t blocks = (nbr + kBlock - 1) / kBlock;
  const int grid = (int)(blocks < 65536 ? (blocks < 1 ? 1 : blocks) : 65536);
  hipLaunchKernelGGL(k_dist_init, dim3(grid), dim3(kBlock), 0, s, words, nb, c.nbo,
                     1 << (c.dshift - c.oshift), tmp);
  hipLaunchKernelGGL(k_dist_axis, dim3(grid), dim3(kBlock), 0, s, tmp, dist, nb, 0);
  hipLaunchKernelGGL(k_dist_axis, dim3(grid), dim3(kBlock), 0, s, dist, tmp, nb, 1);
  hipLaunchKernelGGL(k_dist_axis, dim3(grid), dim3(kBlock), 0, s, tmp, dist, nb, 2);
  return hipGetLastError();
}

hipError_t launch_readback(int fmt, const DevCache &c, float *sigma, float *u, hipStream_t s) {
  switch (fmt) {
    case 0: return launch_readback_f<0>(c, sigma, u, s);
    case 1: return launch_readback_f<1>(c, sigma, u, s);
    case 2: return launch_readback_f<2>(c, sigma, u, s);
    default: return launch_readback_f<3>(c, sigma, u, s);
  }
}

hipError_t launch_lookup(int fmt, bool lin, const DevCache &c, int n, const float *pts,
                         const float *dirs, float *su, float *bo, hipStream_t s) {
  switch (fmt) {
    case 0: return launch_lookup_f<0>(c, lin, n, pts, dirs, su, bo, s);
    case 1: return launch_lookup_f<1>(c, lin, n, pts, dirs, su, bo, s);
    case 2: return launch_lookup_f<2>(c, lin, n, pts, dirs, su, bo, s);
    default: return launch_lookup_f<3>(c, lin, n, pts, dirs, su, bo, s);
  }
}

}  // namespace fnr
