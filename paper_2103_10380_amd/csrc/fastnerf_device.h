// Device-side data layout and lookups of the gfx950 FastNeRF renderer.
//
// Position cache: one record per voxel, {sigma, u[D][3]} in the storage format,
// padded to a power-of-two stride (FP32 D=8: 100 B payload in 128 B, FP16 50 B
// in 64 B, FP8 25 B in 32 B) so that a record never straddles a 128-byte line.
// Records are stored brick-linear in 8^3 bricks (512 consecutive records per
// brick, x fastest inside), so the rays of an 8x8 pixel tile, which sample
// nearby voxels, touch few DRAM pages. Direction cache: FP32 [l][l][Dp] with
// rows padded with zeros to Dp = 4 ceil(D/4) floats, so a cell is whole 16-byte
// loads.
// Occupancy: one bit per brick of 2^oshift voxels, set when any voxel of the
// brick (widened by one voxel for trilinear lookups) has a stored sigma > 0.
// Distance field: one byte per distance brick (the occupancy brick, or 8^3
// voxels when the occupancy brick is smaller), the Chebyshev distance in such
// bricks to the nearest one holding an occupied brick (0 = it holds one,
// capped at kDistCap).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fnr {

constexpr int kWave = 64;
constexpr int kBlock = 256;
// Occupancy words the LDS-staged tile kernel can hold: 128 KiB of the CU's
// 160 KiB, a bitgrid of up to 1,048,576 bricks (k = 768 at 8^3 bricks needs
// 27,648 words).
constexpr int kOccLdsWords = 32768;
constexpr int kMaxD = 16;
constexpr int kMaxCh = 1 + 3 * kMaxD;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The nearest voxel of grid coordinate g is floor(g + kTie): a point on a
// voxel face takes the upper cell also when FP32 rounding puts it slightly
// below the face. With a sample spacing commensurate with the grid (k = 768,
// N = 192 across the box face to face) every sample lies on a face, and the
// FP32 grid coordinates of such samples are within 1.3e-4 voxel of the exact
// ones; kTie = 2^-11 (4.9e-4) clears that, and a point that it moves to the
// upper cell lies within 6.2e-4 voxel of the face, where either cell is an
// admissible nearest voxel under FP32 position error.
constexpr float kTie = 1.0f / 2048.0f;

// Largest stored brick distance (one byte per brick).
constexpr int kDistCap = 63;

// Template component count of the kernels that render a cache with D
// components; records are laid out for it.
__host__ __device__ constexpr int maxd_class(int D) { return D <= 4 ? 4 : (D <= 8 ? 8 : 16); }

struct DevCache {
  const uint8_t *rec;
  const float *beta;
  const uint32_t *occ;   // occupancy bits (one all-ones word without a bitgrid)
  int occ_words;         // 32-bit words of occ
  const uint8_t *dist;   // per-brick distance to the nearest occupied brick (one 0 without)
  const float *scales;   // kMaxCh per-channel scales (FP8; ones past 1 + 3D and otherwise)
  const int32_t *slot;   // brick-sparse: record brick of each 8^3 brick (0: all zero); else null
  const uint32_t *rank;  // brick-sparse: set bitgrid bits before each word
  int k, D, l;
  int bq;                // 16-byte chunks per direction cell (rows of 4 ceil(D/4) floats)
  int nbl;               // layout bricks per axis
  int nbo;               // occupancy bricks per axis (1 without a bitgrid)
  int oshift;            // log2 occupancy brick edge (30 without a bitgrid)
  int nbd;               // distance-field bricks per axis (1 without a bitgrid)
  int dshift;            // log2 distance-field brick edge (30 without a bitgrid)
  int rec_shift;         // log2 record stride in bytes
  int nchunk;            // 16-byte chunks per record: RecWords<fmt, maxd_class(D)>::nchunk
  float kf;              // k as float
  float bmin[3], bmax[3], inv_h[3];
  float th_scale, ph_scale;  // l/pi, l/(2 pi)
  float bg[3];
  int in_box, dir_linear;
  int fmt;               // storage format of the records (0 FP32, 1 FP16, 2 BF16, 3 E4M3)
};

struct DevView {
  double M[9];       // R K^-1: pixel (x+1/2, y+1/2, 1) -> world direction
  double o[3];       // camera centre
  float near_, far_;
  int H, W, tile_begin;
  // pixel rectangle [cx0, cx1) x [cy0, cy1) covered by the view's tiles (edges
  // multiples of 8 or the image's edge): the pixels outside it cannot see the
  // box, and the kernel writes them with the background
  int cx0, cy0, cx1, cy1;
  int tile_offset;   // first tile of the view covered (serving steps cover tile ranges)
  int scene;         // index into RenderArgs::caches (serving)
  int N;             // samples per ray
  float lim;         // ln(1/eps), +inf for eps = 0
  float *out;        // float[H][W][4]
};

struct RenderArgs {
  DevCache c;
  DevView v0;               // used when views == nullptr
  const DevView *views;     // batched launch: nviews views, tile_begin ascending
  int nviews;
  int total_tiles;
  unsigned *counter;        // tile-queue counters (kQueueCounters uints), self-resetting
  unsigned nwaves;
  const DevCache *caches;   // serving: per-scene caches (device), views[i].scene indexes it
  const int *dyn_total;     // serving: {tile count, view count} of the step (device)
  int vox;                  // 1: voxel traversal (every view has N = 0)
  long long fill_px;        // pixels outside the views' render rectangles (host: grid size)
  int interleave;           // > 0: views of equal tile counts interleaved in groups of this many
  int sched;                // kSchedTiles, kSchedRefill or kSchedWide
};

// Schedules of a fixed-N render launch: one 8x8 tile per wave (tiles), the
// wave-level ray queue (refill), tiles with more records in flight per lane
// (wide, for launches with few tiles).
constexpr int kSchedTiles = 0, kSchedRefill = 1, kSchedWide = 2, kSchedSplit = 3;

// ------------------------------------------------------------------ storage formats

template <int FMT> struct Fmt;

template <> struct Fmt<0> {  // FP32
  static constexpr int bytes = 4;
  __device__ static inline float get(const uint32_t *w, int j) { return __uint_as_float(w[j]); }
};

template <> struct Fmt<1> {  // FP16
  static constexpr int bytes = 2;
  __device__ static inline float get(const uint32_t *w, int j) {
    uint32_t h = (w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu;
    return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
  }
};

template <> struct Fmt<2> {  // BF16
  static constexpr int bytes = 2;
  __device__ static inline float get(const uint32_t *w, int j) {
    uint32_t h = (w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu;
    return __uint_as_float(h << 16);
  }
};

template <> struct Fmt<3> {  // OCP E4M3 code; the caller multiplies by the channel scale
  static constexpr int bytes = 1;
  // gfx950 converts OCP E4M3 pairs to FP32 in hardware (exact: every E4M3
  // value is an FP32 value). The NaN code is never stored (saturation).
  __device__ static inline float get(const uint32_t *w, int j) {
    const int word = (int)w[j >> 2];
    const auto v = (j & 2) ? __builtin_amdgcn_cvt_pk_f32_fp8(word, true)
                           : __builtin_amdgcn_cvt_pk_f32_fp8(word, false);
    return (j & 1) ? v[1] : v[0];
  }
};

template <int FMT, int MAXD> struct RecWords {
  static constexpr int nvals = 1 + 3 * MAXD;
  static constexpr int bytes = nvals * Fmt<FMT>::bytes;
  static constexpr int nchunk = (bytes + 15) / 16;
  static constexpr int nwords = nchunk * 4;
};

// ------------------------------------------------------------------ addressing

// Brick-grid index (bz * n + by) * n + bx with 24-bit multiplies (every
// operand is below 2^12, the products below 2^24): one full-rate v_mad_u32_u24
// per multiply-add instead of a 64-bit multiply.
__device__ __forceinline__ uint32_t grid3(uint32_t bx, uint32_t by, uint32_t bz, uint32_t n) {
  return __umul24(__umul24(bz, n) + by, n) + bx;
}

// Nearest voxel coordinate along one axis of grid coordinate g (the cell
// holding it, upper on a face, with FP32 rounding covered by kTie), clamped to
// the grid: the same value as min(max((int)(g + kTie), 0), k - 1) with a
// clamp before the conversion (the conversion truncates towards zero).
__device__ __forceinline__ int voxel_of(float g, float kmax) {
  return (int)__builtin_amdgcn_fmed3f(g + kTie, 0.0f, kmax);
}

__device__ inline uint64_t record_offset(const DevCache &c, int x, int y, int z) {
  uint32_t lb = grid3((uint32_t)(x >> 3), (uint32_t)(y >> 3), (uint32_t)(z >> 3),
                      (uint32_t)c.nbl);
  if (c.slot) lb = (uint32_t)c.slot[lb];  // brick-sparse: stored brick (0 reads as zero)
  uint32_t li = ((uint32_t)(z & 7) << 6) | ((uint32_t)(y & 7) << 3) | (uint32_t)(x & 7);
  return (((uint64_t)lb << 9) | li) << c.rec_shift;
}

// Record offset of voxel (x, y, z) in stored brick sb (brick-sparse caches).
__device__ inline uint64_t record_offset_in(const DevCache &c, uint32_t sb, int x, int y, int z) {
  const uint32_t li = ((uint32_t)(z & 7) << 6) | ((uint32_t)(y & 7) << 3) | (uint32_t)(x & 7);
  return (((uint64_t)sb << 9) | li) << c.rec_shift;
}

// Records of a cache rendered with MAXD hold RecWords<FMT, MAXD>::nchunk
// chunks (zero past the payload), so the loads are unconditional. They are
// ordinary (L1-allocating) loads: the chunks of one record share a cache line,
// and with non-temporal loads every 16-byte chunk went to L2 on its own, which
// halved the speed of the render.

template <int FMT, int MAXD>
__device__ inline void load_record(const DevCache &c, uint64_t off, uint32_t *w) {
  using RW = RecWords<FMT, MAXD>;
  const u32x4 *p = reinterpret_cast<const u32x4 *>(c.rec + off);
#pragma unroll
  for (int q = 0; q < RW::nchunk; ++q) {
    const u32x4 v = p[q];
    w[4 * q + 0] = v.x;
    w[4 * q + 1] = v.y;
    w[4 * q + 2] = v.z;
    w[4 * q + 3] = v.w;
  }
}

// Per-ray colour weights: beta[d] for FP32/FP16/BF16 records; for E4M3
// records the channel scales are folded in once per ray,
// w[3d + ch] = beta[d] * scale[1 + 3d + ch], so a sample costs no scale
// multiplies.
template <int FMT, int MAXD> struct ColourWeights {
  static constexpr int n = FMT == 3 ? 3 * MAXD : MAXD;
};

// sigma of a loaded record; s0 is the sigma channel's scale (E4M3 only)
template <int FMT>
__device__ inline float rec_sigma(const uint32_t *w, float s0) {
  float s = Fmt<FMT>::get(w, 0);
  if (FMT == 3) s *= s0;
  return s;
}

// colour beta . (u, v, w) of a loaded record (Eq. 5) with the per-ray weights
// above; weights are 0 for d >= D
template <int FMT, int MAXD>
__device__ inline void rec_colour(const uint32_t *w, const float *cw, float &r, float &g,
                                  float &b) {
  float cr = 0.f, cg = 0.f, cb = 0.f;
  if constexpr (FMT == 3) {
    // decode the record's codes two at a time
    constexpr int NV = 1 + 3 * MAXD;
    float v[(NV + 3) / 4 * 4];
#pragma unroll
    for (int q = 0; q < (NV + 3) / 4; ++q) {
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[q], false);
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[q], true);
      v[4 * q + 0] = lo[0];
      v[4 * q + 1] = lo[1];
      v[4 * q + 2] = hi[0];
      v[4 * q + 3] = hi[1];
    }
#pragma unroll
    for (int d = 0; d < MAXD; ++d) {
      cr = fmaf(cw[3 * d + 0], v[1 + 3 * d + 0], cr);
      cg = fmaf(cw[3 * d + 1], v[1 + 3 * d + 1], cg);
      cb = fmaf(cw[3 * d + 2], v[1 + 3 * d + 2], cb);
    }
    r = cr;
    g = cg;
    b = cb;
    return;
  }
#pragma unroll
  for (int d = 0; d < MAXD; ++d) {
    const float ur = Fmt<FMT>::get(w, 1 + 3 * d + 0);
    const float ug = Fmt<FMT>::get(w, 1 + 3 * d + 1);
    const float ub = Fmt<FMT>::get(w, 1 + 3 * d + 2);
    cr = fmaf(cw[d], ur, cr);
    cg = fmaf(cw[d], ug, cg);
    cb = fmaf(cw[d], ub, cb);
  }
  r = cr;
  g = cg;
  b = cb;
}

// ------------------------------------------------------------------ compositing

// e^{-x} through the hardware base-2 exponential (v_exp_f32): relative error
// a few ulp for the optical depths of a ray (x up to ln(1/eps) plus one
// sample), where the library expf spends a dozen instructions on range
// reduction.
__device__ __forceinline__ float exp_neg(float x) {
  return __builtin_amdgcn_exp2f(x * -1.44269504088896341f);
}

// 1 - e^{-x} for x >= 0 (a sample's opacity): below 1/16 a Taylor polynomial
// (relative error under 2^-40, no cancellation), above it 1 - exp_neg(x)
// (relative error about 1e-6 there).
__device__ __forceinline__ float opacity(float x) {
  const float p = x * (1.0f - x * (0.5f - x * (1.0f / 6.0f - x * (1.0f / 24.0f -
                  x * (1.0f / 120.0f - x * (1.0f / 720.0f))))));
  return x < 0.0625f ? p : 1.0f - exp_neg(x);
}

// ------------------------------------------------------------------ direction cache

__device__ inline void dir_cell_weights(const DevCache &c, float dx, float dy, float dz,
                                        int cell[4], float wt[4]) {
  float zc = fminf(fmaxf(dz, -1.0f), 1.0f);
  float th = acosf(zc);
  float ph = atan2f(dy, dx);
  if (ph < 0.0f) ph += 6.28318530717958647692f;
  const int l = c.l;
  if (!c.dir_linear) {
    int j = min((int)(th * c.th_scale), l - 1);
    int m = (int)(ph * c.ph_scale);
    if (m >= l) m -= l;
    cell[0] = cell[1] = cell[2] = cell[3] = j * l + m;
    wt[0] = 1.0f;
    wt[1] = wt[2] = wt[3] = 0.0f;
    return;
  }
  float gt = fmaf(th, c.th_scale, -0.5f), gp = fmaf(ph, c.ph_scale, -0.5f);
  float ft = floorf(gt), fp = floorf(gp);
  float a = gt - ft, b = gp - fp;
  int j0 = (int)ft, m0 = (int)fp;
  int ja = min(max(j0, 0), l - 1), jb = min(max(j0 + 1, 0), l - 1);
  int ma = m0 < 0 ? m0 + l : (m0 >= l ? m0 - l : m0);
  int mb = m0 + 1 >= l ? m0 + 1 - l : (m0 + 1 < 0 ? m0 + 1 + l : m0 + 1);
  cell[0] = ja * l + ma;
  cell[1] = ja * l + mb;
  cell[2] = jb * l + ma;
  cell[3] = jb * l + mb;
  wt[0] = (1.0f - a) * (1.0f - b);
  wt[1] = (1.0f - a) * b;
  wt[2] = a * (1.0f - b);
  wt[3] = a * b;
}

template <int MAXD>
__device__ inline void dir_lookup(const DevCache &c, float dx, float dy, float dz,
                                  float *beta) {
  constexpr int NQ = MAXD / 4;
  int cell[4];
  float wt[4];
  dir_cell_weights(c, dx, dy, dz, cell, wt);
  // all loads first (independent), then the blend
  float4 v[4][NQ];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 *bp = reinterpret_cast<const float4 *>(c.beta) + (size_t)cell[q] * c.bq;
#pragma unroll
    for (int j = 0; j < NQ; ++j) v[q][j] = j < c.bq ? bp[j] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc.x = fmaf(wt[q], v[q][j].x, acc.x);
      acc.y = fmaf(wt[q], v[q][j].y, acc.y);
      acc.z = fmaf(wt[q], v[q][j].z, acc.z);
      acc.w = fmaf(wt[q], v[q][j].w, acc.w);
    }
    beta[4 * j + 0] = acc.x;
    beta[4 * j + 1] = acc.y;
    beta[4 * j + 2] = acc.z;
    beta[4 * j + 3] = acc.w;
  }
}

}  // namespace fnr
